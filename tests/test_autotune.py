"""Host logic of the autotuner: the search policy against known cost
functions, the bounds it proposes, and the ratio rule it starts from."""
import json

import pytest

from paper_2206_07244_amd import autotune as at

SYM_T = [128, 1024, 2048, 4096, 8192, 16384, 20448, 40896]
NUM_T = [39, 425, 848, 1700, 3408, 6816, 13632]


def test_derived_bounds_follow_the_library_rule():
    import paper_2206_07244_amd as ops
    for step, t in ((0, SYM_T), (1, NUM_T)):
        for r in (1.0, 1.2, 1.5, 2.0, 3.0):
            assert at.derived_bounds(step, t, r) == ops.bin_bounds(step, t[:7], r)[:7]


def test_search_finds_paper_optimum_of_grid_cost():
    """A cost minimal at Sym 1.2 / Num 2 (the paper's choice) and flat in the
    bounds: the search returns that pair and leaves the bounds derived."""
    def cost(c):
        return (c["sym_ratio"] - 1.2) ** 2 + (c["num_ratio"] - 2.0) ** 2 + 1.0
    best, v = at.search(cost, SYM_T, NUM_T)
    assert best["sym_ratio"] == 1.2 and best["num_ratio"] == 2.0 and v == 1.0


def test_search_refines_between_grid_points():
    def cost(c):
        return abs(c["sym_ratio"] - 1.3) + abs(c["num_ratio"] - 2.25)
    best, v = at.search(cost, SYM_T, NUM_T, coordinate=False, abort=False)
    assert best["sym_ratio"] == pytest.approx(1.3) and best["num_ratio"] == pytest.approx(2.25)
    assert v == pytest.approx(0.0, abs=1e-12)


def test_coordinate_search_moves_single_bounds_within_capacity():
    """Cost rewards a larger numeric bin-1 bound and a smaller symbolic bin-3
    bound: the search moves exactly those, never past a table's size."""
    trace = []

    def cost(c):
        v = 10.0 + (c["sym_ratio"] - 1.2) ** 2 + (c["num_ratio"] - 2.0) ** 2
        if c["num_bounds"][1]:
            v -= c["num_bounds"][1] / 1000.0
        if c["sym_bounds"][3]:
            v += c["sym_bounds"][3] / 10000.0
        return v
    best, v = at.search(cost, SYM_T, NUM_T, trace=trace)
    derived_n = at.derived_bounds(1, NUM_T, best["num_ratio"])
    derived_s = at.derived_bounds(0, SYM_T, best["sym_ratio"])
    assert best["num_bounds"][1] > derived_n[1]
    assert best["sym_bounds"][3] < derived_s[3]
    for c, _ in trace:
        for j in range(7):
            assert -1 <= c["num_bounds"][j] <= NUM_T[j]
            assert -1 <= c["sym_bounds"][j] <= SYM_T[j]
        assert c["sym_ratio"] >= 1.0 and c["num_ratio"] >= 1.0
    # every candidate evaluated once
    keys = [at.Candidate(c).key() for c, _ in trace]
    assert len(keys) == len(set(keys))


def test_abort_fraction_search():
    best, _ = at.search(lambda c: abs(c["sym_abort_fraction"] - 0.7), SYM_T, NUM_T,
                        refine=False, coordinate=False)
    assert best["sym_abort_fraction"] == 0.7


def test_load_config_roundtrip(tmp_path):
    c = at.base_candidate(1.5, 3.0)
    c["num_bounds"] = [10, 200, 0, 0, 0, 0, -1]
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"classes": {"rmat": {"config": dict(c), "ms": 1.0}}}))
    cfg = at.load_config("rmat", str(p))
    from paper_2206_07244_amd import CONFIG_VERSION
    assert cfg.version == CONFIG_VERSION and cfg.sym_ratio == 1.5 and cfg.num_ratio == 3.0
    assert list(cfg.num_bounds) == [10, 200, 0, 0, 0, 0, -1]
    assert at.load_config("stencil", str(p)) is None
    assert at.load_config("rmat", str(tmp_path / "missing.json")) is None


def test_group_lanes_and_streams_search():
    """After the bounds, the search tries bin 0 with 4 and 16 lanes per row
    (its explicit bound re-derived: the table size changes with the lanes)
    and several streams, and keeps what is cheaper."""
    def cost(c):
        v = 10.0
        if c.get("group_lanes", 0) == 16:
            v -= 2.0
            assert c["sym_bounds"][0] == 0 and c["num_bounds"][0] == 0
        if c.get("streams", 0) == 2:
            v -= 1.0
        return v
    best, v = at.search(cost, [128, 1024, 2048, 4096, 8192, 16384, 20448, 40896],
                        [39, 425, 848, 1700, 3408, 6816, 13632], refine=False, coordinate=False)
    assert best["group_lanes"] == 16 and best["streams"] == 2 and v == 7.0

