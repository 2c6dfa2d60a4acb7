"""CPU-side checks of the C ABI library: it loads without a GPU, exports every
function that include/opsp.h declares, and its host-only helpers agree with
the oracle's reading of the paper's binning-range rule."""
import ctypes
import subprocess

import numpy as np
import pytest

import paper_2206_07244_amd as ops


def test_library_loads_and_exports_header_symbols():
    L = ops.lib()
    names = ops.exported_symbols()
    assert "opsp_spgemm" in names and "opsp_spgemm_symbolic" in names
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", ops.library_path()],
                         capture_output=True, text=True, check=True).stdout
    dyn = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in dyn]
    assert not missing, missing


def test_version_and_status_strings():
    L = ops.lib()
    assert b"gfx950" in L.opsp_version()
    for code in range(9):
        assert L.opsp_status_string(code).startswith(b"OPSP_")
    assert b"unknown" in L.opsp_status_string(99)


def test_table_sizes_fit_lds_budget():
    sym = ops.table_sizes(0)
    num = ops.table_sizes(1)
    assert len(sym) == ops.SYM_BINS and sym[-1] == -1
    assert len(num) == ops.NUM_BINS and num[-1] == -1
    # strictly growing LDS tables; last LDS bins use (almost) all 160 KB
    assert all(a < b for a, b in zip(sym[:-1], sym[1:-1]))
    assert all(a < b for a, b in zip(num[:-1], num[1:-1]))
    assert sym[7] * 4 <= 163840 and num[6] * 12 <= 163840
    assert sym[7] * 4 > 160000 and num[6] * 12 > 160000


@pytest.mark.parametrize("ratio", ["1", "1.2", "1.5", "2", "3"])
def test_bin_bounds_match_oracle_rule(oracle_lib, ratio):
    for step in (0, 1):
        sizes = ops.table_sizes(step)[:-1]
        got = ops.bin_bounds(step, sizes, float(ratio))
        want = oracle_lib.bin_ranges(sizes, ratio, numeric=(step == 1))
        assert got == want, (step, ratio)
    # and on the paper's V100 table sizes
    for step, sizes in ((0, [32, 512, 1024, 2048, 4096, 8192, 12287]),
                        (1, [31, 255, 511, 1023, 2047, 4095, 8191])):
        got = ops.bin_bounds(step, sizes, float(ratio))
        assert got == oracle_lib.bin_ranges(sizes, ratio, numeric=(step == 1))


def test_invalid_arguments_rejected_on_host():
    L = ops.lib()
    out = (ctypes.c_int64 * 4)()
    assert L.opsp_table_sizes(7, out, 4) == 1
    assert L.opsp_table_sizes(0, out, 4) == 1
    ts = (ctypes.c_int64 * 2)(10, 20)
    assert L.opsp_bin_bounds(0, ts, 3, 0.5, out) == 1
    # shape mismatch is caught before any device work
    A = ops.opsp_csr(rows=3, cols=4, nnz=0, rpt=1, col=None, val=None)
    B = ops.opsp_csr(rows=5, cols=2, nnz=0, rpt=1, col=None, val=None)
    C = ops.opsp_csr()
    assert L.opsp_spgemm(ctypes.byref(A), ctypes.byref(B), ctypes.byref(C), None) == 2
    assert L.opsp_spgemm(None, ctypes.byref(B), ctypes.byref(C), None) == 1
    assert L.opsp_spgemm(ctypes.byref(A), ctypes.byref(B), None, None) == 1


def test_predictor_arguments_rejected_on_host():
    """The one-phase entry point checks its predictor before any device work
    (the fake device pointers below are never dereferenced)."""
    L = ops.lib()
    A = ops.opsp_csr(rows=3, cols=4, nnz=0, rpt=1, col=None, val=None)
    B = ops.opsp_csr(rows=4, cols=2, nnz=0, rpt=1, col=None, val=None)
    C = ops.opsp_csr()

    def call(**kw):
        p = ops.opsp_predictor(version=ops.PREDICTOR_VERSION, kind=ops.PRED_UPPER)
        for k, v in kw.items():
            setattr(p, k, v)
        return L.opsp_spgemm_learned(ctypes.byref(A), ctypes.byref(B), ctypes.byref(C),
                                     ctypes.byref(p), None, None, None)

    assert call(version=0) == 1
    assert call(kind=7) == 1
    assert call(kind=ops.PRED_MLP) == 1               # no parameters
    assert call(margin=-0.5) == 1
    assert call(margin=float("nan")) == 1
    assert call(kind=ops.PRED_RATIO, ratio=0.0) == 1
    assert call(cap_scale=-1.0) == 1
    assert L.opsp_spgemm_learned(ctypes.byref(A), ctypes.byref(B), ctypes.byref(C), None, None,
                                 None, None) == 1
    Bbad = ops.opsp_csr(rows=5, cols=2, nnz=0, rpt=1, col=None, val=None)
    p = ops.opsp_predictor(version=ops.PREDICTOR_VERSION, kind=ops.PRED_UPPER)
    assert L.opsp_spgemm_learned(ctypes.byref(A), ctypes.byref(Bbad), ctypes.byref(C),
                                 ctypes.byref(p), None, None, None) == 2
    # training entry points
    assert L.opsp_mlp_grad(1, 1, 1, 0, 0.0, 1, None, None) == 1
    assert L.opsp_mlp_grad(1, 1, 1, 5, 1.0, 1, None, None) == 1
    assert L.opsp_mlp_forward(None, 1, 5, 1, None) == 1
    assert L.opsp_mlp_adam(1, 1, 1, 1, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None) == 1
    assert L.opsp_mlp_adam(1, 1, 1, 1, 1, 1e-3, 1.0, 0.999, 1e-8, 1, None) == 1


def test_stats_struct_matches_header():
    """ctypes mirrors have the sizes the header implies."""
    assert ctypes.sizeof(ops.Stats) == 8 * (4 + ops.SYM_BINS + ops.NUM_BINS) + 4 * 8 + 8 * 5 + 8
    assert ctypes.sizeof(ops.opsp_predictor) == 4 + 4 + 8 + 8 * 3 + 8 + 8 + 4 + 4


def test_config_fields_checked_on_host():
    """Configuration errors are caught before any device work (the fake
    device pointers are never dereferenced): stream count, lanes per row of
    bin 0, explicit bounds beyond the table of the chosen variant, and the
    ctypes mirror's layout (version-3 fields at the end)."""
    L = ops.lib()
    A = ops.opsp_csr(rows=3, cols=4, nnz=0, rpt=1, col=None, val=None)
    B = ops.opsp_csr(rows=4, cols=2, nnz=0, rpt=1, col=None, val=None)
    C = ops.opsp_csr()

    def call(**kw):
        c = ops.Config(**kw)
        return L.opsp_spgemm_ex(ctypes.byref(A), ctypes.byref(B), ctypes.byref(C), ctypes.byref(c),
                                None, None)

    assert call(streams=5) == 1
    assert call(streams=-1) == 1
    assert call(group_lanes=5) == 1
    assert call(group_lanes=32) == 1
    # bin 0's table: 128 keys / 39 entries by default, 64 / 19 with 4 lanes
    assert call(group_lanes=4, sym_bounds=[65, 0, 0, 0, 0, 0, 0]) == 1
    assert call(group_lanes=4, num_bounds=[20, 0, 0, 0, 0, 0, 0]) == 1
    assert call(version=4) == 1
    fields = [f for f, _ in ops.Config._fields_]
    assert fields[-2:] == ["streams", "group_lanes"]
    assert ops.Config.group_lanes.offset == ops.Config.streams.offset + 4
