"""Batched products (one block-diagonal product over many problems, run as
two captured graphs) against the CPU oracle, problem by problem."""
import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu


def _ops():
    import paper_2206_07244_amd as ops
    return ops


def _problems(seed):
    rng = np.random.default_rng(seed)
    probs = []
    probs.append((syn.lap5(16), None))
    probs.append((syn.stencil27(7, seed=3), None))
    probs.append((syn.rmat(12, 16, seed=seed), None))
    probs.append((syn.random_csr(0, 10, 0.5, seed=1), syn.random_csr(10, 7, 0.5, seed=2)))   # no rows
    probs.append((syn.random_csr(9, 0, 0.5, seed=3), syn.random_csr(0, 11, 0.5, seed=4)))    # K = 0
    probs.append((syn.random_csr(40, 30, 0.0, seed=5), syn.random_csr(30, 20, 0.3, seed=6)))  # empty A
    for i in range(14):
        m, k, n = (int(x) for x in rng.integers(1, 400, 3))
        A = syn.poisson_uniform(m, k, float(rng.uniform(0.5, 12)), seed=[seed, i, 0])
        B = syn.poisson_uniform(k, n, float(rng.uniform(0.5, 12)), seed=[seed, i, 1])
        probs.append((A, B))
    probs.append((syn.banded(3000, 40, 9, seed=seed), None))
    return [(A, A if B is None else B) for A, B in probs]


def _run(probs, stats=None, config=None):
    import torch
    ops = _ops()
    dev = [(ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)) for A, B in probs]
    batch = ops.Batch([a for a, _ in dev], [b for _, b in dev], config=config)
    views = batch.execute(stats=stats)
    torch.cuda.synchronize()
    return batch, dev, views


def test_batched_matches_oracle_per_problem():
    probs = _problems(7)
    st = _ops().Stats()
    batch, dev, views = _run(probs, st)
    assert st.nprod == sum(oracle.row_stats(A, B)[3] for A, B in probs)
    for (A, B), v in zip(probs, views):
        oracle.compare(*v.to_host(), oracle.spgemm(A, B))


def test_batched_replay_and_new_values():
    import torch
    probs = _problems(8)
    batch, dev, views = _run(probs)
    first = [v.to_host() for v in views]
    # replay both graphs: identical structure, same values within tolerance
    views2 = batch.execute()
    torch.cuda.synchronize()
    for f, v in zip(first, views2):
        g = v.to_host()
        assert np.array_equal(f[0], g[0]) and np.array_equal(f[1], g[1])
    # new values in place (structure unchanged) are picked up by the next run
    rng = np.random.default_rng(0)
    new_probs = []
    for (A, B), (dA, dB) in zip(probs, dev):
        va = rng.standard_normal(A.nnz)
        dA.val.copy_(torch.from_numpy(va).to(dA.val.device))
        A2 = syn.CSR(A.rows, A.cols, A.rpt, A.col, va)
        if B is A:   # uploaded twice: the B copy gets the same new values
            dB.val.copy_(dA.val)
            new_probs.append((A2, A2))
        else:
            new_probs.append((A2, B))
    views3 = batch.execute()
    torch.cuda.synchronize()
    for (A, B), v in zip(new_probs, views3):
        oracle.compare(*v.to_host(), oracle.spgemm(A, B))


def test_batched_all_numeric_bins():
    probs = [(syn.rmat(14, 16, seed=21), None), (syn.lap5(30), None), (syn.stencil27(6, seed=1), None)]
    probs = [(A, A) for A, _ in probs]
    st = _ops().Stats()
    batch, dev, views = _run(probs, st)
    assert all(x > 0 for x in st.num_bin_rows), list(st.num_bin_rows)
    for (A, B), v in zip(probs, views):
        oracle.compare(*v.to_host(), oracle.spgemm(A, B))


def test_batched_structure_equals_plain_path():
    import torch
    ops = _ops()
    probs = [(syn.poisson_uniform(2000, 2000, 8.0, seed=[5, i]), ) * 2 for i in range(6)]
    batch, dev, views = _run(probs)
    for (A, _), (dA, _), v in zip(probs, dev, views):
        C = ops.spgemm(dA, dA)
        torch.cuda.synchronize()
        r1, c1, _ = C.to_host()
        r2, c2, _ = v.to_host()
        assert np.array_equal(r1, r2) and np.array_equal(c1, c2)


@pytest.mark.parametrize("lanes", [4, 16])
def test_batched_group_lanes(lanes):
    """The bin-0 variants (lanes per row and table sizes chosen by the
    autotuner) inside the captured graphs."""
    probs = _problems(9)
    batch, dev, views = _run(probs, config=_ops().Config(group_lanes=lanes))
    for (A, B), v in zip(probs, views):
        oracle.compare(*v.to_host(), oracle.spgemm(A, B))

