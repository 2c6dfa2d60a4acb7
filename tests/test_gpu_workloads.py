"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default config, one call of opsp_spgemm).

* 2-D 5-point Laplacian 64x64 squared: every entry, bit-exact.
* 3-D 27-point stencil 100^3 squared (120.6 M outputs): every entry against
  the oracle, plus the closed-form totals.
* R-MAT scale 20 squared (9.7e9 outputs, ~116 GB of C): sampled rows (the
  longest rows plus seeded random rows) against the oracle row by row, and
  row-pointer properties over all rows.
"""
import time

import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(*a):
    print(*a, flush=True)


def test_stencil27_100_full():
    import torch
    import paper_2206_07244_amd as ops
    g = 100
    t0 = time.time()
    A = syn.stencil27(g, seed=27)
    _say("st27_100 generated", A.nnz, round(time.time() - t0, 1))
    dA = ops.DeviceCSR.from_host(A)
    st = ops.Stats()
    C = ops.spgemm(dA, dA, stats=st)
    torch.cuda.synchronize()
    assert st.nprod == (9 * g - 10) ** 3 == 704969000
    assert st.nnz == (5 * g - 6) ** 3 == 120553784
    got = C.to_host()
    del C
    _say("gpu done", round(time.time() - t0, 1))
    ref = oracle.spgemm(A, A)
    _say("oracle done", round(time.time() - t0, 1))
    info = oracle.compare(*got, ref)
    _say("st27_100", info)
    assert info["max_err_over_S"] < 1e-14


def test_rmat20_sampled_rows():
    import torch
    import paper_2206_07244_amd as ops
    t0 = time.time()
    A = syn.rmat(20, 16, 0.57, 0.19, 0.19, seed=20)
    _say("rmat20 generated", A.nnz, round(time.time() - t0, 1))
    dA = ops.DeviceCSR.from_host(A)
    st = ops.Stats()
    C = ops.spgemm(dA, dA, stats=st)
    torch.cuda.synchronize()
    _say("gpu done", st.as_dict(), round(time.time() - t0, 1))
    nprod, alen, bmax, tot = oracle.row_stats(A, A)
    assert st.nprod == tot
    rpt = C.rpt.cpu().numpy()
    assert rpt[0] == 0 and rpt[-1] == st.nnz == C.nnz
    nnz = np.diff(rpt)
    assert np.all(nnz >= bmax) and np.all(nnz <= np.minimum(nprod, A.cols))
    assert np.all(nnz[alen <= 1] == nprod[alen <= 1])
    rng = np.random.default_rng(2020)
    rows = np.unique(np.concatenate([np.argsort(nprod)[-6:], rng.integers(0, A.rows, 120),
                                     [0, A.rows - 1]])).astype(np.int64)
    ref = oracle.spgemm(A, A, rows=rows)
    _say("oracle rows done", rows.size, round(time.time() - t0, 1))
    for r_i, r in enumerate(rows):
        a, b = int(rpt[r]), int(rpt[r + 1])
        c, d = int(ref[0][r_i]), int(ref[0][r_i + 1])
        assert b - a == d - c, r
        col = C.col[a:b].cpu().numpy()
        val = C.val[a:b].cpu().numpy()
        assert np.array_equal(col, ref[1][c:d]), r
        assert np.all(np.abs(val - ref[2][c:d]) <= 1e-12 * ref[3][c:d]), r
