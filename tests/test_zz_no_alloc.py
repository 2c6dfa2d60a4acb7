"""The numeric phase that allocates nothing (opsp_spgemm_numeric_noalloc)
against the allocating numeric phase (opsp_spgemm_numeric) on the same plan.

The long-row numeric bin is forced for every row, so that its kernels run in
the library's fixed scratch instead of allocated staging or global tables:
the bucketed kernel (rows with a known column range) and the global hash
tables (config.hash_all_rows).  Two calls in a row, the second on a smaller
product.  Row pointers and columns must be identical to the allocating
entry point's and to the oracle's; values within 1e-12 * S of the oracle
(S_ij = sum_k |a_ik b_kj|, the bound on any summation order).  The library's
allocation hook is armed during the call, so any allocation would fail it.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _ops():
    import paper_2206_07244_amd as ops
    return ops


def _cfg(hashed):
    ops = _ops()
    c = ops.Config(force_num_bin=7)
    if hashed:
        c.hash_all_rows = 1
    return c


def _buffers(rows, nnz):
    import torch
    ops = _ops()
    return ops.DeviceCSR(rows, 0, torch.full((rows + 1,), -7, dtype=torch.int64, device="cuda"),
                         torch.full((nnz,), -7, dtype=torch.int32, device="cuda"),
                         torch.full((nnz,), float("nan"), dtype=torch.float64, device="cuda"))


def _pair(A, hashed):
    """(no-allocation result, allocating result) of the numeric phase of A^2."""
    import torch
    ops = _ops()
    dA = ops.DeviceCSR.from_host(A)
    plan = ops.spgemm_symbolic(dA, dA, config=_cfg(hashed))
    ref = ops.spgemm_numeric(plan, dA, dA)
    out = _buffers(A.rows, plan.nnz)
    torch.cuda.synchronize()
    live = ops.cache_live_bytes()
    ops.debug_fail_alloc(0)          # the next library allocation would fail
    try:
        ops.spgemm_numeric_noalloc(plan, dA, dA, out)
    finally:
        ops.debug_fail_alloc(-1)
    torch.cuda.synchronize()
    assert ops.cache_live_bytes() == live
    return out.to_host(), ref.to_host()


@pytest.mark.parametrize("hashed", [False, True])
def test_noalloc_matches_allocating_numeric_twice(hashed):
    for A in (syn.rmat(12, 16, seed=5), syn.rmat(9, 8, seed=6)):
        got, exp = _pair(A, hashed)
        assert np.array_equal(got[0], exp[0]), "rpt differs from the allocating entry point"
        assert np.array_equal(got[1], exp[1]), "col differs from the allocating entry point"
        ref = oracle.spgemm(A, A)
        oracle.compare(*got, ref, tol=TOL)
        oracle.compare(*exp, ref, tol=TOL)


def test_noalloc_empty_product():
    import torch
    ops = _ops()
    A = syn.random_csr(40, 30, 0.0, seed=1)
    B = syn.random_csr(30, 20, 0.0, seed=2)
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    plan = ops.spgemm_symbolic(dA, dB, config=_cfg(False))
    assert plan.nnz == 0
    out = _buffers(A.rows, 0)
    ops.spgemm_numeric_noalloc(plan, dA, dB, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.rpt.cpu().numpy(), np.zeros(A.rows + 1, np.int64))


def test_noalloc_rejects_a_row_beyond_the_scratch():
    """One row of 2400 products per column over 2400 columns: 5.76e6
    products, whose staging (12 B each) exceeds the 64 MiB scratch."""
    import torch
    ops = _ops()
    n = 2400
    A = syn.CSR(1, n, np.array([0, n], np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    rpt = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    B = syn.CSR(n, n, rpt, col, np.ones(n * n))
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    plan = ops.spgemm_symbolic(dA, dB, config=_cfg(False))
    assert plan.nnz == n
    out = _buffers(1, n)
    with pytest.raises(ops.OpspError) as ei:
        ops.spgemm_numeric_noalloc(plan, dA, dB, out)
    assert ei.value.code == ops.ERR_SCRATCH
    # the allocating entry point still computes it
    C = ops.spgemm_numeric(plan, dA, dB)
    torch.cuda.synchronize()
    assert np.array_equal(C.col.cpu().numpy(), np.arange(n, dtype=np.int32))
    assert np.all(C.val.cpu().numpy() == float(n))
