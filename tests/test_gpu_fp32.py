"""FP32 values (opsp_spgemm_f32) against the FP64 oracle.

The inputs are rounded to float32 first; the oracle multiplies those values
exactly representable in FP64.  The GPU rounds every product a_ik b_kj to
float32, sums the terms of an entry in FP64 in any order and rounds the sum
to float32, so with u = 2^-24 each entry obeys |c - c_ref| <= (k_ij + 1) u
S_ij, where k_ij is its number of terms and S_ij = sum |a_ik b_kj| (the
bound for a float32 sum of k rounded terms, which the FP64 sum only
tightens; c_ref is exact to 1e-16 S).  k_ij <= a_len_i, the length of
row i of A, which the tests use.  Rows and columns must be identical to the
oracle's; integer inputs below 2^24 in magnitude are exact in float32 and
must match bit for bit.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _ops():
    import paper_2206_07244_amd as ops
    return ops


def _f32(A):
    return syn.CSR(A.rows, A.cols, A.rpt, A.col, A.val.astype(np.float32).astype(np.float64))


def check32(A, B=None, cfg=None, exact=False, stats=None):
    import torch
    ops = _ops()
    A = _f32(A)
    B = A if B is None else _f32(B)
    dA = ops.DeviceCSR.from_host(A, dtype=np.float32)
    dB = dA if B is A else ops.DeviceCSR.from_host(B, dtype=np.float32)
    C = ops.spgemm_f32(dA, dB, config=cfg if cfg is not None else ops.Config(validate=1), stats=stats)
    torch.cuda.synchronize()
    assert C.val.dtype == torch.float32
    rpt, col, val = C.to_host()
    rrpt, rcol, rval, rabs = oracle.spgemm(A, B)
    assert np.array_equal(rpt - rpt[0], rrpt - rrpt[0]), "rpt"
    assert np.array_equal(col, rcol), "col"
    v = val.astype(np.float64)
    if exact:
        assert np.array_equal(v, rval)
        return 0.0
    alen = np.diff(A.rpt)
    k = np.repeat(alen, np.diff(rrpt)).astype(np.float64)
    err = np.abs(v - rval)
    bound = (k + 1.0) * U32 * rabs
    bad = err > bound
    assert not bad.any(), f"{int(bad.sum())} entries beyond (k+1) u S"
    return float(np.max(err[rabs > 0] / rabs[rabs > 0])) if (rabs > 0).any() else 0.0


def test_fp32_lap5_exact():
    """Integer values: every product and partial sum is exact in float32."""
    st = _ops().Stats()
    check32(syn.lap5(64), exact=True, stats=st)
    assert st.nprod == 100104 and st.nnz == 51972


@pytest.mark.parametrize("g", [2, 9, 20])
def test_fp32_stencils(g):
    check32(syn.stencil27(g, seed=g))
    check32(syn.block_stencil27(max(2, g // 3), 3, seed=g))


@pytest.mark.parametrize("scale", [10, 14])
def test_fp32_rmat_all_bins(scale):
    st = _ops().Stats()
    check32(syn.rmat(scale, 16, seed=scale), stats=st)
    if scale == 14:
        assert all(x > 0 for x in st.num_bin_rows), list(st.num_bin_rows)


@pytest.mark.parametrize("b", list(range(8)))
def test_fp32_forced_numeric_bins(b):
    """Every numeric kernel in float32: each bin forced in turn (bin 7 by the
    bucketed dense kernel and, with every row hashed, by the global tables)."""
    ops = _ops()
    A = syn.rmat(12, 16, seed=b)
    check32(A, cfg=ops.Config(force_num_bin=b, force_sym_bin=min(b, 8)))
    if b == 7:
        check32(A, cfg=ops.Config(force_num_bin=7, hash_all_rows=1))


def test_fp32_rectangular_banded_and_variants():
    ops = _ops()
    A = syn.poisson_uniform(3000, 5000, 6.0, seed=1)
    B = syn.poisson_uniform(5000, 2000, 9.0, seed=2)
    check32(A, B)
    check32(syn.banded(20000, 64, 12, seed=3))
    for lanes in (4, 16):
        check32(A, B, cfg=ops.Config(group_lanes=lanes, force_num_bin=0, force_sym_bin=0))
    check32(syn.random_csr(200, 300, 0.05, seed=4, values="int"),
            syn.random_csr(300, 100, 0.05, seed=5, values="int"), exact=True)


def test_fp32_empty_and_degenerate():
    check32(syn.random_csr(40, 30, 0.0, seed=1), syn.random_csr(30, 20, 0.3, seed=2))
    check32(syn.random_csr(0, 10, 0.5, seed=3), syn.random_csr(10, 7, 0.5, seed=4))


@pytest.mark.parametrize("forced", [-1, 2])
def test_fp32_merged_runs(forced):
    """Runs of entries whose B rows share one column set are merged by the
    numeric step; each product is still rounded to float32 and the run's
    products summed in FP64, so the (k+1) u S bound holds."""
    import test_gpu_parity as tp
    A, B = tp._runs_of_rows(20000, seed=92)
    check32(A, B, cfg=_ops().Config(validate=1, force_num_bin=forced))
