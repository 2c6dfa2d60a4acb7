"""The boundary's error contract on the GPU.

* Validation mode (config.validate = 1) rejects non-canonical operands
  (Section 2.1.1: CSR with strictly ascending columns) with
  OPSP_ERR_INVALID before any kernel gathers through them: a row pointer
  that decreases or does not cover exactly nnz entries, a column index
  outside [0, cols), a row whose columns repeat or descend.  The bad
  operands are built so that nothing but the check reads them.
* Every allocation failure of a call (injected one at a time with the
  library's testing hook) returns OPSP_ERR_ALLOC, zeroes *C and leaves no
  block allocated: the library's live bytes return to what they were.
"""
import ctypes

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

INVALID, ALLOC = 1, 3


def _ops():
    import paper_2206_07244_amd as ops
    return ops


def _call(A, B, cfg):
    import torch
    ops = _ops()
    C = ops.opsp_csr()
    code = ops.lib().opsp_spgemm_ex(ctypes.byref(A._c()), ctypes.byref(B._c()), ctypes.byref(C),
                                    ctypes.byref(cfg), None,
                                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return code, C


def _broken(kind):
    """A 6x6 operand with one defect, and the number of entries its
    col/val buffers hold."""
    import torch
    ops = _ops()
    A = syn.random_csr(6, 6, 0.5, seed=3)
    rpt, col, val = A.rpt.copy(), A.col.copy(), A.val.copy()
    nnz = int(rpt[-1])
    rows_with_two = [i for i in range(6) if rpt[i + 1] - rpt[i] >= 2]
    r = rows_with_two[0]
    if kind == "rpt_decreasing":
        i = next(i for i in range(1, 6) if rpt[i + 1] > rpt[i])
        rpt[i] = rpt[i + 1] + 1
    elif kind == "rpt_past_nnz":
        rpt[-1] = nnz + 5          # the row pointer names entries beyond nnz
    elif kind == "col_high":
        col[rpt[r]] = 6
    elif kind == "col_negative":
        col[rpt[r]] = -1
    elif kind == "col_repeated":
        col[rpt[r] + 1] = col[rpt[r]]
    elif kind == "col_descending":
        col[rpt[r]], col[rpt[r] + 1] = col[rpt[r] + 1], col[rpt[r]]
    dev = torch.device("cuda")
    T = lambda a: torch.from_numpy(a).to(dev)
    # the col/val buffers hold nnz entries; the row pointer may claim more
    # only in the case the check must reject before reading col
    return ops.DeviceCSR(6, 6, T(rpt), T(col), T(val)), nnz


@pytest.mark.parametrize("kind", ["rpt_decreasing", "rpt_past_nnz", "col_high", "col_negative",
                                  "col_repeated", "col_descending"])
@pytest.mark.parametrize("side", ["A", "B"])
def test_validation_rejects_noncanonical(kind, side):
    ops = _ops()
    bad, nnz = _broken(kind)
    good = ops.DeviceCSR.from_host(syn.random_csr(6, 6, 0.5, seed=4))
    A, B = (bad, good) if side == "A" else (good, bad)
    cfg = ops.Config(validate=1)
    C = ops.opsp_csr()
    import torch
    Ac, Bc = A._c(), B._c()
    # the caller's entry count is what the buffers hold
    if side == "A":
        Ac.nnz = nnz
    else:
        Bc.nnz = nnz
    code = ops.lib().opsp_spgemm_ex(ctypes.byref(Ac), ctypes.byref(Bc), ctypes.byref(C),
                                    ctypes.byref(cfg), None, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert code == INVALID, (kind, side, code)
    assert not C.rpt and not C.col and not C.val and C.nnz == 0


def test_validation_accepts_canonical_and_views():
    import torch
    ops = _ops()
    A = syn.rmat(10, 8, seed=2)
    dA = ops.DeviceCSR.from_host(A)
    code, C = _call(dA, dA, ops.Config(validate=1))
    assert code == 0
    ops.free_raw(C, torch.cuda.current_stream().cuda_stream)
    # a row range is a valid operand (absolute offsets, rpt[0] > 0)
    v = ops.DeviceCSR(100, A.cols, dA.rpt[300:401], dA.col, dA.val)
    code, C = _call(v, dA, ops.Config(validate=1))
    assert code == 0
    ops.free_raw(C, torch.cuda.current_stream().cuda_stream)


def _sweep(run, label, max_allocs=64):
    """Fail the k-th allocation for k = 0, 1, ... until the call succeeds."""
    import torch
    ops = _ops()
    run()   # warm-up: the cache holds every block size the call needs
    torch.cuda.synchronize()
    base = ops.cache_live_bytes()
    failures = 0
    for k in range(max_allocs):
        ops.debug_fail_alloc(k)
        try:
            code, release = run()
        finally:
            ops.debug_fail_alloc(-1)
        torch.cuda.synchronize()
        if code == 0:
            release()
            torch.cuda.synchronize()
            assert ops.cache_live_bytes() == base, (label, k)
            break
        assert code == ALLOC, (label, k, code)
        assert ops.cache_live_bytes() == base, (label, k)
        failures += 1
    else:
        pytest.fail(f"{label}: still failing after {max_allocs} injected failures")
    assert failures >= 3, (label, failures)


def test_allocation_failures_leave_nothing_allocated():
    import torch
    ops = _ops()
    sh = torch.cuda.current_stream().cuda_stream
    L = ops.lib()
    A = syn.rmat(14, 16, seed=14)          # every numeric bin, global tables included
    dA = ops.DeviceCSR.from_host(A)
    Ac = dA._c()

    def plain():
        C = ops.opsp_csr()
        code = L.opsp_spgemm(ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(C), sh)
        if code != 0:
            assert not C.rpt and not C.col and not C.val
        return code, (lambda: ops.free_raw(C, sh))
    _sweep(plain, "opsp_spgemm")

    pred = ops.Predictor.load()
    ps = pred.struct()

    def learned():
        C = ops.opsp_csr()
        code = L.opsp_spgemm_learned(ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(C),
                                     ctypes.byref(ps), None, None, sh)
        if code != 0:
            assert not C.rpt and not C.col and not C.val
        return code, (lambda: ops.free_raw(C, sh))
    _sweep(learned, "opsp_spgemm_learned")

    def phases():
        plan = ctypes.c_void_p()
        nnz = ctypes.c_int64()
        code = L.opsp_spgemm_symbolic(ctypes.byref(Ac), ctypes.byref(Ac), None, ctypes.byref(plan),
                                      ctypes.byref(nnz), sh)
        if code != 0:
            assert not plan.value
            return code, None
        C = ops.opsp_csr()
        code = L.opsp_spgemm_numeric(plan, ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(C), sh)
        if code != 0:
            L.opsp_plan_destroy(plan)
            return code, None

        def rel():
            ops.free_raw(C, sh)
            L.opsp_plan_destroy(plan)
        return code, rel
    _sweep(phases, "symbolic + numeric")
