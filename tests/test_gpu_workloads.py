"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the tuned bin configuration of the workload's class, one
call of the product).

* 2-D 5-point Laplacian 64x64 squared: every entry, bit-exact.
* 3-D 27-point stencil 100^3 squared (120.6 M outputs): every entry against
  the oracle, plus the closed-form totals.
* 27-point stencil 40^3 with 3x3 node blocks squared (compression ratio
  17.6): every entry, plus the closed-form totals.
* R-MAT scale 20 squared (9.7e9 outputs, ~116 GB of C): the whole row
  pointer against the oracle's symbolic counts, and every entry of at least
  32 rows of every symbolic and every numeric bin (plus the longest rows).
* Random banded n = 2^21 squared, plain two-pass and one-phase with the
  trained predictor: every entry.
* One row panel of R-MAT scale 21 (1/8 of the products, the hub rows),
  plain and one-phase: the panel's whole row pointer against the oracle's
  symbolic counts, every entry of at least 32 rows per bin.
* 512 independent uneven products as one batch: every problem, every entry.

The oracle runs row-parallel here (identical per-row code, identical bits).
"""
import time

import numpy as np
import pytest

import oracle
import synthetic as syn
from _fullsize import bins_of, compare_rows, per_bin_counts, stratified_rows

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

T0 = time.time()


def _say(*a):
    print(f"[{time.time() - T0:7.1f}s]", *a, flush=True)


def _threads():
    return oracle.host_threads()


def _tuned(cls):
    from paper_2206_07244_amd import autotune
    return autotune.load_config(cls)


def test_lap5_64_full_bit_exact():
    import torch
    import paper_2206_07244_amd as ops
    A = syn.lap5(64)
    dA = ops.DeviceCSR.from_host(A)
    st = ops.Stats()
    C = ops.spgemm(dA, dA, config=_tuned("stencil"), stats=st)
    torch.cuda.synchronize()
    assert st.nprod == 100104 and st.nnz == 51972
    info = oracle.compare(*C.to_host(), oracle.spgemm(A, A))
    assert info["bit_exact_values"], info


def test_stencil27_100_full():
    import torch
    import paper_2206_07244_amd as ops
    g = 100
    A = syn.stencil27(g, seed=27)
    _say("st27_100 generated", A.nnz)
    dA = ops.DeviceCSR.from_host(A)
    st = ops.Stats()
    C = ops.spgemm(dA, dA, config=_tuned("stencil"), stats=st)
    torch.cuda.synchronize()
    assert st.nprod == (9 * g - 10) ** 3 == 704969000
    assert st.nnz == (5 * g - 6) ** 3 == 120553784
    got = C.to_host()
    del C
    _say("gpu done")
    ref = oracle.spgemm(A, A, threads=_threads())
    _say("oracle done")
    info = oracle.compare(*got, ref)
    _say("st27_100", info)
    assert info["max_err_over_S"] < 1e-14


def test_block_stencil27_40_full():
    """27-point stencil 40^3 with 3x3 node blocks squared (compression ratio
    17.6, 65.7 M outputs), in the launch configuration of the benchmark:
    closed-form totals and every entry against the oracle."""
    import torch
    import paper_2206_07244_amd as ops
    g = 40
    A = syn.block_stencil27(g, 3, seed=40)
    dA = ops.DeviceCSR.from_host(A)
    st = ops.Stats()
    C = ops.spgemm(dA, dA, config=_tuned("stencil"), stats=st)
    torch.cuda.synchronize()
    assert st.nprod == 27 * (9 * g - 10) ** 3
    assert st.nnz == 9 * (5 * g - 6) ** 3
    got = C.to_host()
    del C
    ref = oracle.spgemm(A, A, threads=_threads())
    info = oracle.compare(*got, ref)
    _say("bst27_40", info)
    assert info["max_err_over_S"] < 1e-14


def test_stencil27_100_fp32_full():
    """The 27-point stencil 100^3 squared with FP32 values: structure exact,
    every value within (k + 1) 2^-24 S of the FP64 oracle on the rounded
    inputs (see test_gpu_fp32)."""
    import torch
    import paper_2206_07244_amd as ops
    g = 100
    A = syn.stencil27(g, seed=27)
    A = syn.CSR(A.rows, A.cols, A.rpt, A.col, A.val.astype(np.float32).astype(np.float64))
    dA = ops.DeviceCSR.from_host(A, dtype=np.float32)
    st = ops.Stats()
    C = ops.spgemm_f32(dA, dA, config=_tuned("stencil"), stats=st)
    torch.cuda.synchronize()
    assert st.nnz == (5 * g - 6) ** 3
    rpt, col, val = C.to_host()
    del C
    rrpt, rcol, rval, rabs = oracle.spgemm(A, A, threads=_threads())
    assert np.array_equal(rpt, rrpt) and np.array_equal(col, rcol)
    k = np.repeat(np.diff(A.rpt), np.diff(rrpt)).astype(np.float64)
    err = np.abs(val.astype(np.float64) - rval)
    assert np.all(err <= (k + 1.0) * 2.0 ** -24 * rabs)
    _say("st27_100 fp32 max |d|/S", float(np.max(err / np.maximum(rabs, 1e-300))))


def _full_rpt_and_bins(ops, A, rows_abs, C, cfg, tag, extra_rows=()):
    """Whole row pointer of C (rows `rows_abs` of A) against the oracle's
    symbolic counts, then >= 32 rows of every bin compared entry by entry."""
    th = _threads()
    rpt = C.rpt.cpu().numpy()
    assert rpt[0] == 0
    nnz_gpu = np.diff(rpt)
    nnz_ref = oracle.symbolic(A, A, rows=rows_abs, threads=th)
    _say(tag, "oracle symbolic counts done")
    np.testing.assert_array_equal(nnz_gpu, nnz_ref)
    nprod, _, _, _ = oracle.row_stats(A, A)
    nprod = nprod[rows_abs]
    sb, nb = bins_of(ops, cfg, nprod, nnz_ref)
    longest = np.argsort(nprod)[-4:]
    local = stratified_rows(sb, nb, 32, seed=2020, extra=[0, len(rows_abs) - 1, *longest, *extra_rows])
    s_cnt, n_cnt = per_bin_counts(local, sb, nb)
    _say(tag, "rows compared per symbolic bin", s_cnt, "per numeric bin", n_cnt)
    for counts, bins in ((s_cnt, sb), (n_cnt, nb)):
        for b, c in counts.items():
            assert c >= min(32, int(np.sum(bins == b))), (b, c)
    sre = compare_rows(C, rpt, local, A, A, th, ref_rows=rows_abs[local])
    _say(tag, "rows compared:", local.size, "max |d|/S", sre)
    return sb, nb


def test_rmat20_row_pointer_and_bins():
    import torch
    import paper_2206_07244_amd as ops
    A = syn.rmat(20, 16, 0.57, 0.19, 0.19, seed=20)
    _say("rmat20 generated", A.nnz)
    dA = ops.DeviceCSR.from_host(A)
    cfg = _tuned("rmat")
    st = ops.Stats()
    C = ops.spgemm(dA, dA, config=cfg, stats=st)
    torch.cuda.synchronize()
    _say("gpu done", st.as_dict())
    _, _, _, tot = oracle.row_stats(A, A)
    assert st.nprod == tot
    assert C.nnz == st.nnz
    _full_rpt_and_bins(ops, A, np.arange(A.rows), C, cfg, "rmat20")


def test_band21_plain_and_learned_every_entry():
    import torch
    import paper_2206_07244_amd as ops
    A = syn.banded(1 << 21, 64, 12, seed=22)
    _say("band21 generated", A.nnz)
    dA = ops.DeviceCSR.from_host(A)
    ref = oracle.spgemm(A, A, threads=_threads())
    _say("oracle done", int(ref[0][-1]))
    C = ops.spgemm(dA, dA, config=_tuned("banded"))
    torch.cuda.synchronize()
    info = oracle.compare(*C.to_host(), ref)
    _say("band21 plain", info)
    del C
    st = ops.Stats()
    C = ops.spgemm_learned(dA, dA, ops.Predictor.load(), stats=st)
    torch.cuda.synchronize()
    info = oracle.compare(*C.to_host(), ref)
    _say("band21 learned", info, st.as_dict())


def _rmat21_panel(k, P):
    A = syn.rmat(21, 16, 0.57, 0.19, 0.19, seed=21)
    nprod, _, _, tot = oracle.row_stats(A, A)
    cum = np.cumsum(nprod)
    r0 = int(np.searchsorted(cum, tot * k / P, side="right")) if k else 0
    r1 = int(np.searchsorted(cum, tot * (k + 1) / P, side="right")) if k + 1 < P else A.rows
    return A, r0, r1


def test_rmat21_panel_plain_and_learned():
    import torch
    import paper_2206_07244_amd as ops
    A, r0, r1 = _rmat21_panel(0, 8)
    _say("rmat21 generated; panel 0/8 rows", r0, r1)
    dA = ops.DeviceCSR.from_host(A)
    dP = ops.DeviceCSR(r1 - r0, A.cols, dA.rpt[r0:r1 + 1], dA.col, dA.val)
    rows_abs = np.arange(r0, r1)
    cfg = _tuned("rmat")
    C = ops.spgemm(dP, dA, config=cfg)
    torch.cuda.synchronize()
    _say("plain done", C.nnz)
    sb, nb = _full_rpt_and_bins(ops, A, rows_abs, C, cfg, "rmat21 panel plain")
    del C
    st = ops.Stats()
    C = ops.spgemm_learned(dP, dA, ops.Predictor.load(), stats=st)
    torch.cuda.synchronize()
    _say("learned done", st.as_dict())
    _full_rpt_and_bins(ops, A, rows_abs, C, None, "rmat21 panel learned")


def test_batch512_every_problem():
    import torch
    import paper_2206_07244_amd as ops
    pairs = syn.batch_pairs(512, seed=4)
    _say("batch512 generated", sum(a.rows for a, _ in pairs))
    dev = [(ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)) for A, B in pairs]
    batch = ops.Batch([a for a, _ in dev], [b for _, b in dev], config=_tuned("batch"))
    st = ops.Stats()
    views = batch.execute(stats=st)
    torch.cuda.synchronize()
    _say("batch executed", st.nprod, st.nnz)
    th = _threads()
    worst = 0.0
    for p, ((A, B), v) in enumerate(zip(pairs, views)):
        info = oracle.compare(*v.to_host(), oracle.spgemm(A, B, threads=th))
        worst = max(worst, info["max_err_over_S"])
    _say("batch512: every problem matches, max |d|/S", worst)
