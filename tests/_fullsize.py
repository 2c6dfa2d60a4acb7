"""Helpers of the full-size parity tests: which rows each bin holds under a
bin configuration, a stratified sample of them, and the comparison of
sampled rows of a device result with the oracle.

Bin membership follows the binning method (Section 5.1): the first bin
whose inclusive upper bound holds the row's value (n_prod for the
symbolic step, nnz for the numeric step), the last bin unbounded.  The
bounds are the configuration's explicit ones where it gives them, else
the ratio rule of Section 5.7 over the library's table sizes.
"""
import numpy as np

import oracle

TOL = 1e-12


def step_bounds(ops, cfg, step):
    """Inclusive upper bounds of the LDS bins of a step (symbolic 0: bins
    0..6 of the n_prod bins; numeric 1: bins 0..6) under `cfg`."""
    ts = ops.table_sizes(step)
    nb = 7
    ratio = 0.0
    explicit = [0] * nb
    if cfg is not None:
        ratio = cfg.sym_ratio if step == 0 else cfg.num_ratio
        explicit = list(cfg.sym_bounds if step == 0 else cfg.num_bounds)
    if ratio <= 0:
        ratio = 1.2 if step == 0 else 2.0
    derived = oracle.bin_ranges(ts[:nb], ratio, numeric=(step == 1))
    return [e if e != 0 else d for e, d in zip(explicit, derived)]


def bins_of(ops, cfg, nprod, nnz):
    """(symbolic bin, numeric bin) of every row.  Symbolic bin 8 marks the
    rows of bin 7 whose size passes the abort threshold of the largest LDS
    table (they are recomputed with global tables)."""
    sb = oracle.bin_of(nprod, step_bounds(ops, cfg, 0))
    frac = 0.8
    if cfg is not None and cfg.sym_abort_fraction > 0:
        frac = cfg.sym_abort_fraction
    t7 = ops.table_sizes(0)[7]
    sb = np.where((sb == 7) & (nnz > int(frac * t7)), 8, sb)
    nb = oracle.bin_of(nnz, step_bounds(ops, cfg, 1))
    return sb, nb


def stratified_rows(sym_bins, num_bins, per_bin, seed, extra=()):
    """Up to `per_bin` seeded random rows of every symbolic and every
    numeric bin (all rows of a smaller bin), plus `extra`, ascending."""
    rng = np.random.default_rng(seed)
    picks = [np.asarray(extra, np.int64)]
    for bins in (sym_bins, num_bins):
        for b in np.unique(bins):
            rows = np.nonzero(bins == b)[0]
            k = min(per_bin, rows.size)
            picks.append(rng.choice(rows, k, replace=False))
    return np.unique(np.concatenate(picks)).astype(np.int64)


def per_bin_counts(rows, sym_bins, num_bins):
    s = {int(b): int(np.sum(sym_bins[rows] == b)) for b in np.unique(sym_bins)}
    n = {int(b): int(np.sum(num_bins[rows] == b)) for b in np.unique(num_bins)}
    return s, n


def compare_rows(C, rpt_host, rows, A, B, threads, ref_rows=None):
    """Rows `rows` of the device result C (rpt_host = C's row pointer on
    the host) against the oracle's rows `ref_rows` of A*B (default: the
    same indices): columns identical, |c - c_ref| <= TOL * S.  The rows'
    entries are gathered on the device and copied once."""
    import torch
    ref = oracle.spgemm(A, B, rows=rows if ref_rows is None else ref_rows, threads=threads)
    starts = rpt_host[rows]
    lens = rpt_host[rows + 1] - starts
    np.testing.assert_array_equal(lens, np.diff(ref[0]))
    total = int(lens.sum())
    if total == 0:
        return 0.0
    idx = np.repeat(starts - np.cumsum(np.concatenate([[0], lens[:-1]])), lens) + np.arange(total)
    ix = torch.from_numpy(idx).to(C.col.device)
    col = C.col.index_select(0, ix).cpu().numpy()
    val = C.val.index_select(0, ix).cpu().numpy()
    np.testing.assert_array_equal(col, ref[1])
    err = np.abs(val - ref[2])
    bad = err > TOL * ref[3]
    assert not np.any(bad), f"{int(bad.sum())} values outside the tolerance"
    s = ref[3] > 0
    return float(np.max(err[s] / ref[3][s])) if np.any(s) else 0.0
