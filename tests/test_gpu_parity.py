"""GPU parity: the HIP pipeline against the CPU oracle, element by element.

Row pointers and column indices must be identical; values must satisfy
|c - c_ref| <= 1e-12 * S_ij with S_ij = sum_k |a_ik b_kj| (the summation order
of the GPU's hash-table atomics differs from the oracle's sequential order,
and S bounds the rounding difference of any order).  Integer-valued inputs
are exact in any order and must match bit for bit.
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


def gpu_product(A, B=None, cfg=None, stats=None):
    import torch
    ops = _ops()
    dA = ops.DeviceCSR.from_host(A)
    dB = dA if B is None else ops.DeviceCSR.from_host(B)
    C = ops.spgemm(dA, dB, config=cfg, stats=stats)
    torch.cuda.synchronize()
    return C.to_host()


def check(A, B=None, cfg=None, exact=False, stats=None):
    Bm = A if B is None else B
    if cfg is None:
        cfg = _ops().Config(validate=1)
    got = gpu_product(A, B, cfg, stats)
    ref = oracle.spgemm(A, Bm)
    info = oracle.compare(*got, ref, tol=TOL)
    if exact:
        assert info["bit_exact_values"], info
    return info


def test_lap5_64_bit_exact():
    st = _ops().Stats()
    info = check(syn.lap5(64), exact=True, stats=st)
    assert st.nprod == 100104 and st.nnz == 51972


@pytest.mark.parametrize("g", [1, 2, 5, 20])
def test_stencil27_small(g):
    check(syn.stencil27(g, seed=g))


@pytest.mark.parametrize("g", [1, 2, 6, 12])
def test_block_stencil27_small(g):
    """High compression-ratio rows (3x3 node blocks): closed-form totals and
    every entry."""
    st = _ops().Stats()
    check(syn.block_stencil27(g, 3, seed=g), stats=st)
    if g >= 2:
        assert st.nprod == 27 * (9 * g - 10) ** 3
    if g >= 4:
        assert st.nnz == 9 * (5 * g - 6) ** 3


@pytest.mark.parametrize("scale", [10, 14])
def test_rmat_all_bins(scale):
    st = _ops().Stats()
    check(syn.rmat(scale, 16, seed=scale), stats=st)
    if scale == 14:
        # every numeric bin, including the global-table bin, is exercised
        assert all(x > 0 for x in st.num_bin_rows), list(st.num_bin_rows)


def test_banded_and_poisson_rectangular():
    check(syn.banded(20000, 64, 12, seed=3))
    A = syn.poisson_uniform(3000, 5000, 6.0, seed=1)
    B = syn.poisson_uniform(5000, 2000, 9.0, seed=2)
    check(A, B)


@pytest.mark.parametrize("m,k,n,d", [(1, 1, 1, 1.0), (7, 0, 5, 0.5), (0, 4, 4, 0.5),
                                     (30, 40, 0, 0.5), (50, 60, 70, 0.0), (257, 300, 129, 0.05),
                                     (100, 100, 100, 0.6)])
def test_small_and_degenerate(m, k, n, d):
    A = syn.random_csr(m, k, d, seed=m + k, values="int")
    B = syn.random_csr(k, n, d, seed=n + k + 1, values="int")
    check(A, B, exact=True)


def test_identity_products_exact():
    A = syn.random_csr(300, 200, 0.03, seed=4)
    check(A, syn.identity(200), exact=True)
    check(syn.identity(300), A, exact=True)


def test_explicit_zero_kept():
    A = syn.CSR(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    B = syn.CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([1.0, -1.0]))
    rpt, col, val = gpu_product(A, B)
    assert list(rpt) == [0, 1] and list(col) == [0] and val[0] == 0.0


@pytest.mark.parametrize("b", list(range(9)))
@pytest.mark.parametrize("hash_all", [0, 1])
def test_forced_symbolic_bin(b, hash_all):
    ops = _ops()
    cfg = ops.Config(force_sym_bin=b, validate=1, hash_all_rows=hash_all)
    st = ops.Stats()
    check(syn.rmat(12, 16, seed=5), cfg=cfg, stats=st)
    assert st.sym_bin_rows[b] > 0


@pytest.mark.parametrize("b", list(range(8)))
@pytest.mark.parametrize("hash_all", [0, 1])
def test_forced_numeric_bin(b, hash_all):
    ops = _ops()
    cfg = ops.Config(force_num_bin=b, validate=1, hash_all_rows=hash_all)
    st = ops.Stats()
    check(syn.rmat(12, 16, seed=6), cfg=cfg, stats=st)
    assert st.num_bin_rows[b] > 0


def test_every_big_row_recomputed_globally():
    """With every row hashed (the paper's method), abort-fraction -1 sends
    every bin-7 row to the global tables."""
    ops = _ops()
    cfg = ops.Config(sym_abort_fraction=-1.0, validate=1, hash_all_rows=1)
    st = ops.Stats()
    check(syn.rmat(14, 16, seed=7), cfg=cfg, stats=st)
    assert st.sym_bin_rows[7] > 0 and st.sym_bin_rows[8] >= st.sym_bin_rows[7]


@pytest.mark.parametrize("rowlen", [1, 3, 8, 20, 40, 70, 100, 300])
def test_b_row_lengths(rowlen):
    """Uniform B rows of many lengths drive both product mappings (grouped
    lanes for B rows up to 64 entries, flat windows beyond)."""
    A = syn.poisson_uniform(700, 900, 6.0, seed=rowlen)
    B = syn.poisson_uniform(900, 5000, float(rowlen), seed=rowlen + 1)
    check(A, B)


@pytest.mark.parametrize("ratios", [(1.0, 1.0), (1.5, 3.0)])
def test_other_binning_ratios(ratios):
    ops = _ops()
    check(syn.rmat(13, 16, seed=9), cfg=ops.Config(sym_ratio=ratios[0], num_ratio=ratios[1], validate=1))


def test_symbolic_numeric_split_and_rerun():
    import torch
    ops = _ops()
    A = syn.rmat(12, 16, seed=10)
    dA = ops.DeviceCSR.from_host(A)
    plan = ops.spgemm_symbolic(dA, dA)
    ref = oracle.spgemm(A, A)
    assert plan.nnz == ref[0][-1]
    C1 = ops.spgemm_numeric(plan, dA, dA)
    torch.cuda.synchronize()
    oracle.compare(*C1.to_host(), ref)
    # same structure, new values: the plan is reused
    A2 = syn.CSR(A.rows, A.cols, A.rpt, A.col, np.random.default_rng(1).standard_normal(A.nnz))
    dA2 = ops.DeviceCSR.from_host(A2)
    out = ops.DeviceCSR(A.rows, A.cols, torch.empty(A.rows + 1, dtype=torch.int64, device="cuda"),
                        torch.empty(plan.nnz, dtype=torch.int32, device="cuda"),
                        torch.empty(plan.nnz, dtype=torch.float64, device="cuda"))
    C2 = ops.spgemm_numeric(plan, dA2, dA2, out=out)
    torch.cuda.synchronize()
    oracle.compare(*C2.to_host(), oracle.spgemm(A2, A2))


def test_row_range_view_of_A():
    """rpt holds absolute offsets, so a slice of rows is a valid input."""
    import torch
    ops = _ops()
    A = syn.rmat(11, 16, seed=11)
    dA = ops.DeviceCSR.from_host(A)
    lo, hi = 300, 1500
    view = ops.DeviceCSR(hi - lo, A.cols, dA.rpt[lo:hi + 1], dA.col, dA.val)
    C = ops.spgemm(view, dA)
    torch.cuda.synchronize()
    ref = oracle.spgemm(A, A, rows=np.arange(lo, hi))
    oracle.compare(*C.to_host(), ref)


def test_structure_deterministic_over_runs():
    """Twenty runs give the same row pointer and columns (row order in the
    bins, the tile lists of long rows and the bins on side streams vary
    from run to run; the structure must not)."""
    import torch
    ops = _ops()
    A = syn.rmat(12, 16, seed=12)
    dA = ops.DeviceCSR.from_host(A)
    first = None
    for _ in range(20):
        C = ops.spgemm(dA, dA)
        torch.cuda.synchronize()
        r, c, _v = C.to_host()
        if first is None:
            first = (r, c)
        else:
            assert np.array_equal(first[0], r) and np.array_equal(first[1], c)


@pytest.mark.parametrize("b", list(range(9)))
@pytest.mark.parametrize("hash_all", [0, 1])
def test_forced_bins_persistent_launch(b, hash_all):
    """Symbolic bin kernels (and numeric bin 0) launched with a small fixed
    grid, so each workgroup walks many rows (the launch form of captured
    graphs)."""
    ops = _ops()
    st = ops.Stats()
    cfg = ops.Config(force_sym_bin=b, force_num_bin=0 if b == 0 else -1, validate=1, fixed_grid=7,
                     hash_all_rows=hash_all)
    check(syn.rmat(12, 16, seed=13), cfg=cfg, stats=st)
    assert st.sym_bin_rows[b] > 0


def test_persistent_launch_all_bins_rmat14():
    ops = _ops()
    st = ops.Stats()
    check(syn.rmat(14, 16, seed=14), cfg=ops.Config(validate=1, fixed_grid=5), stats=st)
    assert all(x > 0 for x in st.num_bin_rows)


@pytest.mark.parametrize("b", list(range(9)))
@pytest.mark.parametrize("grid", [0, 7])
def test_forced_symbolic_bin_narrow_rows(b, grid):
    """Rows whose output columns span a narrow range are counted with a
    bitmap of that range in bins 1-7 (hash tables in bins 0 and 8): force
    every row of a banded matrix and of a 27-point stencil through each bin,
    with one team per row and with a small persistent grid."""
    ops = _ops()
    mats = [syn.banded(3000, 40, 9, seed=b)]
    if b > 0:   # no 27-point row has as few products as bin 0 holds
        mats.append(syn.stencil27(9, seed=b))
    for A in mats:
        st = ops.Stats()
        cfg = ops.Config(force_sym_bin=b, validate=1, fixed_grid=grid)
        check(A, cfg=cfg, stats=st)
        assert st.sym_bin_rows[b] > 0


def test_narrow_and_wide_rows_mixed():
    """One product whose rows alternate between a narrow column range and
    the full width (wide rows take the hash table)."""
    n = 4000
    A = syn.banded(n, 8, 5, seed=1)
    W = syn.random_csr(n, n, 3.0 / n, seed=2)
    rows = np.arange(n)
    pick = (rows % 2 == 0)
    rpt = [0]
    col, val = [], []
    for i in range(n):
        src = A if pick[i] else W
        a, b = src.rpt[i], src.rpt[i + 1]
        col.append(src.col[a:b])
        val.append(src.val[a:b])
        rpt.append(rpt[-1] + (b - a))
    M = syn.CSR(n, n, np.array(rpt, np.int64), np.concatenate(col).astype(np.int32),
                np.concatenate(val))
    check(M)


def _stack_rows(parts, n_cols):
    """Rows of several CSR matrices, one after the other, as one matrix with
    n_cols columns (each part shifted right by its column offset)."""
    rpt, col, val = [np.zeros(1, np.int64)], [], []
    for M, shift in parts:
        rpt.append(rpt[-1][-1] + M.rpt[1:])
        col.append(M.col.astype(np.int64) + shift)
        val.append(M.val)
    rows = sum(M.rows for M, _ in parts)
    return syn.CSR(rows, n_cols, np.concatenate(rpt), np.concatenate(col).astype(np.int32),
                   np.concatenate(val))


@pytest.mark.parametrize("n_cols", [3 * (1 << 20) + 12345, 9 * (1 << 20) + 7])
@pytest.mark.parametrize("hash_all", [0, 1])
def test_global_symbolic_bin_wide_ranges(n_cols, hash_all):
    """Every row forced into the global symbolic bin, with output ranges of
    a few thousand columns (one bitmap window), of several windows, and (at
    more than 8 * 2^20 columns) wider than the bitmap takes, which go to the
    global hash tables; numeric in its own bins and forced to the bucketed
    kernel."""
    ops = _ops()
    Bn = syn.poisson_uniform(1500, 70000, 40.0, seed=1)        # narrow rows of B
    Bw = syn.poisson_uniform(1500, n_cols, 40.0, seed=2)       # rows over all columns
    B = _stack_rows([(Bn, n_cols // 2), (Bw, 0)], n_cols)
    An = syn.poisson_uniform(120, 1500, 50.0, seed=3)          # references narrow rows only
    Aw = syn.poisson_uniform(120, 3000, 50.0, seed=4)
    A = _stack_rows([(An, 0), (Aw, 0)], 3000)
    for force_num in (-1, 7):
        st = ops.Stats()
        cfg = ops.Config(force_sym_bin=8, force_num_bin=force_num, validate=1,
                         hash_all_rows=hash_all)
        check(A, B, cfg=cfg, stats=st)
        assert st.sym_bin_rows[8] == A.rows


def _rows_with_output_counts(counts, n_cols=200003, seed=11):
    """A, B with row i of A·B holding exactly counts[i] distinct columns
    spread over n_cols (wider than any numeric LDS table, so rows are hashed
    and then ordered): B rows k < K hold one column each, (48271 k) mod
    n_cols (distinct, n_cols prime); B rows K + k repeat row k's column, and
    A rows also reference up to five of those, so some outputs accumulate
    two products."""
    rng = np.random.default_rng(seed)
    K = 4096
    bcol = np.array([(48271 * k) % n_cols for k in range(K)] * 2, dtype=np.int32)
    B = syn.CSR(2 * K, n_cols, np.arange(2 * K + 1, dtype=np.int64), bcol, rng.uniform(-1, 1, 2 * K))
    rpt, col = [0], []
    for i, n in enumerate(counts):
        k0 = (131 * i) % (K - 200)
        ent = list(range(k0, k0 + n)) + list(range(K + k0, K + k0 + min(n, 5)))
        col.extend(sorted(ent))
        rpt.append(len(col))
    A = syn.CSR(len(counts), 2 * K, np.array(rpt, np.int64), np.array(col, np.int32),
                rng.uniform(-1, 1, len(col)))
    return A, B


@pytest.mark.parametrize("hash_all", [0, 1])
def test_one_wave_rows_around_64_outputs(hash_all):
    """One-wave numeric rows of 0-128 outputs, on both sides of the 64-entry
    limit below which entries are ranked from registers instead of the
    two-level bitmap."""
    ops = _ops()
    counts = [0, 1, 2, 31, 63, 64, 65, 66, 100, 127, 128] * 3
    A, B = _rows_with_output_counts(counts)
    st = ops.Stats()
    cfg = ops.Config(force_num_bin=1, validate=1, hash_all_rows=hash_all)
    check(A, B, cfg=cfg, stats=st)
    assert st.num_bin_rows[1] == A.rows
    assert st.nnz == sum(counts)


@pytest.mark.parametrize("hash_all", [1, 0])
def test_multi_access_hash_variant(hash_all):
    """The library built with the multiple-access hash probe (the hashing
    ablation of Section 6.3.2) computes the same product."""
    import ctypes
    import torch
    ops = _ops()
    V = ops.lib_variant("multi_access")
    for A in (syn.rmat(13, 16, seed=7), syn.stencil27(12, seed=3), syn.banded(5000, 64, 12, seed=4)):
        dA = ops.DeviceCSR.from_host(A)
        Ac = dA._c()
        cfg = ops.Config(validate=1, hash_all_rows=hash_all)
        Cc = ops.opsp_csr()
        sh = torch.cuda.current_stream().cuda_stream
        code = V.opsp_spgemm_ex(ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(Cc), ctypes.byref(cfg),
                                None, sh)
        assert code == 0, code
        rpt = ops._wrap(Cc.rpt, Cc.rows + 1, torch.int64, None, dA.rpt.device).cpu().numpy()
        col = ops._wrap(Cc.col, Cc.nnz, torch.int32, None, dA.rpt.device).cpu().numpy()
        val = ops._wrap(Cc.val, Cc.nnz, torch.float64, None, dA.rpt.device).cpu().numpy()
        assert V.opsp_csr_free(ctypes.byref(Cc), sh) == 0
        oracle.compare(rpt, col, val, oracle.spgemm(A, A), tol=TOL)



@pytest.mark.parametrize("streams", [2, 4])
def test_bins_on_several_streams(streams):
    """Bin kernels spread over the calling stream and library side streams
    give the same product (every symbolic and numeric bin populated)."""
    st = _ops().Stats()
    cfg = _ops().Config(validate=1, streams=streams)
    check(syn.rmat(14, 16, seed=14), cfg=cfg, stats=st)
    assert all(x > 0 for x in st.num_bin_rows), list(st.num_bin_rows)
    for b in (0, 3, 7):
        check(syn.rmat(12, 16, seed=b), cfg=_ops().Config(streams=streams, force_num_bin=b,
                                                          force_sym_bin=b))


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_group_lanes_variants(lanes):
    """Bin 0 with 4, 8 or 16 lanes per row (tables of 64 / 128 / 256 keys and
    19 / 39 / 79 entries), every row that fits routed there."""
    ops = _ops()
    cases = [(syn.poisson_uniform(5000, 4000, 3.0, seed=1), syn.poisson_uniform(4000, 3000, 4.0, seed=2)),
             (syn.lap5(30), None), (syn.rmat(12, 4, seed=12), None),
             (syn.random_csr(300, 200, 0.08, seed=3, values="int"),
              syn.random_csr(200, 300, 0.08, seed=4, values="int"))]
    for i, (A, B) in enumerate(cases):
        for forced in (-1, 0):
            st = ops.Stats()
            check(A, B, cfg=ops.Config(validate=1, group_lanes=lanes, force_sym_bin=forced,
                                       force_num_bin=forced), stats=st)
            if forced == 0 and i == 0:   # rows of about 12 products: all fit bin 0
                assert st.sym_bin_rows[0] > 0 and st.num_bin_rows[0] > 0



def _narrow_range_rows(widths, ms, L=64, G=1100, seed=21):
    """A, B whose product rows have exactly the given column range widths and
    numbers of products: B holds, per width w, G rows of L entries in
    [base, base + w) that all include base and base + w - 1; A row (w, m)
    references m distinct B rows of width w's group (m * L products, range
    exactly w)."""
    rng = np.random.default_rng(seed)
    uw = sorted(set(widths))
    n_cols = sum(uw) + 17
    brpt, bcol, base, group = [0], [], 0, {}
    for gi, w in enumerate(uw):
        group[w] = gi * G
        for _ in range(G):
            mid = rng.choice(np.arange(1, w - 1), L - 2, replace=False)
            bcol.append(np.sort(np.concatenate([[0, w - 1], mid])) + base)
            brpt.append(brpt[-1] + L)
        base += w
    B = syn.CSR(len(uw) * G, n_cols, np.array(brpt, np.int64),
                np.concatenate(bcol).astype(np.int32), rng.uniform(-1, 1, brpt[-1]))
    arpt, acol = [0], []
    for w, m in zip(widths, ms):
        acol.append(np.sort(rng.choice(G, m, replace=False)) + group[w])
        arpt.append(arpt[-1] + m)
    A = syn.CSR(len(widths), B.rows, np.array(arpt, np.int64),
                np.concatenate(acol).astype(np.int32), rng.uniform(-1, 1, arpt[-1]))
    return A, B


@pytest.mark.parametrize("hash_all", [0, 1])
def test_symbolic_rows_routed_by_range(hash_all):
    """Rows of thousands of products whose output range fits the one-wave
    kernel's bitmap (32 * 1024 columns) are counted there up to 2^13
    products; a column more, or a B row more, keeps them in the bin of their
    n_prod.  Without ranges (every row hashed) nothing is routed."""
    ops = _ops()
    widths, ms, routed = [], [], 0
    for w in (1000, 20000, 32768, 32769):
        for m in (31, 128, 129, 1024):
            widths.append(w)
            ms.append(m)
            routed += (w <= 32768 and m * 64 <= 8192)
    A, B = _narrow_range_rows(widths, ms)
    st = ops.Stats()
    check(A, B, cfg=ops.Config(validate=1, hash_all_rows=hash_all), stats=st)
    assert st.sym_bin_rows[1] == (0 if hash_all else routed)


def _rows_of_lengths(lengths, K, seed):
    """A with rows of the given entry counts over K columns (distinct sorted
    columns, U(-1, 1) values)."""
    rng = np.random.default_rng(seed)
    rpt, cols = [0], []
    for L in lengths:
        cols.append(np.sort(rng.choice(K, L, replace=False)))
        rpt.append(rpt[-1] + L)
    return syn.CSR(len(lengths), K, np.array(rpt, np.int64),
                   np.concatenate(cols).astype(np.int32), rng.uniform(-1, 1, rpt[-1]))


LONG_ROW_LENGTHS = ([0, 1, 512, 513, 1023, 1024, 1025, 2049, 0, 5000, 70000, 3, 1500] + [7] * 200 +
                    [600] * 70 + [0] * 30 + [3000])


@pytest.mark.parametrize("hash_all", [0, 1])
def test_setup_long_rows_in_tiles(hash_all):
    """Rows of more than 512 A entries are walked by the setup step in tiles
    of 512 entries on many waves: lengths on both sides of one and two
    tiles, one row of 70,000 entries, a wave of 64 rows that are all long,
    long rows next to empty ones; n_prod is compared through the product and
    the per-row features."""
    import torch
    ops = _ops()
    A = _rows_of_lengths(LONG_ROW_LENGTHS, 80000, seed=31)
    B = syn.random_csr(80000, 5000, 0.0006, seed=32)
    st = ops.Stats()
    check(A, B, cfg=ops.Config(validate=1, hash_all_rows=hash_all), stats=st)
    nprod, alen, bmax, _ = oracle.row_stats(A, B)
    assert st.nprod == int(nprod.sum())
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    al, npd, bm = ops.row_features(dA, dB)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(npd.cpu().numpy(), nprod)
    np.testing.assert_array_equal(al.cpu().numpy(), alen)
    np.testing.assert_array_equal(bm.cpu().numpy(), bmax)
    # a view of rows 5..300 (rpt[0] != 0, the long rows cut at both ends)
    lo, hi = 5, 300
    view = ops.DeviceCSR(hi - lo, A.cols, dA.rpt[lo:hi + 1], dA.col, dA.val)
    C = ops.spgemm(view, dB, config=ops.Config(validate=1, hash_all_rows=hash_all))
    torch.cuda.synchronize()
    oracle.compare(*C.to_host(), oracle.spgemm(A, B, rows=np.arange(lo, hi)), tol=TOL)


def _setup_wave_lengths(seed=41):
    """Row lengths per 64-row wave of the setup step: all 81; uniform in
    65..256; one row of 256 among rows of 3 (longest above twice the mean);
    one of 257 among rows of 200; 64 and 65 mixed; rows of 128 beside empty
    ones (longest exactly twice the mean); a last partial wave of 10 rows of
    200."""
    rng = np.random.default_rng(seed)
    waves = [[81] * 64,
             list(rng.integers(65, 257, 64)),
             [256] + [3] * 63,
             [257] + [200] * 63,
             [64, 65] * 32,
             [128, 0] * 32,
             [200] * 10]
    return [int(x) for w in waves for x in w]


@pytest.mark.parametrize("hash_all", [0, 1])
def test_setup_rows_of_65_to_256_entries(hash_all):
    """The setup step lets every lane walk its own row when the wave's rows
    have at most 256 entries and the longest at most twice their mean, and
    walks the flat entry range otherwise: n_prod, a_len and b_max per row
    and the product must match the oracle on both sides of those limits."""
    import torch
    ops = _ops()
    A = _rows_of_lengths(_setup_wave_lengths(), 3000, seed=42)
    B = syn.random_csr(3000, 4000, 0.01, seed=43)
    st = ops.Stats()
    check(A, B, cfg=ops.Config(validate=1, hash_all_rows=hash_all), stats=st)
    nprod, alen, bmax, _ = oracle.row_stats(A, B)
    assert st.nprod == int(nprod.sum())
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    al, npd, bm = ops.row_features(dA, dB)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(npd.cpu().numpy(), nprod)
    np.testing.assert_array_equal(al.cpu().numpy(), alen)
    np.testing.assert_array_equal(bm.cpu().numpy(), bmax)
    # a view starting at row 7 shifts every wave's rows
    lo, hi = 7, A.rows
    view = ops.DeviceCSR(hi - lo, A.cols, dA.rpt[lo:hi + 1], dA.col, dA.val)
    C = ops.spgemm(view, dB, config=ops.Config(validate=1, hash_all_rows=hash_all))
    torch.cuda.synchronize()
    oracle.compare(*C.to_host(), oracle.spgemm(A, B, rows=np.arange(lo, hi)), tol=TOL)


@pytest.mark.parametrize("hash_all", [0, 1])
def test_b_rows_of_65_to_128_entries(hash_all):
    """B rows of exactly 63-65, 100, 127-129 entries, around the limit of
    the grouped product mapping (B rows of at most 64 entries) and beyond
    it (flat windows).  A's rows mix the lengths, one row per length alone,
    in several symbolic and numeric bin kernels (forced) and in the binned
    default."""
    ops = _ops()
    rng = np.random.default_rng(65)
    lens = [63, 64, 65, 100, 127, 128, 129]
    K, N = 700, 6000
    brpt, bcol = [0], []
    for k in range(K):
        L = lens[k % len(lens)]
        bcol.append(np.sort(rng.choice(N, L, replace=False)))
        brpt.append(brpt[-1] + L)
    B = syn.CSR(K, N, np.array(brpt, np.int64), np.concatenate(bcol).astype(np.int32),
                rng.uniform(-1, 1, brpt[-1]))
    arpt, acol = [0], []
    for i in range(300):
        if i < len(lens):   # one row per length alone
            cols = np.arange(i, K, len(lens))[:5 + i]
        else:
            cols = np.sort(rng.choice(K, 1 + i % 90, replace=False))
        acol.append(cols)
        arpt.append(arpt[-1] + len(cols))
    A = syn.CSR(300, K, np.array(arpt, np.int64), np.concatenate(acol).astype(np.int32),
                rng.uniform(-1, 1, arpt[-1]))
    check(A, B, cfg=ops.Config(validate=1, hash_all_rows=hash_all))
    for b in (1, 4, 7):
        check(A, B, cfg=ops.Config(validate=1, hash_all_rows=hash_all, force_sym_bin=b, force_num_bin=b))


@pytest.mark.parametrize("declared_nnz", [3000, 42000])
def test_setup_long_row_list_full(declared_nnz):
    """The setup step's list of long rows is sized from A's declared entry
    count.  An A that declares fewer entries than its rows span (the arrays
    themselves are whole) fills the list: with 3,000 no wave's reservation
    fits, with 42,000 the first wave's long rows are listed and the later
    waves' are not; waves whose reservation does not fit walk their long
    rows themselves.  The product is unchanged (validation off: it would
    reject the declared count)."""
    import ctypes
    import torch
    ops = _ops()
    A = _rows_of_lengths(LONG_ROW_LENGTHS, 80000, seed=31)
    B = syn.random_csr(80000, 5000, 0.0006, seed=32)
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    Ac, Bc, Cc = dA._c(), dB._c(), ops.opsp_csr()
    assert Ac.nnz > declared_nnz
    Ac.nnz = declared_nnz
    s = torch.cuda.current_stream().cuda_stream
    st = ops.Stats()
    code = ops.lib().opsp_spgemm_ex(ctypes.byref(Ac), ctypes.byref(Bc), ctypes.byref(Cc), None,
                                    ctypes.byref(st), s)
    assert code == 0, code
    C = ops._adopt(Cc, s, dA.rpt.device)
    torch.cuda.synchronize()
    nprod, _, _, _ = oracle.row_stats(A, B)
    assert st.nprod == int(nprod.sum())
    oracle.compare(*C.to_host(), oracle.spgemm(A, B), tol=TOL)


def _repeated_pattern_rows(seed=77):
    """B with runs of rows that share one column set (three unknowns of a
    node), rows that match a neighbour in length and end columns but not in
    the middle, and identical rows longer than the compared length (300
    entries); A rows that take whole runs, parts of runs, and runs with a
    row left out."""
    rng = np.random.default_rng(seed)
    N = 4000
    brows = []
    for g in range(120):
        kind = g % 4
        L = [20, 64, 100, 300][kind]
        pat = np.sort(rng.choice(N, L, replace=False))
        if kind == 2 and g % 8 == 2:   # same length and ends, one middle column moved
            alt = pat.copy()
            free = np.setdiff1d(np.arange(pat[0] + 1, pat[-1]), pat)
            alt[L // 2] = free[0]
            brows += [pat, np.sort(alt), pat]
        else:
            brows += [pat, pat, pat]
    brpt = np.concatenate([[0], np.cumsum([len(r) for r in brows])]).astype(np.int64)
    B = syn.CSR(len(brows), N, brpt, np.concatenate(brows).astype(np.int32),
                rng.uniform(-1, 1, int(brpt[-1])))
    K = len(brows)
    arows = []
    for i in range(400):
        m = i % 5
        if m == 0:      # whole runs
            g = rng.choice(K // 3, 4, replace=False)
            cols = np.concatenate([[3 * x, 3 * x + 1, 3 * x + 2] for x in g])
        elif m == 1:    # the last two of a run
            g = rng.choice(K // 3, 5, replace=False)
            cols = np.concatenate([[3 * x + 1, 3 * x + 2] for x in g])
        elif m == 2:    # a run with its middle row left out
            g = rng.choice(K // 3, 5, replace=False)
            cols = np.concatenate([[3 * x, 3 * x + 2] for x in g])
        elif m == 3:    # random rows
            cols = rng.choice(K, 12, replace=False)
        else:           # one whole run alone
            x = int(rng.integers(K // 3))
            cols = np.array([3 * x, 3 * x + 1, 3 * x + 2])
        arows.append(np.unique(cols))
    arpt = np.concatenate([[0], np.cumsum([len(r) for r in arows])]).astype(np.int64)
    A = syn.CSR(len(arows), K, arpt, np.concatenate(arows).astype(np.int32),
                rng.uniform(-1, 1, int(arpt[-1])))
    return A, B


@pytest.mark.parametrize("forced", [-1, 1, 4, 7, 8])
def test_symbolic_skips_repeated_row_patterns(forced):
    """The symbolic step skips an A entry whose B row has the same columns as
    the B row of the entry before it (flagged by the B row records); the
    counts, and so the product, must equal the oracle's whatever the
    symbolic kernel."""
    ops = _ops()
    A, B = _repeated_pattern_rows()
    check(A, B, cfg=ops.Config(validate=1, force_sym_bin=forced))


def _runs_of_rows(N, seed, integer=False):
    """B made of groups of 1, 2, 3, 4, 5 or 7 consecutive rows with one
    column set (rows of 40, 64 or 100 entries); A rows that take whole
    groups, stretches of 65-140 consecutive B rows (runs cross the 64-entry
    chunks of a row), groups with a row left out, a lone group of 7 (longer
    than a merged run) and random rows."""
    rng = np.random.default_rng(seed)
    brows, groups = [], []
    for g in range(72):
        R = [1, 2, 3, 4, 5, 7][g % 6]
        L = [40, 64, 100][(g // 6) % 3]
        pat = np.sort(rng.choice(N, L, replace=False))
        groups.append((len(brows), R))
        brows += [pat] * R
    K = len(brows)
    brpt = np.concatenate([[0], np.cumsum([len(r) for r in brows])]).astype(np.int64)
    nb = int(brpt[-1])
    ints = np.array([-3.0, -2.0, -1.0, 1.0, 2.0, 3.0])   # nonzero: no signed zeros in the sums
    bval = rng.choice(ints, nb) if integer else rng.uniform(-1, 1, nb)
    B = syn.CSR(K, N, brpt, np.concatenate(brows).astype(np.int32), bval)
    arows = []
    for i in range(300):
        m = i % 5
        if m == 0:
            gs = rng.choice(len(groups), 5, replace=False)
            cols = np.concatenate([np.arange(groups[x][0], groups[x][0] + groups[x][1]) for x in gs])
        elif m == 1:
            s0 = int(rng.integers(0, K - 140))
            cols = np.arange(s0, s0 + int(rng.integers(65, 141)))
        elif m == 2:
            gs = rng.choice(len(groups), 5, replace=False)
            parts = []
            for x in gs:
                s, R = groups[x]
                c = np.arange(s, s + R)
                parts.append(np.delete(c, int(rng.integers(R))) if R > 1 else c)
            cols = np.concatenate(parts)
        elif m == 3:
            s = groups[5][0]
            cols = np.arange(s, s + 7)
        else:
            cols = rng.choice(K, 12, replace=False)
        arows.append(np.unique(cols))
    arpt = np.concatenate([[0], np.cumsum([len(r) for r in arows])]).astype(np.int64)
    na = int(arpt[-1])
    aval = rng.choice(ints, na) if integer else rng.uniform(-1, 1, na)
    A = syn.CSR(len(arows), K, arpt, np.concatenate(arows).astype(np.int32), aval)
    return A, B


@pytest.mark.parametrize("narrow", [False, True])
@pytest.mark.parametrize("forced", [-1, 1, 2, 3, 4, 5, 6])
def test_numeric_merges_repeated_row_patterns(forced, narrow):
    """The numeric step hands a run of up to three entries whose B rows share
    one column set to the run's first entry, which adds their summed
    products once per column: the product must equal the oracle's in every
    table kernel, with the dense accumulator of narrow rows (420 columns)
    and with hashing (20,000 columns)."""
    ops = _ops()
    A, B = _runs_of_rows(420 if narrow else 20000, seed=91 + int(narrow))
    check(A, B, cfg=ops.Config(validate=1, force_num_bin=forced))


@pytest.mark.parametrize("forced", [-1, 1, 4])
def test_numeric_merged_runs_exact(forced):
    """Integer values: every merged sum is exact, so the product matches the
    oracle bit for bit."""
    ops = _ops()
    A, B = _runs_of_rows(20000, seed=93, integer=True)
    check(A, B, cfg=ops.Config(validate=1, force_num_bin=forced), exact=True)


def _runs_of_identical_rows(seed=51):
    """A whose rows come in runs of identical column sets: runs of 1 to 70
    rows (longer than the 32-row cut, and across it), rows of 50 to 300
    entries (those above 256 are not compared), empty rows between runs;
    B random with rows of 0 to 60 entries."""
    rng = np.random.default_rng(seed)
    K = 3000
    rows = []
    while len(rows) < 1500:
        R = int(rng.choice([1, 2, 3, 5, 31, 33, 70]))
        L = int(rng.choice([50, 81, 256, 257, 300]))
        pat = np.sort(rng.choice(K, L, replace=False))
        rows += [pat] * R
        if rng.random() < 0.2:
            rows.append(np.zeros(0, np.int64))
    rpt = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    A = syn.CSR(len(rows), K, rpt, np.concatenate(rows).astype(np.int32),
                rng.uniform(-1, 1, int(rpt[-1])))
    blen = rng.integers(0, 61, K)
    brows = [np.sort(rng.choice(5000, int(n), replace=False)) for n in blen]
    brpt = np.concatenate([[0], np.cumsum(blen)]).astype(np.int64)
    B = syn.CSR(K, 5000, brpt, np.concatenate(brows).astype(np.int32),
                rng.uniform(-1, 1, int(brpt[-1])))
    return A, B


@pytest.mark.parametrize("forced", [-1, 1, 3, 7, 8])
def test_symbolic_counts_runs_of_identical_rows(forced):
    """Rows of A with the columns of the row before them are counted once
    per run (runs cut every 32 rows) and the count copied: every row's
    count must equal the oracle's whatever the symbolic kernel."""
    ops = _ops()
    A, B = _runs_of_identical_rows()
    check(A, B, cfg=ops.Config(validate=1, force_sym_bin=forced))


@pytest.mark.parametrize("g", [5, 8])
def test_block_stencil_square_runs_of_identical_rows(g):
    """C = A^2 for the 3x3-block stencil: A's rows of a node are identical,
    flagged by the B row records of the same matrix."""
    check(syn.block_stencil27(g, seed=g))


@pytest.mark.parametrize("n,L", [(2000, 64), (700, 300)])
def test_all_rows_identical(n, L):
    """Every row of A = B has the same L columns: every B row repeats the
    one before it (entries merged three at a time, rows of more than 256
    entries not compared), and every A row after the first of its 32-row
    block copies that row's count."""
    rng = np.random.default_rng(n + L)
    pat = np.sort(rng.choice(n, L, replace=False)).astype(np.int32)
    rpt = np.arange(n + 1, dtype=np.int64) * L
    A = syn.CSR(n, n, rpt, np.tile(pat, n), rng.uniform(-1, 1, n * L))
    check(A)


@pytest.mark.parametrize("share", [0.0, 0.2, 0.4])
def test_repeated_rows_below_and_above_merge_share(share):
    """B rows of 64 entries of which a given share repeat the row before
    them: the numeric step merges runs only from a third of B's rows up,
    the symbolic step skips repeats at any share; the product must match
    the oracle either way."""
    rng = np.random.default_rng(int(share * 10) + 61)
    N, K = 6000, 900
    rows = []
    while len(rows) < K:
        pat = np.sort(rng.choice(N, 64, replace=False))
        rows.append(pat)
        if rng.random() < share / (1 - share) and len(rows) < K:
            rows.append(pat)
    rows = rows[:K]
    brpt = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    B = syn.CSR(K, N, brpt, np.concatenate(rows).astype(np.int32), rng.uniform(-1, 1, int(brpt[-1])))
    arows = []
    for i in range(500):
        s0 = int(rng.integers(0, K - 12))
        arows.append(np.arange(s0, s0 + int(rng.integers(4, 12))))
    arpt = np.concatenate([[0], np.cumsum([len(r) for r in arows])]).astype(np.int64)
    A = syn.CSR(len(arows), K, arpt, np.concatenate(arows).astype(np.int32),
                rng.uniform(-1, 1, int(arpt[-1])))
    check(A, B)


def test_runs_of_identical_rows_in_a_view():
    """A view of A's rows 5.. (row pointer not starting at zero): the runs of
    identical rows are found from the view's own rows."""
    import torch
    ops = _ops()
    A, B = _runs_of_identical_rows(seed=52)
    dA, dB = ops.DeviceCSR.from_host(A), ops.DeviceCSR.from_host(B)
    lo, hi = 5, A.rows
    view = ops.DeviceCSR(hi - lo, A.cols, dA.rpt[lo:hi + 1], dA.col, dA.val)
    C = ops.spgemm(view, dB, config=ops.Config(validate=1))
    torch.cuda.synchronize()
    oracle.compare(*C.to_host(), oracle.spgemm(A, B, rows=np.arange(lo, hi)), tol=TOL)
