"""Pins for the CPU oracle: each checks it against something other than
itself (closed forms, the inner-product definition, dense and library
products, algebraic identities, invariants, the paper's printed tables)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synthetic as syn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scipy(A):
    return sp.csr_matrix((A.val, A.col, A.rpt), shape=(A.rows, A.cols))


def _pattern(A):
    return sp.csr_matrix((np.ones(A.nnz, np.int64), A.col, A.rpt), shape=(A.rows, A.cols))


def _csr_of(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return syn.CSR(M.shape[0], M.shape[1], M.indptr.astype(np.int64),
                   M.indices.astype(np.int32), M.data.astype(np.float64))


def _rows_of(rpt):
    return np.repeat(np.arange(len(rpt) - 1), np.diff(rpt))


# --------------------------------------------------------------------------
# Definition (Eq. 1): inner products on tiny inputs, pure Python
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_inner_product_definition_tiny(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    m, k, n = (int(x) for x in rng.integers(0, 9, 3))
    A = syn.random_csr(m, k, float(rng.uniform(0, 0.7)), seed=seed)
    B = syn.random_csr(k, n, float(rng.uniform(0, 0.7)), seed=seed + 100)
    Ad = {(i, int(A.col[p])): A.val[p] for i in range(m) for p in range(A.rpt[i], A.rpt[i + 1])}
    Bd = {(i, int(B.col[p])): B.val[p] for i in range(k) for p in range(B.rpt[i], B.rpt[i + 1])}
    rpt, col, val, S = oracle_lib.spgemm(A, B)
    got = {}
    for i in range(m):
        for p in range(rpt[i], rpt[i + 1]):
            got[(i, int(col[p]))] = (val[p], S[p])
    want = {}
    for i in range(m):
        for j in range(n):
            terms = [Ad[(i, kk)] * Bd[(kk, j)] for kk in range(k)
                     if (i, kk) in Ad and (kk, j) in Bd]
            if terms:
                s = 0.0
                for t in terms:          # ascending k, as the row-wise sum visits them
                    s += t
                want[(i, j)] = (s, sum(abs(t) for t in terms))
    assert got.keys() == want.keys()
    for key in want:
        assert got[key][0] == want[key][0]
        assert got[key][1] == pytest.approx(want[key][1], rel=1e-15)
    # columns ascending inside rows
    for i in range(m):
        assert np.all(np.diff(col[rpt[i]:rpt[i + 1]]) > 0)


# --------------------------------------------------------------------------
# Dense products (library matmul) with structure from pattern counts
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,dens", [((48, 40, 44), 0.0), ((48, 40, 44), 0.05),
                                        ((33, 47, 29), 0.3), ((40, 40, 40), 0.6),
                                        ((1, 48, 7), 0.4), ((17, 1, 23), 0.5)])
def test_against_dense(oracle_lib, shape, dens):
    m, k, n = shape
    for vals, exact in (("int", True), ("uniform", False)):
        A = syn.random_csr(m, k, dens, seed=m * 7 + k, values=vals)
        B = syn.random_csr(k, n, dens, seed=n * 11 + k, values=vals)
        Ad, Bd = syn.to_dense(A), syn.to_dense(B)
        cnt = (Ad != 0).astype(np.int64) @ (Bd != 0).astype(np.int64)
        rpt, col, val, S = oracle_lib.spgemm(A, B)
        r = _rows_of(rpt)
        mask = np.zeros((m, n), bool)
        mask[r, col] = True
        assert np.array_equal(mask, cnt > 0)            # structural product
        D = Ad @ Bd
        Sd = np.abs(Ad) @ np.abs(Bd)
        if exact:
            assert np.array_equal(val, D[r, col])
        else:
            assert np.all(np.abs(val - D[r, col]) <= 1e-13 * Sd[r, col] + 1e-300)
        assert np.allclose(S, Sd[r, col], rtol=1e-14, atol=0)


def test_explicit_zero_is_kept(oracle_lib):
    A = syn.CSR(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    B = syn.CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([1.0, -1.0]))
    rpt, col, val, S = oracle_lib.spgemm(A, B)
    assert list(rpt) == [0, 1] and list(col) == [0] and val[0] == 0.0 and S[0] == 2.0


def test_empty_shapes(oracle_lib):
    for m, k, n in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (0, 0, 0), (3, 4, 5)]:
        A = syn.random_csr(m, k, 0.0 if (m, k, n) == (3, 4, 5) else 0.5, seed=1)
        B = syn.random_csr(k, n, 0.5, seed=2)
        rpt, col, val, S = oracle_lib.spgemm(A, B)
        assert rpt.shape == (m + 1,) and rpt[-1] == 0 and col.size == 0


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def _lap5_square_closed(g):
    """13-point stencil of the squared 5-point Laplacian, from grid geometry."""
    n = g * g
    ent = {}
    for y in range(g):
        for x in range(g):
            p = y * g + x
            deg = (x > 0) + (x < g - 1) + (y > 0) + (y < g - 1)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    if abs(dx) + abs(dy) > 2:
                        continue
                    xx, yy = x + dx, y + dy
                    if not (0 <= xx < g and 0 <= yy < g):
                        continue
                    if dx == 0 and dy == 0:
                        v = 16.0 + deg
                    elif abs(dx) + abs(dy) == 1:
                        v = -8.0
                    elif abs(dx) == 2 or abs(dy) == 2:
                        v = 1.0
                    else:
                        v = 2.0
                    ent[(p, yy * g + xx)] = v
    return n, ent


@pytest.mark.parametrize("g", [1, 2, 3, 8, 17])
def test_lap5_square_closed_form_entries(oracle_lib, g):
    A = syn.lap5(g)
    n, ent = _lap5_square_closed(g)
    rpt, col, val, S = oracle_lib.spgemm(A, A)
    got = {(int(i), int(j)): v for i, j, v in zip(_rows_of(rpt), col, val)}
    assert got == ent


def test_lap5_64_counts(oracle_lib):
    g = 64
    A = syn.lap5(g)
    nprod, _, _, tot = oracle_lib.row_stats(A, A)
    assert tot == 4 * 9 + 4 * (g - 2) * 16 + (g - 2) ** 2 * 25 == 100104
    rpt, col, val, S = oracle_lib.spgemm(A, A)
    assert rpt[-1] == 13 * g * g - 20 * g + 4 == 51972
    assert set(np.unique(val).tolist()) == {-8.0, 1.0, 2.0, 18.0, 19.0, 20.0}


@pytest.mark.parametrize("g", [3, 4, 9])
def test_stencil27_square_closed_form(oracle_lib, g):
    A = syn.stencil27(g, seed=5)
    nnzA = (3 * g - 2) ** 3
    assert A.nnz == nnzA
    nprod, _, _, tot = oracle_lib.row_stats(A, A)
    nnz = oracle_lib.symbolic(A, A)
    if g >= 4:
        assert nnz.sum() == (5 * g - 6) ** 3
    assert tot == (9 * g - 10) ** 3
    # per-row: separable box counts
    f = np.array([min(x, 2) + min(g - 1 - x, 2) + 1 for x in range(g)])
    h = np.array([min(x, 1) + min(g - 1 - x, 1) + 1 for x in range(g)])
    hn = np.array([sum(h[xx] for xx in range(max(0, x - 1), min(g, x + 2))) for x in range(g)])
    idx = np.arange(g ** 3)
    x, y, z = idx % g, (idx // g) % g, idx // (g * g)
    assert np.array_equal(nnz, f[x] * f[y] * f[z])
    assert np.array_equal(nprod, hn[x] * hn[y] * hn[z])


@pytest.mark.parametrize("g", [2, 3, 4, 7])
def test_block_stencil27_square_closed_form(oracle_lib, g):
    """27-point stencil with dense 3x3 node blocks (the high compression-ratio
    finite-element class): nnz(A) = 9 (3g-2)^3, n_prod = 27 (9g-10)^3 and
    nnz(C) = 9 (5g-6)^3, and per scalar row 3x the node-level output count
    and 9x the node-level product count of the 27-point stencil."""
    d = 3
    A = syn.block_stencil27(g, d, seed=g)
    A.check()
    assert A.rows == d * g ** 3 and A.nnz == 9 * (3 * g - 2) ** 3
    nprod, _, _, tot = oracle_lib.row_stats(A, A)
    nnz = oracle_lib.symbolic(A, A)
    assert tot == 27 * (9 * g - 10) ** 3
    if g >= 4:
        assert nnz.sum() == 9 * (5 * g - 6) ** 3
    f = np.array([min(x, 2) + min(g - 1 - x, 2) + 1 for x in range(g)])
    h = np.array([min(x, 1) + min(g - 1 - x, 1) + 1 for x in range(g)])
    hn = np.array([sum(h[xx] for xx in range(max(0, x - 1), min(g, x + 2))) for x in range(g)])
    node = np.arange(g ** 3).repeat(d)
    x, y, z = node % g, (node // g) % g, node // (g * g)
    assert np.array_equal(nnz, d * f[x] * f[y] * f[z])
    assert np.array_equal(nprod, d * d * hn[x] * hn[y] * hn[z])


def test_block_stencil27_against_dense(oracle_lib):
    A = syn.block_stencil27(2, 3, seed=11)
    D = syn.to_dense(A)
    rpt, col, val, S = oracle_lib.spgemm(A, A)
    r = _rows_of(rpt)
    P = D @ D
    Sd = np.abs(D) @ np.abs(D)
    cnt = (D != 0).astype(np.int64) @ (D != 0).astype(np.int64)
    mask = np.zeros_like(cnt, dtype=bool)
    mask[r, col] = True
    assert np.array_equal(mask, cnt > 0)
    assert np.all(np.abs(val - P[r, col]) <= 1e-13 * Sd[r, col])


# --------------------------------------------------------------------------
# Identities
# --------------------------------------------------------------------------

def test_identity_both_sides(oracle_lib):
    A = syn.random_csr(37, 23, 0.2, seed=9)
    for L, R in ((A, syn.identity(23)), (syn.identity(37), A)):
        rpt, col, val, S = oracle_lib.spgemm(L, R)
        assert np.array_equal(rpt, A.rpt) and np.array_equal(col, A.col)
        assert np.array_equal(val.view(np.int64), A.val.view(np.int64))


@pytest.mark.parametrize("seed", [0, 1])
def test_transpose_identity_bit_exact(oracle_lib, seed):
    A = syn.random_csr(30, 45, 0.15, seed=seed)
    B = syn.random_csr(45, 26, 0.2, seed=seed + 10)
    C = oracle_lib.spgemm(A, B)
    At, Bt = _csr_of(_scipy(A).T), _csr_of(_scipy(B).T)
    Ct = oracle_lib.spgemm(Bt, At)
    Cs = _csr_of(sp.csr_matrix((Ct[2], Ct[1], Ct[0]), shape=(26, 30)).T)
    assert np.array_equal(Cs.rpt, C[0]) and np.array_equal(Cs.col, C[1])
    assert np.array_equal(Cs.val.view(np.int64), C[2].view(np.int64))


def test_permutation_similarity_structure(oracle_lib):
    A = syn.rmat(9, 8, seed=3)
    perm = np.random.default_rng(0).permutation(A.rows)
    P = sp.csr_matrix((np.ones(A.rows), (np.arange(A.rows), perm)), shape=(A.rows, A.rows))
    As = _scipy(A)
    PA = _csr_of(P @ As @ P.T)
    C = oracle_lib.spgemm(A, A)
    Cp = oracle_lib.spgemm(PA, PA)
    Cs = sp.csr_matrix((np.ones_like(C[2]), C[1], C[0]), shape=(A.rows, A.rows))
    want = _csr_of(P @ Cs @ P.T)
    assert np.array_equal(want.rpt, Cp[0]) and np.array_equal(want.col, Cp[1])
    Cv = _csr_of(P @ sp.csr_matrix((C[2], C[1], C[0]), shape=(A.rows, A.rows)) @ P.T)
    # values agree within the summation-order bound (k order changes)
    Sv = _csr_of(P @ sp.csr_matrix((C[3], C[1], C[0]), shape=(A.rows, A.rows)) @ P.T)
    assert np.all(np.abs(Cv.val - Cp[2]) <= 1e-14 * Sv.val)


# --------------------------------------------------------------------------
# Library product (scipy) on a power-law graph; per-row invariants
# --------------------------------------------------------------------------

def test_rmat_against_scipy_pattern_and_invariants(oracle_lib):
    A = syn.rmat(11, 16, seed=7)
    P = _pattern(A)
    cnt = (P @ P).tocsr()
    cnt.sort_indices()
    rpt, col, val, S = oracle_lib.spgemm(A, A)
    assert np.array_equal(rpt, cnt.indptr) and np.array_equal(col, cnt.indices)
    nprod, alen, bmax, tot = oracle_lib.row_stats(A, A)
    assert tot == cnt.data.sum()
    assert np.array_equal(nprod, np.asarray(cnt.sum(axis=1)).ravel())
    nnz = np.diff(rpt)
    assert np.all(bmax <= nnz) and np.all(nnz <= np.minimum(nprod, A.cols))
    assert np.all(nnz[alen <= 1] == nprod[alen <= 1])
    colcount = np.bincount(A.col, minlength=A.cols)
    assert tot == int((colcount * np.diff(A.rpt)).sum())
    # positive values: S equals |c|
    assert np.allclose(S, np.abs(val), rtol=1e-15, atol=0)
    ref = (_scipy(A) @ _scipy(A)).tocsr()
    ref.sort_indices()
    assert np.allclose(val, ref.data, rtol=1e-14, atol=0)


def test_sampled_rows_match_full(oracle_lib):
    A = syn.banded(3000, 20, 6, seed=4)
    full = oracle_lib.spgemm(A, A)
    rows = np.array([0, 5, 2999, 1234, 5], np.int64)
    part = oracle_lib.spgemm(A, A, rows=rows)
    for r_i, r in enumerate(rows):
        a, b = full[0][r], full[0][r + 1]
        c, d = part[0][r_i], part[0][r_i + 1]
        assert np.array_equal(full[1][a:b], part[1][c:d])
        assert np.array_equal(full[2][a:b], part[2][c:d])


# --------------------------------------------------------------------------
# Binning: membership rule and the paper's printed range tables
# --------------------------------------------------------------------------

def test_bin_membership_rule(oracle_lib):
    up = [26, 426, 853]
    v = np.array([0, 26, 27, 426, 427, 853, 854, 10 ** 9])
    assert list(oracle_lib.bin_of(v, up)) == [0, 0, 1, 1, 2, 2, 3, 3]


def test_paper_range_tables(oracle_lib):
    with open(os.path.join(GOLDEN, "paper_binning_ranges.json")) as f:
        g = json.load(f)
    odd = g["printed_inconsistencies"]
    for step, sizes in (("symbolic", g["symbolic_table_sizes"]), ("numeric", g["numeric_table_sizes"])):
        for ratio, printed in g[step].items():
            derived = oracle_lib.bin_ranges(sizes, ratio, numeric=(step == "numeric"))
            for j, (d, p) in enumerate(zip(derived, printed)):
                if f"{step}/{ratio}/{j}" in odd:
                    assert d != p
                else:
                    assert d == p, (step, ratio, j)


# --------------------------------------------------------------------------
# Row-parallel form: the same per-row code on several threads
# --------------------------------------------------------------------------

@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threads_bit_identical(oracle_lib, threads):
    """Rows are independent (Section 2.1): the threaded oracle returns the
    single-threaded result bit for bit, for all rows and for a row list."""
    import synthetic as syn
    A = syn.rmat(12, 8, seed=5)
    one = oracle_lib.spgemm(A, A)
    many = oracle_lib.spgemm(A, A, threads=threads)
    for x, y in zip(one, many):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
    rows = np.random.default_rng(threads).choice(A.rows, 700, replace=False)
    one = oracle_lib.spgemm(A, A, rows=rows)
    many = oracle_lib.spgemm(A, A, rows=rows, threads=threads)
    for x, y in zip(one, many):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
    np.testing.assert_array_equal(oracle_lib.symbolic(A, A, threads=threads),
                                  oracle_lib.symbolic(A, A))
