"""Seeded synthetic sparse matrices in CSR form.

This module only *builds inputs*.  It holds none of the SpGEMM arithmetic:
the CPU oracle and the GPU library both consume what it returns, and neither
imports the other.

Every matrix is returned as a :class:`CSR` with

* ``rpt``  int64[rows+1]   row pointer (absolute offsets, ``rpt[0] == 0``)
* ``col``  int32[nnz]      column indices, strictly ascending inside a row
* ``val``  float64[nnz]    values, drawn in CSR order

which is the canonical (sorted, duplicate-free) CSR storage of the paper's
Section 2.1.1.  Random draws use numpy's PCG64 (``numpy.random.default_rng``),
a published generator, so every matrix is a pure function of its seed.

The workload families stand in for the paper's SuiteSparse A^2 benchmarks
(Section 6.1, matrix table): regular stencils (FEM/structured class; with
dense node blocks, the high compression-ratio FEM matrices),
R-MAT power-law graphs (webbase/wb-edu class, giant rows), random banded and
Poisson-uniform rows (low compression-ratio class).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "CSR", "lap5", "stencil27", "stencil", "rmat", "poisson_uniform",
    "banded", "random_csr", "identity", "batch_pairs", "training_set", "training_matrix",
    "WORKLOADS",
    "block_stencil27",
]


@dataclass
class CSR:
    rows: int
    cols: int
    rpt: np.ndarray   # int64[rows+1]
    col: np.ndarray   # int32[nnz]
    val: np.ndarray   # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1] - self.rpt[0])

    def check(self) -> "CSR":
        assert self.rpt.dtype == np.int64 and self.rpt.shape == (self.rows + 1,)
        assert self.col.dtype == np.int32 and self.val.dtype == np.float64
        assert self.col.shape == self.val.shape == (self.nnz,)
        assert np.all(np.diff(self.rpt) >= 0)
        if self.nnz:
            assert self.col.min() >= 0 and self.col.max() < self.cols
            # strictly ascending inside each row
            d = np.diff(self.col.astype(np.int64))
            row_start = np.zeros(self.nnz, dtype=bool)
            starts = self.rpt[:-1][np.diff(self.rpt) > 0] - self.rpt[0]
            row_start[starts] = True
            assert np.all(d[~row_start[1:]] > 0)
        return self


def _from_sorted_keys(keys: np.ndarray, rows: int, cols: int, val: np.ndarray) -> CSR:
    """keys = row*cols + col, already unique and ascending."""
    r = keys // cols
    c = (keys - r * cols).astype(np.int32)
    counts = np.bincount(r, minlength=rows).astype(np.int64)
    rpt = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rpt[1:])
    return CSR(rows, cols, rpt, c, val)


def _from_masked_offsets(n_rows: int, n_cols: int, col_table: np.ndarray,
                         mask: np.ndarray, val_table: np.ndarray) -> CSR:
    """Rows given as fixed candidate lists (already ascending per row) + mask."""
    counts = mask.sum(axis=1).astype(np.int64)
    rpt = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rpt[1:])
    col = col_table[mask].astype(np.int32)
    val = val_table[mask].astype(np.float64)
    return CSR(n_rows, n_cols, rpt, col, val)


# ---------------------------------------------------------------------------
# Stencils
# ---------------------------------------------------------------------------

def stencil(grid: Sequence[int], offsets: Sequence[Sequence[int]],
            values: str = "uniform", seed: int = 0,
            center: float = 4.0, off: float = -1.0) -> CSR:
    """Square matrix of a d-dimensional stencil on a grid, natural ordering.

    Grid point (x0, x1, ..., x_{d-1}) has index ((x_{d-1}*g_{d-2} + ...)*g_0 + x0)
    with x0 fastest.  ``offsets`` are tuples (dx0, dx1, ...).  Points whose
    neighbour falls outside the grid drop that entry (no wrap-around).
    values: "uniform" -> U[-1,1) in CSR order from ``seed``;
            "laplacian" -> ``center`` on the diagonal, ``off`` elsewhere.
    """
    grid = [int(g) for g in grid]
    d = len(grid)
    n = int(np.prod(grid))
    strides = [1]
    for g in grid[:-1]:
        strides.append(strides[-1] * g)
    offs = np.array(offsets, dtype=np.int64).reshape(-1, d)
    lin = (offs * np.array(strides, dtype=np.int64)).sum(axis=1)
    order = np.argsort(lin, kind="stable")
    offs, lin = offs[order], lin[order]
    # On grids narrower than the stencil two offsets can share a linear offset;
    # they are never both inside the grid for one row, so columns stay distinct.
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for g in grid:
        coords.append(rem % g)
        rem = rem // g
    mask = np.ones((n, len(lin)), dtype=bool)
    for j in range(len(lin)):
        for dim in range(d):
            c = coords[dim] + offs[j, dim]
            mask[:, j] &= (c >= 0) & (c < grid[dim])
    col_table = idx[:, None] + lin[None, :]
    if values == "laplacian":
        vt = np.where(lin == 0, center, off)[None, :].repeat(n, axis=0)
        return _from_masked_offsets(n, n, col_table, mask, vt)
    A = _from_masked_offsets(n, n, col_table, mask, np.zeros((n, len(lin))))
    rng = np.random.default_rng(seed)
    A.val = rng.random(A.nnz) * 2.0 - 1.0
    return A


def lap5(g: int) -> CSR:
    """2-D 5-point Poisson Laplacian on a g x g grid, idx = y*g + x,
    4 on the diagonal and -1 on the four axial neighbours."""
    return stencil([g, g], [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)],
                   values="laplacian", center=4.0, off=-1.0)


def stencil27(g: int, seed: int = 27) -> CSR:
    """3-D 27-point stencil on a g^3 grid, idx = (z*g + y)*g + x; every offset
    in {-1,0,1}^3 that stays in the grid; values U[-1,1) from ``seed``."""
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return stencil([g, g, g], offs, values="uniform", seed=seed)


def block_stencil27(g: int, dof: int = 3, seed: int = 40) -> CSR:
    """27-point stencil on a g^3 grid with a dense dof x dof block per node
    coupling (a finite-element-like matrix with `dof` unknowns per node):
    scalar index dof * node + component, node index (z*g + y)*g + x; node i
    couples to every in-grid node j with |x_i - x_j|, |y_i - y_j|,
    |z_i - z_j| <= 1, and row dof*i + a holds columns dof*j + b for all such
    j and every b.  Values U[-1,1) in CSR order from ``seed``."""
    node = stencil27(g, seed=0)
    n_nodes = node.rows
    nlen = np.diff(node.rpt)
    # the columns of one node row, each expanded into its dof components
    exp = (dof * node.col.astype(np.int64))[:, None] + np.arange(dof, dtype=np.int64)[None, :]
    exp = exp.reshape(-1)                                   # node rows back to back
    seg_start = dof * node.rpt[:-1]                          # where node row i starts in exp
    seg_len = dof * nlen
    # every node row repeated dof times (once per component)
    rep_start = np.repeat(seg_start, dof)
    rep_len = np.repeat(seg_len, dof)
    rpt = np.zeros(dof * n_nodes + 1, dtype=np.int64)
    np.cumsum(rep_len, out=rpt[1:])
    idx = np.repeat(rep_start - rpt[:-1], rep_len) + np.arange(rpt[-1], dtype=np.int64)
    col = exp[idx].astype(np.int32)
    rng = np.random.default_rng(seed)
    val = rng.random(col.size) * 2.0 - 1.0
    return CSR(dof * n_nodes, dof * n_nodes, rpt, col, val)


# ---------------------------------------------------------------------------
# Random graphs / rows
# ---------------------------------------------------------------------------

def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 20) -> CSR:
    """R-MAT adjacency (Chakrabarti, Zhan, Faloutsos 2004), n = 2^scale,
    edge_factor*n directed edges.  Per recursion level one u ~ U[0,1) picks the
    quadrant: top-left [0,a), top-right [a,a+b), bottom-left [a+b,a+b+c),
    bottom-right [a+b+c,1).  No noise, no vertex permutation; self-loops kept;
    duplicate edges merged before values U(0,1] are drawn in CSR order."""
    n = 1 << scale
    E = edge_factor * n
    rng = np.random.default_rng(seed)
    rows = np.zeros(E, dtype=np.int64)
    cols = np.zeros(E, dtype=np.int64)
    for lvl in range(scale):
        u = rng.random(E)
        bit = np.int64(1) << np.int64(scale - 1 - lvl)
        rows |= (u >= a + b).astype(np.int64) * bit
        cbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)
        cols |= cbit.astype(np.int64) * bit
        del u, cbit
    keys = np.unique(rows * n + cols)
    del rows, cols
    val = 1.0 - rng.random(keys.size)
    return _from_sorted_keys(keys, n, n, val)


def _distinct_rows(rng: np.random.Generator, lengths: np.ndarray, n_cols: int,
                   draw) -> np.ndarray:
    """Sorted unique keys row*n_cols+col with exactly lengths[i] distinct
    columns in row i; ``draw(rng, row_ids)`` returns one candidate column per
    requested row id.  Redraws until every row has its count."""
    rows_n = lengths.size
    need = lengths.astype(np.int64).copy()
    keys = np.empty(0, dtype=np.int64)
    while True:
        rid = np.repeat(np.arange(rows_n, dtype=np.int64), need)
        if rid.size == 0:
            break
        cand = draw(rng, rid)
        keys = np.unique(np.concatenate([keys, rid * n_cols + cand]))
        have = np.bincount(keys // n_cols, minlength=rows_n)
        need = lengths - have
        assert np.all(need >= 0)
    return keys


def poisson_uniform(n_rows: int, n_cols: int, mean: float, seed=0,
                    values: str = "normal") -> CSR:
    """Row lengths ~ Poisson(mean) (capped at n_cols); each row holds that many
    distinct columns drawn uniformly from [0, n_cols); values N(0,1) or
    U[-1,1) in CSR order."""
    rng = np.random.default_rng(seed)
    L = np.minimum(rng.poisson(mean, n_rows), n_cols).astype(np.int64)
    keys = _distinct_rows(rng, L, n_cols,
                          lambda r, rid: r.integers(0, n_cols, rid.size, dtype=np.int64))
    if values == "normal":
        val = rng.standard_normal(keys.size)
    else:
        val = rng.random(keys.size) * 2.0 - 1.0
    return _from_sorted_keys(keys, n_rows, n_cols, val)


def banded(n: int, half_bw: int = 64, per_row: int = 12, seed: int = 22) -> CSR:
    """Square random banded matrix: row i holds ``per_row`` distinct columns
    drawn uniformly without replacement from [i-half_bw, i+half_bw] ∩ [0, n);
    values U[-1,1) in CSR order."""
    rng = np.random.default_rng(seed)
    lo_all = np.maximum(np.arange(n, dtype=np.int64) - half_bw, 0)
    hi_all = np.minimum(np.arange(n, dtype=np.int64) + half_bw, n - 1)
    width = hi_all - lo_all + 1
    L = np.minimum(width, per_row)

    def draw(r, rid):
        return lo_all[rid] + (r.random(rid.size) * width[rid]).astype(np.int64)

    keys = _distinct_rows(rng, L, n, draw)
    val = rng.random(keys.size) * 2.0 - 1.0
    return _from_sorted_keys(keys, n, n, val)


def random_csr(rows: int, cols: int, density: float, seed: int = 0,
               values: str = "uniform") -> CSR:
    """Bernoulli(density) pattern; values U[-1,1), N(0,1), or small integers
    ("int": uniform in {-3..3}\\{0}, exact in any summation order)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((rows, cols)) < density
    r, c = np.nonzero(mask)
    keys = r.astype(np.int64) * max(cols, 1) + c
    n = keys.size
    if values == "normal":
        val = rng.standard_normal(n)
    elif values == "int":
        v = rng.integers(1, 4, n) * np.where(rng.random(n) < 0.5, -1, 1)
        val = v.astype(np.float64)
    else:
        val = rng.random(n) * 2.0 - 1.0
    if cols == 0:
        return CSR(rows, 0, np.zeros(rows + 1, np.int64), np.zeros(0, np.int32),
                   np.zeros(0, np.float64))
    return _from_sorted_keys(keys, rows, cols, val)


def identity(n: int) -> CSR:
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
               np.ones(n, dtype=np.float64))


def from_dense(D: np.ndarray) -> CSR:
    r, c = np.nonzero(D)
    keys = r.astype(np.int64) * D.shape[1] + c
    return _from_sorted_keys(keys, D.shape[0], D.shape[1], D[r, c].astype(np.float64))


def to_dense(A: CSR) -> np.ndarray:
    D = np.zeros((A.rows, A.cols))
    r = np.repeat(np.arange(A.rows), np.diff(A.rpt))
    D[r, A.col] = A.val
    return D


# ---------------------------------------------------------------------------
# Batched pairs and the predictor's training set
# ---------------------------------------------------------------------------

def batch_pairs(count: int = 512, seed: int = 4, n_lo: int = 1000,
                n_hi: int = 64000, mean: float = 8.0) -> List[Tuple[CSR, CSR]]:
    """``count`` independent square pairs (A_i, B_i): n_i ~ U{n_lo..n_hi},
    row lengths ~ Poisson(mean) with distinct uniform columns, values N(0,1)."""
    top = np.random.default_rng(seed)
    sizes = top.integers(n_lo, n_hi + 1, count)
    out = []
    for i, n in enumerate(sizes):
        A = poisson_uniform(int(n), int(n), mean, seed=[seed, i, 0])
        B = poisson_uniform(int(n), int(n), mean, seed=[seed, i, 1])
        out.append((A, B))
    return out


def training_matrix(j: int, seed0: int = 1000, n_lo_log2: int = 14,
                    n_hi_log2: int = 18) -> Tuple[str, CSR]:
    """Matrix j of the predictor's training set: family j mod 4 (R-MAT with
    a in [.45,.6] and degree 4..32; banded with half-bandwidth 8..128 and 4..24
    per row; Poisson-uniform rows with mean 2..16; stencils 2-D 5/9-point or
    3-D 7/27-point), n = 2^k with k uniform in [n_lo_log2, n_hi_log2], all
    drawn from seed seed0 + j."""
    s = seed0 + j
    r = np.random.default_rng([s, 7])
    fam = j % 4
    logn = int(r.integers(n_lo_log2, n_hi_log2 + 1))
    n = 1 << logn
    if fam == 0:
        a = float(r.uniform(0.45, 0.6))
        bb = (1.0 - a) * float(r.uniform(0.3, 0.4))
        deg = int(r.integers(4, 33))
        return f"rmat{logn}_a{a:.2f}_d{deg}", rmat(logn, deg, a, bb, bb, seed=s)
    if fam == 1:
        hb = int(r.integers(8, 129))
        pr = int(r.integers(4, 25))
        return f"band{logn}_h{hb}_k{pr}", banded(n, hb, min(pr, 2 * hb + 1), seed=s)
    if fam == 2:
        mean = float(r.uniform(2, 16))
        return f"poisson{logn}_m{mean:.1f}", poisson_uniform(n, n, mean, seed=s, values="uniform")
    kind = int(r.integers(0, 4))
    if kind == 0:
        g = int(round(n ** 0.5))
        return f"st5_{g}", stencil([g, g], [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)], seed=s)
    if kind == 1:
        g = int(round(n ** 0.5))
        offs = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        return f"st9_{g}", stencil([g, g], offs, seed=s)
    if kind == 2:
        g = int(round(n ** (1 / 3)))
        offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        return f"st7_{g}", stencil([g, g, g], offs, seed=s)
    g = int(round(n ** (1 / 3)))
    return f"st27_{g}", stencil27(g, seed=s)


def training_set(count: int = 200, seed0: int = 1000, n_lo_log2: int = 14,
                 n_hi_log2: int = 18) -> List[Tuple[str, CSR]]:
    """The first `count` matrices of the predictor's training set
    (see training_matrix)."""
    return [training_matrix(j, seed0, n_lo_log2, n_hi_log2) for j in range(count)]


# Named workloads: (description, builder).  Sizes are the full benchmark sizes.
WORKLOADS = {
    "lap5_64": ("2-D 5-point Laplacian 64x64, C = A^2", lambda: lap5(64)),
    "st27_100": ("3-D 27-point stencil 100^3, U[-1,1) seed 27, C = A^2",
                 lambda: stencil27(100, seed=27)),
    "rmat20": ("R-MAT scale 20, degree 16, (.57,.19,.19,.05), U(0,1] seed 20, C = A^2",
               lambda: rmat(20, 16, 0.57, 0.19, 0.19, seed=20)),
    "rmat21": ("R-MAT scale 21, degree 16, (.57,.19,.19,.05), seed 21, C = A^2",
               lambda: rmat(21, 16, 0.57, 0.19, 0.19, seed=21)),
    "band21": ("random banded n=2^21, half-bandwidth 64, 12 per row, seed 22, C = A^2",
               lambda: banded(1 << 21, 64, 12, seed=22)),
    "bst27_40": ("3-D 27-point stencil 40^3 with dense 3x3 node blocks (3 unknowns per node, "
                 "compression ratio 17.6), U[-1,1) seed 40, C = A^2",
                 lambda: block_stencil27(40, 3, seed=40)),
}
