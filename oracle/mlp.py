"""Reference of the per-row output-size predictor (TEST INFRASTRUCTURE ONLY).

Used by the tests and by the checks of the training driver, never by the
library path.  Plain numpy, written from the definition of a multilayer
perceptron, mean squared error and Adam; it shares no code with the HIP
kernels.  The predictor is an extension on top of OpSparse: the paper's
one-phase alternative (Section 2.2) needs an output-size bound per row, and
the network supplies one.

Model: three weight layers with ReLU between them,
    z1 = W1 x + b1,   h1 = bf16(relu(z1))      W1: 64 x 3
    z2 = W2 h1 + b2,  h2 = relu(z2)            W2: 64 x 64
    y  = W3 h2 + b3                            W3: 1 x 64
on the features x = log2(1 + (a_len, n_prod, b_max)) of a row of C = A*B
(a_len: entries of A's row; n_prod: its intermediate products; b_max: the
longest B row it references), predicting y = log2(1 + nnz) of the row.
Parameters are bfloat16 values packed in the order W1, b1, W2, b2, W3, b3
(row-major).

Precision.  The hidden layer h1 is the bfloat16 input of the second layer
(a bf16 x bf16 product with fp32 accumulation), so the rounding of z1 to
bfloat16 is a quantisation decided in floating point.  Both sides take that
decision in the kernel's precision: z1 is evaluated in float32 in the fixed
order ((b1 + w0*x0) + w1*x1) + w2*x2, every product and sum rounded to
float32 (no fused multiply-add), then rounded to bfloat16 (nearest, ties to
even).  Everything after h1 is float64 here (float32 accumulation on the
GPU).  `quant=False` evaluates the plain float64 network instead (used for
the finite-difference checks, where the quantisation would make the loss
piecewise constant in W1 and b1).

Backward pass: mean squared error (or the pinball loss of a quantile level
tau, which makes the network predict an upper quantile of the row size) over
a batch of B rows, gradients by the chain rule with the bf16 rounding of h1
passed straight through (its derivative taken as 1).  `absolute=True` evaluates the same formulas on the
absolute values of every factor, which bounds the magnitude of the terms
summed into each gradient entry (the scale for rounding-error tolerances).
"""
from __future__ import annotations

import numpy as np

IN, H = 3, 64
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], np.float64).ravel() for n, _ in SHAPES])


def init(seed: int = 0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, in float64."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) after conversion to float32;
    the result is returned as float64.  NaN is not expected here."""
    f = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    r = ((f + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """uint16 bit patterns of round_bf16(x)."""
    return (np.asarray(round_bf16(x), np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def features(alen, nprod, bmax) -> np.ndarray:
    """x = log2(1 + v) per feature, float64, shape [rows, 3]."""
    v = np.stack([np.asarray(alen, np.float64), np.asarray(nprod, np.float64),
                  np.asarray(bmax, np.float64)], axis=1)
    return np.log2(1.0 + v)


def target(nnz) -> np.ndarray:
    return np.log2(1.0 + np.asarray(nnz, np.float64))


def layer1(W1, b1, X, quant=True):
    """(z1, h1) of the first layer for inputs X [B, 3]."""
    if not quant:
        z = np.asarray(X, np.float64) @ W1.T + b1
        return z, np.maximum(z, 0.0)
    x = np.asarray(X, np.float32)
    w = np.asarray(W1, np.float32)
    b = np.asarray(b1, np.float32)
    z = b[None, :] + w[None, :, 0] * x[:, 0:1]
    z = z + w[None, :, 1] * x[:, 1:2]
    z = z + w[None, :, 2] * x[:, 2:3]
    assert z.dtype == np.float32
    return z.astype(np.float64), round_bf16(np.maximum(z, np.float32(0.0)))


def forward(theta: np.ndarray, X: np.ndarray, quant: bool = True):
    """Predictions y [B] and the intermediate values (X, z1, h1, z2, h2)."""
    p = unpack(theta)
    z1, h1 = layer1(p["W1"], p["b1"], X, quant)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, (np.asarray(X, np.float64), z1, h1, z2, h2)


def pointwise_loss(y, t, tau=None):
    """Squared error (tau None), or the pinball (quantile) loss of level tau
    on r = t - y: tau * r for r > 0, (tau - 1) * r otherwise."""
    r = np.asarray(t, np.float64) - np.asarray(y, np.float64)
    if tau is None:
        return r * r
    return np.where(r > 0, tau * r, (tau - 1.0) * r)


def loss(theta: np.ndarray, X: np.ndarray, t: np.ndarray, quant: bool = True, tau=None) -> float:
    y, _ = forward(theta, X, quant)
    return float(np.mean(pointwise_loss(y, t, tau)))


def grad(theta: np.ndarray, X: np.ndarray, t: np.ndarray, quant: bool = True,
         absolute: bool = False, tau=None):
    """(loss, dloss/dtheta) of the mean squared error (tau None) or of the
    mean pinball loss of level tau over the batch.  The pinball loss has
    derivative -tau / B for t > y and (1 - tau) / B otherwise."""
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X, quant)
    B = X.shape[0]
    t = np.asarray(t, np.float64)
    if tau is None:
        dy = 2.0 * (y - t) / B
    else:
        dy = np.where(t - y > 0, -tau, 1.0 - tau) / B
    W2, W3 = p["W2"], p["W3"]
    if absolute:
        dy, W2, W3, X, h1, h2 = (np.abs(a) for a in (dy, W2, W3, X, h1, h2))
    g = {}
    g["W3"] = dy[None, :] @ h2
    g["b3"] = np.array([dy.sum()])
    dz2 = (dy[:, None] * W3) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean(pointwise_loss(y, t, tau))), pack(g)


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1); `step` counts from 1.
    Returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


CAL_SPAN_MAX = 8 << 20     # widest column range a sampled row may have
CAL_OCT_PRODUCTS = 1 << 24 # products sampled per octave (about)
CAL_MIN_ROWS = 4           # sampled rows an octave needs to be scaled
CAL_MAX_OCT = 20           # rows of larger octaves (n_prod >= 2^21) are not sampled


def row_ranges(A, B):
    """(lo, hi) column range of every row of A*B: the smallest first and the
    largest last column of the B rows it references (lo > hi when the row
    has no products)."""
    blen = np.diff(B.rpt)
    bcol = np.asarray(B.col, np.int64)
    if bcol.size == 0:
        bcol = np.zeros(1, np.int64)
    first = np.where(blen > 0, bcol[np.minimum(B.rpt[:-1], bcol.size - 1)], np.iinfo(np.int64).max)
    last = np.where(blen > 0, bcol[np.maximum(B.rpt[1:] - 1, 0)], -1)
    lo = np.full(A.rows, np.iinfo(np.int64).max)
    hi = np.full(A.rows, -1)
    rows = np.repeat(np.arange(A.rows), np.diff(A.rpt))
    if rows.size:
        np.minimum.at(lo, rows, first[A.col])
        np.maximum.at(hi, rows, last[A.col])
    return lo, hi


def fmix64(x: np.ndarray) -> np.ndarray:
    """MurmurHash3's 64-bit finalizer (A. Appleby, MurmurHash3, public
    domain): xor-shift 33, multiply by 0xff51afd7ed558ccd, xor-shift 33,
    multiply by 0xc4ceb9fe1a85ec53, xor-shift 33, all modulo 2^64."""
    k = np.asarray(x, np.uint64).copy()
    with np.errstate(over="ignore"):
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xFF51AFD7ED558CCD)
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xC4CEB9FE1A85EC53)
        k ^= k >> np.uint64(33)
    return k


def calibration_pick(alen, nprod, span, per_octave=64):
    """Rows counted exactly for the calibration, by a rule both sides apply
    in integer arithmetic.  Eligible rows have a_len >= 2,
    1 <= n_prod < 2^(CAL_MAX_OCT + 1) and a column range of at most
    CAL_SPAN_MAX columns; they are grouped by octave o = floor(log2 n_prod).
    An octave with c eligible rows has the quota
    K = min(c, clamp(CAL_OCT_PRODUCTS >> o, CAL_MIN_ROWS, per_octave)); each
    of its rows is picked with probability K / c, by the draw
    u(i) * c < K * 2^32 with u(i) the high 32 bits of fmix64(i), so an
    octave yields K rows on average and every row when c <= K.
    Returns the picked rows (ascending) and every row's octave."""
    alen, nprod, span = (np.asarray(a, np.int64) for a in (alen, nprod, span))
    M = nprod.size
    octave = np.where(nprod >= 1, np.floor(np.log2(np.maximum(nprod, 1))).astype(np.int64), -1)
    elig = (alen >= 2) & (nprod >= 1) & (octave <= CAL_MAX_OCT) & (span <= CAL_SPAN_MAX)
    picked = np.zeros(M, bool)
    u = fmix64(np.arange(M, dtype=np.uint64)) >> np.uint64(32)    # < 2^32
    for o in np.unique(octave[elig]):
        sel = elig & (octave == o)
        c = int(sel.sum())
        k = min(c, min(max(CAL_OCT_PRODUCTS >> int(o), CAL_MIN_ROWS), per_octave))
        # u * c < 2^63 and K * 2^32 < 2^39: exact in uint64
        picked |= sel & (u * np.uint64(c) < np.uint64(k << 32))
    return np.nonzero(picked)[0], octave


def calibration(pred_log2, nnz_exact, alen, nprod, bmax, ncols, span, per_octave=64):
    """Per-octave scales of the network's estimates from the rows of
    calibration_pick, counted exactly by nnz_exact(rows).  An octave with at
    least CAL_MIN_ROWS picked rows gets the scale max(size / estimate) over
    them (the estimate 2^pred - 1 clamped to [min(b_max, U), U],
    U = min(n_prod, N), at least 1 for a row with products), so that most of
    the octave's rows fit even when its rows are biased differently; every
    row of that octave (n_prod >= 1) is scaled by it, other rows keep 1.
    Returns (scale of every row, overall ratio sum(sizes) / sum(estimates)
    over all picked rows (1 when none), picked rows)."""
    alen, nprod, bmax = (np.asarray(a, np.int64) for a in (alen, nprod, bmax))
    scale = np.ones(nprod.size)
    rows, octave = calibration_pick(alen, nprod, span, per_octave)
    if rows.size == 0:
        return scale, 1.0, rows
    hi = np.minimum(nprod[rows], ncols).astype(np.float64)
    lo = np.minimum(bmax[rows], hi).astype(np.float64)
    est = np.clip(np.exp2(np.asarray(pred_log2, np.float64)[rows]) - 1.0, lo, hi)
    ex = np.asarray(nnz_exact(rows), np.float64)
    o_rows = octave[rows]
    for o in np.unique(o_rows):
        sel = o_rows == o
        if sel.sum() >= CAL_MIN_ROWS:
            scale[(octave == o) & (nprod >= 1)] = np.max(ex[sel] / est[sel])
    overall = float(ex.sum() / est.sum()) if est.sum() > 0 else 1.0
    return scale, overall, rows


def capacity(pred_log2, margin, alen, nprod, bmax, ncols, scale=1.0) -> np.ndarray:
    """Slot capacity of each row from a prediction of log2(1 + nnz):
    ceil((2^pred - 1) * scale * (1 + margin)) (scale a number or one per
    row) clamped to
    [b_max, min(n_prod, ncols)], since a row of C holds at least its longest
    referenced B row and at most min(n_prod, N) entries; a row with at most
    one A entry has exactly n_prod entries.  Evaluated in float64."""
    est = np.ceil((np.exp2(np.asarray(pred_log2, np.float64)) - 1.0) * np.asarray(scale, np.float64)
                  * (1.0 + margin))
    nprod = np.asarray(nprod, np.int64)
    hi = np.minimum(nprod, ncols)
    lo = np.minimum(np.asarray(bmax, np.int64), hi)
    est = np.where(np.isfinite(est), est, hi)
    cap = np.clip(est, lo, hi).astype(np.int64)
    return np.where(np.asarray(alen) <= 1, nprod, cap)
