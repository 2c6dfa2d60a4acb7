"""GPU parity of the predictor kernels against the reference in oracle/mlp.py:
row features (bit-exact), network inputs (float32 log2 within 2 ulp),
inference on the matrix cores, the mean-squared-error gradient, Adam, and a
short training run through the C ABI.

Tolerances come from the float32 arithmetic of the kernels:
* forward: layer 1 and the bf16 rounding of h1 are evaluated identically on
  both sides (same float32 operations in the same order), so h1 agrees
  exactly; z2 sums 64 exact bf16 x bf16 products in float32 in an
  unspecified order and y sums 64 rounded products, so per row
  |dy| <= 2^-24 (70 sum_j |W3_j| |h2_j| + 70 sum_j |W3_j| S2_j + |y|) with
  S2_j = sum_k |W2_jk h1_k| + |b2_j|;
* gradient: every entry is a float32 sum over at most 64 rows per block of
  terms that are themselves float32 dot products of 64 terms, then a float64
  sum over blocks; the bound is a few hundred float32 units of the sum of the
  absolute terms (oracle grad with absolute=True).  Rows whose z2 lies within
  rounding of 0 (a ReLU kink, where the derivative legitimately differs) are
  left out of the batch.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import mlp

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _ops():
    import paper_2206_07244_amd as ops
    return ops


def _torch():
    import torch
    return torch


def params_bits(seed, noise=0.1):
    th = mlp.init(seed) + np.random.default_rng(seed + 100).normal(0, noise, mlp.NPARAM)
    return mlp.bf16_bits(th)


def dev_params(bits):
    torch = _torch()
    return torch.from_numpy(bits.view(np.int16).copy()).cuda()


def rand_X(n, seed):
    r = np.random.default_rng(seed)
    alen = r.integers(0, 60, n)
    nprod = alen * r.integers(1, 80, n) + r.integers(0, 3, n)
    bmax = np.minimum(r.integers(0, 80, n), nprod)
    return mlp.features(alen, nprod, bmax).astype(np.float32)


def forward_tol(th, X):
    p = mlp.unpack(th)
    y, (_, _, h1, z2, h2) = mlp.forward(th, X.astype(np.float64), quant=True)
    S2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    w3 = np.abs(p["W3"][0])
    return y, U32 * (70 * np.abs(h2) @ w3 + 70 * S2 @ w3 + np.abs(y) + np.abs(p["b3"][0])) * 2


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1037, 70001])
def test_forward_matches_reference(n):
    torch = _torch()
    ops = _ops()
    bits = params_bits(n)
    th = mlp.from_bf16_bits(bits)
    X = rand_X(n, n + 1)
    y = ops.mlp_forward(dev_params(bits), torch.from_numpy(X).cuda()).cpu().numpy()
    ref, tol = forward_tol(th, X)
    err = np.abs(y.astype(np.float64) - ref)
    assert np.all(err <= tol), (np.max(err / tol), n)


def test_forward_closed_form_network():
    """Pass-through network: y = x0 + 2 x1 + 3 x2 + 0.5 exactly for inputs
    that are bf16 values (every intermediate is exact)."""
    torch = _torch()
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W1"][0, 0] = p["W1"][1, 1] = p["W1"][2, 2] = 1.0
    p["W2"][0, 0] = p["W2"][1, 1] = p["W2"][2, 2] = 1.0
    p["W3"][0, :3] = [1.0, 2.0, 3.0]
    p["b3"][0] = 0.5
    bits = mlp.bf16_bits(mlp.pack(p))
    X = np.array([[0, 0, 0], [1, 2, 3], [0.5, 0.25, 4], [10, 11.5, 7]] * 9, np.float32)
    y = _ops().mlp_forward(dev_params(bits), torch.from_numpy(X).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y, X.astype(np.float64) @ [1, 2, 3] + 0.5)


def kink_free(th, X, rel=1e-3):
    p = mlp.unpack(th)
    _, (_, _, h1, z2, _) = mlp.forward(th, X.astype(np.float64), quant=True)
    S2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    return np.all(np.abs(z2) > rel * S2 + 1e-30, axis=1)


@pytest.mark.parametrize("n,seed", [(1, 5), (64, 6), (100, 7), (2000, 8), (20000, 9)])
@pytest.mark.parametrize("tau", [0.0, 0.9])
def test_gradient_matches_reference(n, seed, tau):
    torch = _torch()
    ops = _ops()
    bits = params_bits(seed)
    th = mlp.from_bf16_bits(bits)
    X = rand_X(4 * n + 20, seed)
    X = X[kink_free(th, X)][:n]
    assert X.shape[0] == n
    y0, _ = mlp.forward(th, X.astype(np.float64))
    r = np.random.default_rng(seed)
    t = (y0 + np.where(r.random(n) < 0.5, -1, 1) * (0.5 + r.random(n))).astype(np.float32)
    g, loss = ops.mlp_grad(dev_params(bits), torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(),
                           tau=tau)
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu().numpy()[0])
    tr = None if tau == 0.0 else float(np.float32(tau))
    lref, gref = mlp.grad(th, X.astype(np.float64), t.astype(np.float64), tau=tr)
    _, gabs = mlp.grad(th, X.astype(np.float64), t.astype(np.float64), absolute=True, tau=tr)
    tol = 400 * U32 * gabs + 1e-12 * np.max(gabs)
    bad = np.abs(g - gref) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:10], np.max(np.abs(g - gref) / (gabs + 1e-300)))
    assert abs(loss - lref) <= 1e-5 * lref


@pytest.mark.parametrize("step", [1, 2, 10, 1000])
def test_adam_matches_reference(step):
    """Moments within a few float32 roundings of the magnitude of their two
    terms (they may cancel); the parameter update, recomputed in float64 from
    the kernel's own moments, within a few roundings of the update and of the
    parameter."""
    torch = _torch()
    ops = _ops()
    r = np.random.default_rng(step)
    P = ops.MLP_NPARAM
    master = r.normal(0, 0.3, P).astype(np.float32)
    m = (r.normal(0, 0.01, P) * (step > 1)).astype(np.float32)
    v = (np.abs(r.normal(0, 1e-4, P)) * (step > 1)).astype(np.float32)
    g = r.normal(0, 0.05, P).astype(np.float32)
    dm, dmm, dv, dg = (torch.from_numpy(a.copy()).cuda() for a in (master, m, v, g))
    pb = torch.zeros(P, dtype=torch.int16, device="cuda")
    ops.mlp_adam(dm, dmm, dv, dg, step, pb, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    # the kernel's hyper-parameters are float32 values: the reference uses
    # exactly those (1 - float32(0.999) differs from 0.001 by 1.3e-5 relative)
    f = lambda x: float(np.float32(x))
    lr, b1, b2, eps = f(2e-3), f(0.9), f(0.999), f(1e-8)
    M0, V0, G, W0 = (a.astype(np.float64) for a in (m, v, g, master))
    th, m2, v2 = mlp.adam_step(W0, M0, V0, G, step, lr=lr, b1=b1, b2=b2, eps=eps)
    gm = dmm.cpu().numpy().astype(np.float64)
    gv = dv.cpu().numpy().astype(np.float64)
    got = dm.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gm - m2) <= 4 * U32 * (b1 * np.abs(M0) + (1 - b1) * np.abs(G)))
    assert np.all(np.abs(gv - v2) <= 5 * U32 * (b2 * V0 + (1 - b2) * G * G))
    # the update from the kernel's moments
    c1 = 1.0 / (1.0 - b1 ** step)
    c2 = 1.0 / (1.0 - b2 ** step)
    upd = lr * (gm * c1) / (np.sqrt(gv * c2) + eps)
    assert np.all(np.abs(got - (W0 - upd)) <= 10 * U32 * np.abs(upd) + U32 * np.abs(W0))
    # and it is the reference step up to the moments' rounding
    assert np.max(np.abs(got - th)) <= 1e-3 * lr
    # the bf16 copy is the kernel's own float32 master rounded to nearest even
    np.testing.assert_array_equal(pb.cpu().numpy().view(np.uint16), mlp.bf16_bits(got))


@pytest.mark.parametrize("case", ["rmat12", "st27_12", "rect", "empty_rows"])
def test_row_features_bit_exact(case):
    torch = _torch()
    ops = _ops()
    if case == "rmat12":
        A = B = syn.rmat(12, 8, seed=3)
    elif case == "st27_12":
        A = B = syn.stencil27(12, seed=1)
    elif case == "rect":
        A = syn.poisson_uniform(3001, 2000, 5.0, seed=4)
        B = syn.poisson_uniform(2000, 700, 3.0, seed=5)
    else:
        A = syn.random_csr(500, 300, 0.01, seed=6)
        B = syn.random_csr(300, 200, 0.05, seed=7)
    dA = ops.DeviceCSR.from_host(A)
    dB = dA if B is A else ops.DeviceCSR.from_host(B)
    al, npd, bm = ops.row_features(dA, dB)
    X = ops.mlp_features(dA, dB).cpu().numpy()
    nprod, alen, bmax, _ = oracle.row_stats(A, B)
    np.testing.assert_array_equal(al.cpu().numpy(), alen)
    np.testing.assert_array_equal(npd.cpu().numpy(), nprod)
    np.testing.assert_array_equal(bm.cpu().numpy(), bmax)
    ref = mlp.features(alen, nprod, bmax)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(X.astype(np.float64) - ref) <= 2 * ulp + 1e-30)


def test_training_reduces_loss():
    """200 Adam steps of the GPU kernels on a fixed batch of labelled rows."""
    torch = _torch()
    ops = _ops()
    A = syn.rmat(12, 8, seed=11)
    B = A
    nprod, alen, bmax, _ = oracle.row_stats(A, B)
    nnz = oracle.symbolic(A, B)
    X = torch.from_numpy(mlp.features(alen, nprod, bmax).astype(np.float32)).cuda()
    T = torch.from_numpy(mlp.target(nnz).astype(np.float32)).cuda()
    th = mlp.init(1)
    master = torch.from_numpy(th.astype(np.float32)).cuda()
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    P = dev_params(mlp.bf16_bits(th))
    _, l0 = ops.mlp_grad(P, X, T)
    l0 = float(l0.cpu()[0])
    for step in range(1, 201):
        g, _ = ops.mlp_grad(P, X, T)
        ops.mlp_adam(master, m, v, g, step, P, lr=3e-3)
    _, l1 = ops.mlp_grad(P, X, T)
    l1 = float(l1.cpu()[0])
    assert l1 < 0.05 * l0, (l0, l1)
    # the trained network's forward pass agrees with the reference at the same weights
    bits = P.cpu().numpy().view(np.uint16)
    y = ops.mlp_forward(P, X).cpu().numpy()
    ref, tol = forward_tol(mlp.from_bf16_bits(bits), X.cpu().numpy())
    assert np.all(np.abs(y - ref) <= tol)
