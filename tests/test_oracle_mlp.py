"""Pins of the predictor reference (oracle/mlp.py) against things other than
itself: central finite differences, torch's float64 autograd and Adam, torch's
bfloat16 conversion, closed-form networks and the capacity invariants."""
import numpy as np
import pytest
import torch

from oracle import mlp


def rand_batch(B, seed):
    r = np.random.default_rng(seed)
    alen = r.integers(0, 40, B)
    nprod = alen * r.integers(1, 60, B) + r.integers(0, 5, B)
    bmax = np.minimum(r.integers(0, 60, B), nprod)
    X = mlp.features(alen, nprod, bmax)
    t = mlp.target(np.maximum(bmax, (nprod * r.uniform(0.2, 1.0, B)).astype(np.int64)))
    return X, t


def test_param_count():
    assert mlp.NPARAM == 64 * 3 + 64 + 64 * 64 + 64 + 64 + 1 == 4481


def test_grad_matches_central_differences():
    X, t = rand_batch(37, 1)
    th = mlp.init(3)
    th[mlp.NPARAM - 1] = 0.3
    th += np.random.default_rng(4).normal(0, 0.05, th.shape)   # nonzero biases
    _, g = mlp.grad(th, X, t, quant=False)
    h = 1e-6
    idx = np.random.default_rng(5).choice(mlp.NPARAM, 300, replace=False)
    idx = np.unique(np.concatenate([idx, np.arange(0, 192, 17), [4480, 4479, 4416, 4352]]))
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, t, quant=False) - mlp.loss(tm, X, t, quant=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def torch_net(th):
    p = mlp.unpack(th)
    net = torch.nn.Sequential(torch.nn.Linear(3, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64),
                              torch.nn.ReLU(), torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(p["W1"]))
        net[0].bias.copy_(torch.from_numpy(p["b1"]))
        net[2].weight.copy_(torch.from_numpy(p["W2"]))
        net[2].bias.copy_(torch.from_numpy(p["b2"]))
        net[4].weight.copy_(torch.from_numpy(p["W3"]))
        net[4].bias.copy_(torch.from_numpy(p["b3"]))
    return net


def test_forward_and_grad_match_torch_float64():
    X, t = rand_batch(200, 2)
    th = mlp.init(7) + np.random.default_rng(8).normal(0, 0.05, mlp.NPARAM)
    net = torch_net(th)
    xt = torch.from_numpy(X)
    y = net(xt)[:, 0]
    L = torch.mean((y - torch.from_numpy(t)) ** 2)
    L.backward()
    yo, _ = mlp.forward(th, X, quant=False)
    lo, go = mlp.grad(th, X, t, quant=False)
    np.testing.assert_allclose(yo, y.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(lo - L.item()) <= 1e-12 * max(1, L.item())
    gt = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                         net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                         net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
    np.testing.assert_allclose(go, gt, rtol=1e-10, atol=1e-13)


def test_round_bf16_matches_torch():
    r = np.random.default_rng(9)
    x = np.concatenate([r.normal(0, 1, 20000), r.normal(0, 1e-30, 200), r.normal(0, 1e30, 200),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40]]).astype(np.float32)
    # exact ties: low 16 bits 0x8000 with even and odd kept parts
    bits = (r.integers(0, 1 << 6, 500).astype(np.uint32) << 17) | (r.integers(100, 150, 500).astype(np.uint32) << 23)
    ties = np.concatenate([(bits | 0x8000).view(np.float32), (bits | 0x18000).view(np.float32)])
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.round_bf16(x), ref)
    np.testing.assert_array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)), ref)


def test_quantised_layer1_matches_torch_float32_ops():
    X, _ = rand_batch(500, 3)
    th = mlp.round_bf16(mlp.init(11) + np.random.default_rng(12).normal(0, 0.1, mlp.NPARAM))
    p = mlp.unpack(th)
    z, h = mlp.layer1(p["W1"], p["b1"], X, quant=True)
    x = torch.from_numpy(X.astype(np.float32))
    w = torch.from_numpy(p["W1"].astype(np.float32))
    b = torch.from_numpy(p["b1"].astype(np.float32))
    zt = b[None, :] + w[None, :, 0] * x[:, 0:1]
    zt = zt + w[None, :, 1] * x[:, 1:2]
    zt = zt + w[None, :, 2] * x[:, 2:3]
    np.testing.assert_array_equal(z, zt.double().numpy())
    ht = torch.relu(zt).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(h, ht)
    # the quantised forward differs from the exact one only through h1
    y, (_, _, h1, _, _) = mlp.forward(th, X, quant=True)
    y2, (_, _, h1x, _, _) = mlp.forward(th, X, quant=False)
    assert np.max(np.abs(h1 - h1x)) <= 2.0 ** -8 * np.max(np.abs(h1x)) + 1e-6


def test_closed_form_network():
    """A network that computes x0 + 2 x1 + 3 x2 + 0.5 on nonnegative inputs:
    three pass-through neurons in each hidden layer."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W1"][0, 0] = p["W1"][1, 1] = p["W1"][2, 2] = 1.0
    p["W2"][0, 0] = p["W2"][1, 1] = p["W2"][2, 2] = 1.0
    p["W3"][0, :3] = [1.0, 2.0, 3.0]
    p["b3"][0] = 0.5
    th = mlp.pack(p)
    X = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 3.0], [0.5, 0.25, 4.0], [10.0, 11.5, 7.0]])
    for q in (True, False):
        y, _ = mlp.forward(th, X, quant=q)
        np.testing.assert_array_equal(y, X @ [1.0, 2.0, 3.0] + 0.5)
    _, g = mlp.grad(th, X, X @ [1.0, 2.0, 3.0] + 0.5, quant=False)
    np.testing.assert_array_equal(g, 0.0)   # exact fit, zero loss


def test_adam_matches_torch():
    r = np.random.default_rng(13)
    th0 = r.normal(0, 1, 50)
    w = torch.tensor(th0.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.85, 0.995), eps=1e-7)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 8):
        g = r.normal(0, 1, 50) * (step % 3 + 0.1)
        w.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m, v = mlp.adam_step(th, m, v, g, step, lr=3e-3, b1=0.85, b2=0.995, eps=1e-7)
        np.testing.assert_allclose(th, w.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_training_reduces_loss():
    X, t = rand_batch(512, 21)
    th = mlp.init(22)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, X, t)
    for step in range(1, 301):
        _, g = mlp.grad(th, X, t)
        th, m, v = mlp.adam_step(th, m, v, g, step, lr=3e-3)
    assert mlp.loss(th, X, t) < 0.1 * l0


def test_capacity_rules():
    pred = np.log2(1 + np.array([10.0, 10.0, 0.0, 1000.0, 3.2, 5.0]))
    alen = np.array([3, 1, 4, 5, 2, 0])
    nprod = np.array([40, 7, 12, 50, 30, 0])
    bmax = np.array([12, 7, 5, 20, 9, 0])
    cap = mlp.capacity(pred, 0.25, alen, nprod, bmax, ncols=45)
    # ceil(10*1.25)=13 within [12, 40]; a_len<=1 exact; 0 -> b_max; 1250 -> min(50,45);
    # ceil(3.2*1.25)=4 -> b_max 9; empty row 0
    np.testing.assert_array_equal(cap, [13, 7, 5, 45, 9, 0])
    r = np.random.default_rng(5)
    n = 1000
    alen = r.integers(0, 30, n)
    nprod = alen * r.integers(0, 30, n)
    bmax = np.minimum(r.integers(0, 30, n), nprod)
    cap = mlp.capacity(r.normal(4, 3, n), 0.1, alen, nprod, bmax, ncols=200)
    hi = np.minimum(nprod, 200)
    assert np.all((cap >= np.minimum(bmax, hi)) & (cap <= np.maximum(hi, nprod * (alen <= 1))))


def test_pinball_gradient_matches_torch_and_differences():
    """Pinball loss: gradient against torch autograd of the same loss in
    float64, and against central differences at a point away from kinks."""
    X, t = rand_batch(120, 31)
    th = mlp.init(17) + np.random.default_rng(18).normal(0, 0.05, mlp.NPARAM)
    y0, _ = mlp.forward(th, X, quant=False)
    t = y0 + np.random.default_rng(19).choice([-1.0, 1.0], 120) * (0.3 + np.random.default_rng(20).random(120))
    for tau in (0.5, 0.9):
        net = torch_net(th)
        y = net(torch.from_numpy(X))[:, 0]
        r = torch.from_numpy(t) - y
        L = torch.mean(torch.where(r > 0, tau * r, (tau - 1.0) * r))
        L.backward()
        lo, go = mlp.grad(th, X, t, quant=False, tau=tau)
        gt = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                             net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                             net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
        assert abs(lo - L.item()) <= 1e-12
        np.testing.assert_allclose(go, gt, rtol=1e-10, atol=1e-13)
        h = 1e-7
        for i in (0, 5, 200, 1000, 4400, 4480):
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            fd = (mlp.loss(tp, X, t, quant=False, tau=tau) - mlp.loss(tm, X, t, quant=False, tau=tau)) / (2 * h)
            assert abs(fd - go[i]) <= 1e-5 * max(1.0, abs(go[i])), (tau, i, fd, go[i])


def test_pinball_level_is_the_empirical_quantile():
    """A constant model trained with the pinball loss of level tau settles at
    the tau-quantile of the targets (the defining property of the loss)."""
    r = np.random.default_rng(3)
    tgt = r.exponential(2.0, 1001)
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    X = np.zeros((tgt.size, 3))
    th = mlp.pack(p)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 2001):
        _, g = mlp.grad(th, X, tgt, quant=False, tau=0.9)
        g[:-1] = 0.0                  # only the output bias moves
        th, m, v = mlp.adam_step(th, m, v, g, step, lr=0.02)
    assert abs(th[-1] - np.quantile(tgt, 0.9)) < 0.08


def test_row_ranges_brute_force():
    import synthetic as syn
    A = syn.random_csr(60, 50, 0.08, seed=3)
    B = syn.random_csr(50, 70, 0.06, seed=4)
    lo, hi = mlp.row_ranges(A, B)
    for i in range(A.rows):
        cols = [c for k in A.col[A.rpt[i]:A.rpt[i + 1]] for c in B.col[B.rpt[k]:B.rpt[k + 1]]]
        if cols:
            assert (lo[i], hi[i]) == (min(cols), max(cols))
        else:
            assert lo[i] > hi[i]


def test_fmix64_is_a_bijection_with_avalanche():
    """MurmurHash3's finalizer is invertible (each xor-shift by 33 >= 32 is
    its own inverse, each multiplier is odd) and mixes: flipping one input
    bit flips about half of the output bits."""
    r = np.random.default_rng(11)
    x = r.integers(0, 2 ** 63, 2000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    y = mlp.fmix64(x)
    inv1, inv2 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64), pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    for a, b in zip(x[:200], y[:200]):
        k = int(b)
        k ^= k >> 33
        k = (k * inv2) % (1 << 64)
        k ^= k >> 33
        k = (k * inv1) % (1 << 64)
        k ^= k >> 33
        assert k == int(a)
    flips = []
    for bit in range(64):
        d = mlp.fmix64(x ^ np.uint64(1 << bit)) ^ y
        flips.append(np.mean([bin(int(v)).count("1") for v in d[:300]]))
    assert 30.0 < np.mean(flips) < 34.0 and min(flips) > 28.0


def test_calibration_pick_eligibility_and_small_octaves():
    """Picks are eligible rows only (a_len >= 2, 1 <= n_prod < 2^21, range
    <= CAL_SPAN_MAX columns, each bound checked on both sides), octaves are
    floor(log2 n_prod), and an octave with no more rows than its quota
    gives every row."""
    alen = np.array([2, 1, 2, 2, 2, 2, 2, 2, 3, 2])
    nprod = np.array([1, 5, 0, (1 << 21) - 1, 1 << 21, 8, 7, 1 << 19, 100, 100])
    span = np.array([1, 1, 1, 5, 5, mlp.CAL_SPAN_MAX, mlp.CAL_SPAN_MAX + 1, 3, 3, 3])
    rows, octave = mlp.calibration_pick(alen, nprod, span)
    assert list(octave) == [0, 2, -1, 20, 21, 3, 2, 19, 6, 6]
    assert list(rows) == [0, 3, 5, 7, 8, 9]
    # a quota of 64 (octave 6) and of 32 (octave 19): c <= K takes every row
    M = 96
    nprod = np.where(np.arange(M) < 64, 100, 1 << 19)
    rows, _ = mlp.calibration_pick(np.full(M, 2), nprod, np.zeros(M))
    assert rows.size == 64 + 32


def test_calibration_pick_counts_near_quota():
    """An octave with c > K eligible rows yields about K picks: over seeded
    layouts (octaves contiguous or scattered over the row indices) the
    count lies in [K/2, 2K] for at least 99 % of the octaves, and the mean
    of count / K is 1 within 5 %.  A stride or quota off by a factor of two
    fails this."""
    r = np.random.default_rng(1)
    ratios, inside = [], []
    for trial in range(200):
        M = int(r.integers(2000, 40000))
        base = int(r.integers(0, 1 << 17))   # different row indices per layout
        npd = (2.0 ** r.uniform(0, 21.5, M)).astype(np.int64)
        if trial % 2:
            npd = np.sort(npd)
        alen = r.integers(1, 6, M)
        span = np.where(r.random(M) < 0.05, 1 << 24, 100)
        big_alen = np.concatenate([np.zeros(base, np.int64), alen])
        big_np = np.concatenate([np.zeros(base, np.int64), npd])
        big_span = np.concatenate([np.zeros(base, np.int64), span])
        rows, octave = mlp.calibration_pick(big_alen, big_np, big_span)
        elig = (big_alen >= 2) & (big_np >= 1) & (octave <= mlp.CAL_MAX_OCT) & (big_span <= mlp.CAL_SPAN_MAX)
        for o in np.unique(octave[elig]):
            c = int(np.sum(elig & (octave == o)))
            k = min(c, min(max(mlp.CAL_OCT_PRODUCTS >> int(o), mlp.CAL_MIN_ROWS), 64))
            if c <= k:
                continue
            got = int(np.sum(octave[rows] == o))
            ratios.append(got / k)
            inside.append(k / 2 <= got <= 2 * k)
    assert len(ratios) > 2000
    assert np.mean(inside) >= 0.99
    assert abs(np.mean(ratios) - 1.0) < 0.05


def test_calibration_scale_covers_every_picked_row():
    """With margin 0, every picked row of an octave that is scaled gets a
    capacity of at least its exact size (the scale is the largest ratio of
    the octave's picked rows); a mean ratio would leave rows short here."""
    r = np.random.default_rng(5)
    M = 20000
    nprod = (2.0 ** r.uniform(2, 16, M)).astype(np.int64)
    alen = np.full(M, 4)
    bmax = np.minimum(nprod, 3)
    true = np.maximum(bmax, (nprod * r.uniform(0.2, 0.9, M)).astype(np.int64))
    # the estimates err by a random factor in [0.5, 2] per row
    pred = np.log2(1.0 + true * 2.0 ** r.uniform(-1, 1, M))
    sc, _, rows = mlp.calibration(pred, lambda q: true[q], alen, nprod, bmax, ncols=1 << 20,
                                  span=np.full(M, 100))
    cap = mlp.capacity(pred, 0.0, alen, nprod, bmax, 1 << 20, scale=sc)
    octave = np.floor(np.log2(nprod)).astype(np.int64)
    scaled = [o for o in np.unique(octave[rows]) if np.sum(octave[rows] == o) >= mlp.CAL_MIN_ROWS]
    assert len(scaled) >= 10
    pr = rows[np.isin(octave[rows], scaled)]
    assert np.all(cap[pr] >= true[pr])
    # the same rule with the mean ratio instead would not cover them
    est = np.clip(np.exp2(pred) - 1.0, np.minimum(bmax, nprod), nprod)
    mean_sc = np.ones(M)
    for o in scaled:
        sel = rows[octave[rows] == o]
        mean_sc[octave == o] = np.mean(true[sel] / est[sel])
    cap_mean = mlp.capacity(pred, 0.0, alen, nprod, bmax, 1 << 20, scale=mean_sc)
    assert np.any(cap_mean[pr] < true[pr])


def test_calibration_scales_per_octave():
    """Two octaves with opposite biases get their own scales; the exact
    sizes used are those of the picked rows only; within an octave the scale
    is the largest size / estimate ratio of its picked rows."""
    M = 4000
    nprod = np.where(np.arange(M) < M // 2, 100, 1500)          # octaves 6 and 10
    alen = np.full(M, 4)
    bmax = np.full(M, 10)
    true = np.where(nprod == 100, 50, 1000)
    pred = np.log2(1 + np.where(nprod == 100, 25.0, 1200.0))    # 2x under, 1.2x over
    seen = []
    sc, overall, rows = mlp.calibration(pred, lambda r: (seen.append(r), true[r])[1], alen, nprod, bmax,
                                        ncols=10 ** 6, span=np.full(M, 5000))
    np.testing.assert_array_equal(seen[0], rows)
    assert 64 <= rows.size <= 256
    np.testing.assert_allclose(sc[nprod == 100], 2.0)
    np.testing.assert_allclose(sc[nprod == 1500], 1000 / 1200)
    n6 = np.sum(nprod[rows] == 100)
    n10 = rows.size - n6
    assert abs(overall - (n6 * 50 + n10 * 1000) / (n6 * 25 + n10 * 1200)) < 1e-12
    # estimates clamped to [min(b_max, U), U] before the ratio; a capacity uses the row's scale
    cap = mlp.capacity(pred, 0.0, alen, nprod, bmax, 10 ** 6, scale=sc)
    assert cap[0] == 50 and cap[-1] == 1000
    # a spread inside one octave: the scale is the largest ratio of the picked rows
    true2 = np.where(np.arange(M) % 3 == 0, 60, 50) * (nprod == 100) + true * (nprod == 1500)
    sc2, _, rows2 = mlp.calibration(pred, lambda r: true2[r], alen, nprod, bmax, ncols=10 ** 6,
                                    span=np.full(M, 5000))
    r6 = rows2[nprod[rows2] == 100]
    assert abs(sc2[0] - 60 / 25.0) < 1e-12 and np.all(sc2[nprod == 100] == sc2[0])
