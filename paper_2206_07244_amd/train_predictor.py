"""Train the row-size predictor on the GPU with the library's own kernels.

Labels are exact row sizes of C = A*A from the library's two-phase product
(the symbolic result, read from C's row pointer) on generated matrices of
four families (R-MAT, banded, Poisson-uniform rows, stencils; see
``synthetic.training_set``).  Up to ``--rows`` rows are sampled per matrix.
Features come from ``opsp_mlp_features``, gradients from ``opsp_mlp_grad``
and the updates from ``opsp_mlp_adam`` (float32 master weights, bf16 copy);
PyTorch only holds the arrays and draws the minibatch permutations.  The
default loss is the pinball loss of level 0.9, so the network estimates an
upper quantile of each row's size and the capacity margin stays small.

Every tenth matrix is held out.  After training, the capacity margin is
chosen on the held-out rows (see choose_margin), and the parameters (bf16
bit patterns), the margin and the training summary are written as JSON.

Usage: python -m paper_2206_07244_amd.train_predictor [--out FILE] [--count 200]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print("[train]", *a, file=sys.stderr, flush=True)


def he_init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, packed W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((3, (64, 3)), (None, (64,)), (64, (64, 64)), (None, (64,)),
                          (64, (1, 64)), (None, (1,))):
        if fan_in is None:
            parts.append(np.zeros(shape))
        else:
            b = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-b, b, shape))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def label_matrix(ops, torch, A, rows: int, rng):
    """(X float32 [k,3], target float32 [k]) for up to `rows` sampled rows."""
    dA = ops.DeviceCSR.from_host(A)
    C = ops.spgemm(dA, dA)
    nnz = (C.rpt[1:] - C.rpt[:-1]).to(torch.float32)
    X = ops.mlp_features(dA, dA)
    if A.rows > rows:
        idx = torch.from_numpy(np.sort(rng.choice(A.rows, rows, replace=False))).to(X.device)
        X, nnz = X[idx], nnz[idx]
    T = torch.log2(1.0 + nnz)
    del C, dA
    return X.contiguous(), T.contiguous()


def evaluate(ops, torch, P, X, T, tau=0.0):
    """Mean training loss (squared error, or pinball loss of level tau)."""
    y = ops.mlp_forward(P, X)
    r = (T - y).double()
    if tau > 0:
        return float(torch.where(r > 0, tau * r, (tau - 1.0) * r).mean())
    return float((r * r).mean())


def choose_margin(ops, torch, P, X, T, max_table_overflow: float = 0.002,
                  max_arena_share: float = 0.1) -> dict:
    """Smallest margin m on a grid of 0.05 with which, on the given rows,
    (i) at most `max_table_overflow` of the rows exceed 1.6x their capacity
    (where the one-phase kernels abandon a row's table and recompute it) and
    (ii) the rows exceeding their capacity hold at most `max_arena_share` of
    the capacity total (the overflow arena holds an eighth of it).  Slots
    that are too small cost only an arena store, so the margin stays small;
    it sets the temporary space and the table sizes of the numeric bins."""
    y = ops.mlp_forward(P, X).double()
    est = torch.exp2(y) - 1.0
    nnz = torch.exp2(T.double()) - 1.0
    nprod = torch.exp2(X[:, 1].double()) - 1.0
    bmax = torch.exp2(X[:, 2].double()) - 1.0
    alen = torch.round(torch.exp2(X[:, 0].double()) - 1.0)
    chosen = None
    for i in range(0, 41):
        m = 0.05 * i
        cap = torch.minimum(torch.maximum(torch.ceil(est * (1 + m)), torch.minimum(bmax, nprod)), nprod)
        cap = torch.where(alen <= 1, nprod, cap)
        tab = float((nnz > 1.6 * cap).double().mean())
        arena = float(nnz[nnz > cap].sum() / cap.sum().clamp(min=1))
        if tab <= max_table_overflow and arena <= max_arena_share:
            chosen = (m, cap, tab, arena)
            break
    if chosen is None:
        m = 2.0
        cap = torch.minimum(torch.maximum(torch.ceil(est * (1 + m)), torch.minimum(bmax, nprod)), nprod)
        chosen = (m, cap, float((nnz > 1.6 * cap).double().mean()),
                  float(nnz[nnz > cap].sum() / cap.sum().clamp(min=1)))
    m, cap, tab, arena = chosen
    pr = (est / nnz.clamp(min=1)).cpu().numpy()
    return {"margin": round(m, 2), "slot_overflow_frac": float((nnz > cap).double().mean()),
            "table_overflow_frac": tab, "arena_share": arena,
            "cap_over_nnz": float(cap.sum() / nnz.sum()),
            "pred_over_true_median": float(np.median(pr)),
            "pred_over_true_p01": float(np.quantile(pr, 0.01)),
            "pred_over_true_p99": float(np.quantile(pr, 0.99))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "predictor_weights.json"))
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--rows", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--tau", type=float, default=0.9,
                    help="0 = mean squared error; 0 < tau < 1 = pinball loss of level tau "
                         "(the network estimates the tau-quantile of log2(1 + nnz))")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--n-lo-log2", type=int, default=14)
    ap.add_argument("--n-hi-log2", type=int, default=18)
    args = ap.parse_args(argv)

    import torch
    import synthetic as syn
    import paper_2206_07244_amd as ops

    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    torch.cuda.set_device(0)
    rng = np.random.default_rng(args.seed)
    t0 = time.time()
    Xs, Ts, Xv, Tv = [], [], [], []
    names = []
    for j in range(args.count):
        name, A = syn.training_matrix(j, n_lo_log2=args.n_lo_log2, n_hi_log2=args.n_hi_log2)
        X, T = label_matrix(ops, torch, A, args.rows, rng)
        (Xv if j % 10 == 9 else Xs).append(X)
        (Tv if j % 10 == 9 else Ts).append(T)
        names.append(name)
        if j % 20 == 0:
            log(f"matrix {j}: {name} rows={A.rows} nnz={A.nnz} ({time.time() - t0:.0f}s)")
        del A
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    Xval = torch.cat(Xv)
    Tval = torch.cat(Tv)
    log(f"labelled {X.shape[0]} training rows, {Xval.shape[0]} held out, {time.time() - t0:.0f}s")

    master = torch.from_numpy(he_init(args.seed)).cuda()
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    P = torch.zeros(ops.MLP_NPARAM, dtype=torch.int16, device="cuda")
    # bf16 copy of the initial weights through a zero-rate Adam step
    ops.mlp_adam(master, m, v, torch.zeros_like(master), 1, P, lr=0.0)
    m.zero_()
    v.zero_()
    n = X.shape[0]
    steps_per_epoch = max(1, n // args.batch)
    total = steps_per_epoch * args.epochs
    gen = torch.Generator().manual_seed(args.seed)
    step = 0
    hist = []
    t1 = time.time()
    for ep in range(args.epochs):
        perm = torch.randperm(n, generator=gen).cuda()
        for i in range(steps_per_epoch):
            idx = perm[i * args.batch:(i + 1) * args.batch]
            g, _ = ops.mlp_grad(P, X[idx].contiguous(), T[idx].contiguous(), tau=args.tau)
            step += 1
            lr = args.lr * 0.5 * (1 + math.cos(math.pi * step / total))   # cosine decay
            ops.mlp_adam(master, m, v, g, step, P, lr=lr)
        tr = evaluate(ops, torch, P, X, T, args.tau)
        va = evaluate(ops, torch, P, Xval, Tval, args.tau)
        hist.append((ep, tr, va))
        log(f"epoch {ep}: train loss {tr:.5f}  held-out loss {va:.5f}  ({time.time() - t1:.0f}s)")
    stats = choose_margin(ops, torch, P, Xval, Tval)
    log("held-out:", stats)
    bits = P.cpu().numpy().view(np.uint16).tolist()
    out = {
        "format": "opsp-predictor-v1",
        "layout": "W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3; bfloat16 bit patterns",
        "features": "log2(1 + a_len), log2(1 + n_prod), log2(1 + b_max)",
        "target": "log2(1 + nnz)",
        "loss": "pinball" if args.tau > 0 else "mse",
        "tau": args.tau,
        "params_bf16": bits,
        "margin": stats["margin"],
        "train": {"matrices": args.count, "rows_per_matrix": args.rows, "train_rows": int(n),
                  "heldout_rows": int(Xval.shape[0]), "epochs": args.epochs, "batch": args.batch,
                  "lr": args.lr, "seed": args.seed, "loss_history": hist, "heldout": stats,
                  "seconds": round(time.time() - t0, 1)},
    }
    with open(args.out, "w") as f:
        json.dump(out, f)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
