"""Autotuner of the binning configuration (bin ranges of both steps).

The paper sizes its bins with a ratio rule (Section 5.7: a row goes to the
first table at least `ratio` times its n_prod or nnz) and measures a grid of
ratios (Sym 1x/1.2x/1.5x, Num 1x/1.5x/2x/3x) to pick Sym_1.2x and Num_2x.
This tuner starts from that grid, refines the best pair of ratios, then
moves each bin boundary of the best configuration on its own (coordinate
search over the explicit per-bin bounds of opsp_config version 2, each kept
within its table's capacity), then the abort fraction of the largest
symbolic table and hashing every row, the lanes per row of bin 0 with its
table sizes (4 / 8 / 16 lanes: tables of 64 / 128 / 256 keys), and the
number of streams the bin kernels are spread over.  Each candidate is timed on sample inputs of one workload
class; the fastest configuration per class is written to JSON.

The search policy (``search``) is separate from the timing (``GpuTimer``) so
that it can be exercised with any cost function.

Usage:
  python -m paper_2206_07244_amd.autotune --out tuning.json [--classes stencil,fem,rmat,banded,batch]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Callable, Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_TUNING = os.path.join(HERE, "tuning.json")
PAPER_SYM = [1.0, 1.2, 1.5]
PAPER_NUM = [1.0, 1.5, 2.0, 3.0]
BOUND_STEPS = [0.5, 0.75, 1.25, 1.5]
ABORT_FRACTIONS = [0.6, 0.7, 0.8, 0.9]
GROUP_LANES = [4, 16]       # bin 0: lanes per row (and with them its table sizes)
STREAMS = [2, 4]            # bin kernels spread over several streams


def log(*a):
    print("[tune]", *a, file=sys.stderr, flush=True)


class Candidate(dict):
    """A configuration as a plain dict: sym_ratio, num_ratio, sym_bounds[7],
    num_bounds[7], sym_abort_fraction."""

    def key(self):
        return (round(self["sym_ratio"], 6), round(self["num_ratio"], 6), tuple(self["sym_bounds"]),
                tuple(self["num_bounds"]), round(self["sym_abort_fraction"], 6),
                int(self.get("hash_all_rows", 0)), int(self.get("group_lanes", 0)),
                int(self.get("streams", 0)))


def base_candidate(sr=1.2, nr=2.0) -> Candidate:
    return Candidate(sym_ratio=sr, num_ratio=nr, sym_bounds=[0] * 7, num_bounds=[0] * 7,
                     sym_abort_fraction=0.8, hash_all_rows=0, group_lanes=0, streams=0)


def derived_bounds(step: int, tsizes: List[int], ratio: float) -> List[int]:
    """Bounds of bins 0..6 from the ratio rule (same rule as the library's
    opsp_bin_bounds)."""
    from fractions import Fraction
    r = Fraction(str(ratio))
    out = []
    for t in tsizes[:7]:
        if step == 0:
            out.append(int(Fraction(t) / r))
        else:
            out.append(min(t, int(Fraction(t + 1) / r)))
    return out


def search(cost: Callable[[Candidate], float], sym_t: List[int], num_t: List[int],
           refine: bool = True, coordinate: bool = True, abort: bool = True,
           trace: Optional[list] = None) -> (Candidate, float):
    """Return the cheapest candidate found and its cost.  `cost` is called
    once per distinct candidate; sym_t / num_t are the table sizes of bins
    0..6 (0..7 for the symbolic step's abort bin)."""
    seen: Dict[tuple, float] = {}

    def ev(c: Candidate) -> float:
        k = c.key()
        if k not in seen:
            seen[k] = cost(c)
            if trace is not None:
                trace.append((dict(c), seen[k]))
        return seen[k]

    best, bc = None, float("inf")
    # 1. the paper's grid of ratios
    for sr in PAPER_SYM:
        for nr in PAPER_NUM:
            c = base_candidate(sr, nr)
            v = ev(c)
            if v < bc:
                best, bc = c, v
    # 2. finer ratios around the best pair
    if refine:
        sr0, nr0 = best["sym_ratio"], best["num_ratio"]
        for dsr in (-0.1, 0.0, 0.1):
            for dnr in (-0.25, 0.0, 0.25):
                sr = round(sr0 + dsr, 3)
                nr = round(nr0 + dnr, 3)
                if sr < 1.0 or nr < 1.0:
                    continue
                c = base_candidate(sr, nr)
                v = ev(c)
                if v < bc:
                    best, bc = c, v
    # 3. each bin boundary on its own, starting from the ratio-derived bounds
    if coordinate:
        cur = Candidate(best)
        cur["sym_bounds"] = derived_bounds(0, sym_t, cur["sym_ratio"])
        cur["num_bounds"] = derived_bounds(1, num_t, cur["num_ratio"])
        cc = ev(cur)   # the same bins as `best`, written out
        for field, tsz in (("num_bounds", num_t), ("sym_bounds", sym_t)):
            for j in range(7):
                base_ub = cur[field][j]
                for f in BOUND_STEPS:
                    ub = int(round(base_ub * f))
                    ub = max(1, min(ub, tsz[j]))
                    if ub == cur[field][j]:
                        continue
                    c = Candidate(cur)
                    c[field] = list(cur[field])
                    c[field][j] = ub
                    v = ev(c)
                    if v < cc:
                        cur, cc = c, v
        if cc < bc:
            best, bc = cur, cc
    # 4. abort fraction of the largest symbolic table, and hashing every row
    #    (the paper's method) against the bitmap / dense paths for narrow rows
    if abort:
        for a in ABORT_FRACTIONS:
            c = Candidate(best)
            c["sym_abort_fraction"] = a
            v = ev(c)
            if v < bc:
                best, bc = c, v
        c = Candidate(best)
        c["hash_all_rows"] = 1 - int(best.get("hash_all_rows", 0))
        v = ev(c)
        if v < bc:
            best, bc = c, v
    # 5. lanes per row of bin 0 (its tables grow or shrink with them; an
    #    explicit bin-0 bound is re-derived from the ratio), then several
    #    streams for the bin kernels
    if abort:
        for g in GROUP_LANES:
            c = Candidate(best)
            c["group_lanes"] = g
            c["sym_bounds"] = [0] + list(best["sym_bounds"][1:])
            c["num_bounds"] = [0] + list(best["num_bounds"][1:])
            v = ev(c)
            if v < bc:
                best, bc = c, v
        for n in STREAMS:
            c = Candidate(best)
            c["streams"] = n
            v = ev(c)
            if v < bc:
                best, bc = c, v
    return best, bc


def to_config(c: dict):
    import paper_2206_07244_amd as ops
    return ops.Config(sym_ratio=c["sym_ratio"], num_ratio=c["num_ratio"],
                      sym_abort_fraction=c["sym_abort_fraction"], sym_bounds=c["sym_bounds"],
                      num_bounds=c["num_bounds"], hash_all_rows=int(c.get("hash_all_rows", 0)),
                      group_lanes=int(c.get("group_lanes", 0)), streams=int(c.get("streams", 0)))


def load_config(cls: str, path: Optional[str] = None):
    """The tuned Config of a workload class, or None when none is stored."""
    p = path or DEFAULT_TUNING
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    c = d.get("classes", {}).get(cls)
    return to_config(c["config"]) if c else None


class GpuTimer:
    """Median time (ms) of `reps` rounds of `calls` products with a config,
    measured with HIP events on the current stream."""

    def __init__(self, run: Callable, calls: int = 3, reps: int = 3):
        self.run, self.calls, self.reps = run, calls, reps

    def __call__(self, c: Candidate) -> float:
        import torch
        cfg = to_config(c)
        self.run(cfg)   # warm-up (memory cache)
        torch.cuda.synchronize()
        ts = []
        for _ in range(self.reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.calls):
                self.run(cfg)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / self.calls)
        ts.sort()
        return ts[len(ts) // 2]


def class_inputs(cls: str):
    """Sample inputs of a workload class (smaller than the benchmark inputs)."""
    import synthetic as syn
    if cls == "stencil":
        A = syn.stencil27(60, seed=60)
        return [(A, A)]
    if cls == "fem":
        A = syn.block_stencil27(24, 3, seed=24)
        return [(A, A)]
    if cls == "rmat":
        A = syn.rmat(18, 16, seed=18)
        return [(A, A)]
    if cls == "banded":
        A = syn.banded(1 << 19, 64, 12, seed=19)
        return [(A, A)]
    if cls == "batch":
        return syn.batch_pairs(64, seed=40)
    raise ValueError(cls)


def make_runner(cls: str, dev):
    import paper_2206_07244_amd as ops
    import torch
    pairs = class_inputs(cls)
    if cls == "batch":
        dA = [ops.DeviceCSR.from_host(A, dev) for A, _ in pairs]
        dB = [ops.DeviceCSR.from_host(B, dev) for _, B in pairs]
        stream = torch.cuda.current_stream()

        def run(cfg):
            b = ops.Batch(dA, dB, config=cfg, stream=stream)
            b.raw_execute(stream.cuda_stream)
            del b
        return run
    dA = ops.DeviceCSR.from_host(pairs[0][0], dev)
    Ac = dA._c()
    sh = torch.cuda.current_stream().cuda_stream

    def run(cfg):
        C = ops.opsp_csr()
        code = ops.lib().opsp_spgemm_ex(ops.byref(Ac), ops.byref(Ac), ops.byref(C), ops.byref(cfg),
                                        None, sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_ex")
        ops.free_raw(C, sh)
    return run


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TUNING)
    ap.add_argument("--classes", default="stencil,fem,rmat,banded,batch")
    ap.add_argument("--calls", type=int, default=3)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    import paper_2206_07244_amd as ops
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sym_t = ops.table_sizes(0)[:8]
    num_t = ops.table_sizes(1)[:7]
    out = {"device": torch.cuda.get_device_name(0), "library": ops.lib().opsp_version().decode(),
           "classes": {}}
    for cls in args.classes.split(","):
        t0 = time.time()
        timer = GpuTimer(make_runner(cls, dev), args.calls, args.reps)
        trace = []
        base = timer(base_candidate())
        best, ms = search(timer, sym_t, num_t, trace=trace)
        out["classes"][cls] = {"config": dict(best), "ms": ms, "default_ms": base,
                               "speedup_vs_default": base / ms, "trials": len(trace),
                               "seconds": round(time.time() - t0, 1)}
        log(f"{cls}: default {base:.3f} ms -> {ms:.3f} ms with {dict(best)} ({len(trace)} trials)")
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
