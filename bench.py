#!/usr/bin/env python3
"""Benchmark of the opsp SpGEMM hot path on one MI355X.

One step = one full C = A*B through the C ABI (``opsp_spgemm``: setup,
both binnings, symbolic, scan, allocation of C, numeric, release of C), on
inputs already resident in HBM.  The default workload is the square of an
R-MAT graph of 2^20 vertices, degree 16, (a,b,c,d) = (.57,.19,.19,.05),
values U(0,1] from seed 20 (C has 9.7e9 entries, 116 GB); the 3-D
27-point stencil on a 100^3 grid (values U[-1,1) from seed 27) and the
27-point stencil on a 40^3 grid with dense 3x3 node blocks (compression
ratio 17.6, the finite-element class) are reported beside it.

Metric (OpSparse Section 6): GFLOPS = 2 * n_prod / time, FP64.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOPS (2·nprod/s) C=A², FP64, + % HBM roofline; learned vs plain"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Sources whose change invalidates a stored HBM-traffic measurement of the
# numeric kernels (the counters were taken on the build of these files).
TRAFFIC_SOURCES = ["paper_2206_07244_amd/csrc/kernels_num.hip", "paper_2206_07244_amd/csrc/opsp_dev.h",
                   "paper_2206_07244_amd/csrc/opsp_tables.h"]


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summaries under profiles/ (a line 'traffic_record: {json}'),
    scaled by the copy calibration; None when no record matches the current
    kernel sources."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    digest = sources_digest()
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(d, f)) as fh:
            for line in fh:
                if line.startswith("traffic_record:"):
                    try:
                        r = json.loads(line.split(":", 1)[1])
                    except ValueError:
                        continue
                    if (r.get("kernel") == kernel and r.get("workload") == workload
                            and r.get("sources_sha1") == digest):
                        return r
    return None


def workload_class(name: str) -> str:
    """Autotuner class of a named workload."""
    if name.startswith("rmat"):
        return "rmat"
    if name.startswith("band"):
        return "banded"
    if name.startswith("bst"):
        return "fem"
    return "stencil"


def numeric_bytes(M, nnzA, nprod, nnzC):
    """Algorithmic HBM bytes of the numeric step (one launch over all rows):
    A col+val 12 B/entry and B row bounds 16 B per A entry; B col+val 12 B per
    intermediate product; C col+val 12 B per output; C.rpt 16 B and row id
    8 B per row."""
    return 12 * nprod + 28 * nnzA + 12 * nnzC + 24 * M


def symbolic_bytes(M, nnzA, nprod):
    """Symbolic step: A col 4 B + B row bounds 16 B per A entry, B col 4 B per
    product, n_prod read + nnz written 16 B per row, row id 8 B per row."""
    return 4 * nprod + 20 * nnzA + 24 * M


def bucket_bytes(ops, torch, dA, crpt, bounds_num):
    """Algorithmic HBM bytes of one launch of the long-row numeric kernel
    (bin 7): the numeric_bytes model over the rows of that bin only (rows
    whose nnz exceeds every numeric LDS bin bound), and the rows, products
    and outputs it covers."""
    _, npd, _ = ops.row_features(dA, dA)
    nnz = crpt[1:] - crpt[:-1]
    alen = dA.rpt[1:] - dA.rpt[:-1]
    in_lds = torch.zeros_like(nnz, dtype=torch.bool)
    for ub in bounds_num:
        in_lds |= nnz <= ub
    big = ~in_lds
    rows = int(big.sum().item())
    nprod = int(npd[big].sum().item())
    nnzc = int(nnz[big].sum().item())
    annz = int(alen[big].sum().item())
    return numeric_bytes(rows, annz, nprod, nnzc), {"rows": rows, "nprod": nprod, "nnzC": nnzc,
                                                     "nnzA": annz}


def numeric_bounds(ops, cfg):
    """Inclusive nnz bounds of numeric bins 0..6 under `cfg` (explicit
    bounds where given, else the ratio rule over the table sizes)."""
    ts = ops.table_sizes(1)[:7]
    ratio = cfg.num_ratio if cfg is not None and cfg.num_ratio > 0 else 2.0
    derived = ops.bin_bounds(1, ts, ratio)
    explicit = list(cfg.num_bounds) if cfg is not None else [0] * 7
    return [e if e != 0 else d for e, d in zip(explicit, derived)]


def measure_plain(ops, torch, np, syn, name, steps, warmup, dev, tuned_cls=True, builtin=True):
    """Time `steps` whole products C = A^2 of a named workload (inputs
    resident, C allocated and released inside the timed region) and the
    dominant kernel's duration with HIP events on the call's stream."""
    from paper_2206_07244_amd import autotune
    desc, builder = syn.WORKLOADS[name]
    t0 = time.time()
    A = builder()
    log(f"workload {name}: {A.rows} rows, {A.nnz} nnz, generated in {time.time() - t0:.1f}s")
    dA = ops.DeviceCSR.from_host(A, dev)
    torch.cuda.synchronize()
    sh = torch.cuda.current_stream().cuda_stream
    Ac = dA._c_fast(A.nnz)
    L = ops.lib()
    cls = workload_class(name)
    tuned = autotune.load_config(cls) if tuned_cls else None
    tref = ops.byref(tuned) if tuned is not None else None
    log(f"bin configuration: {'tuned for ' + cls if tuned is not None else 'built-in'}")

    st = ops.Stats()
    for _ in range(max(warmup, 1)):
        Cc = ops.opsp_csr()
        code = L.opsp_spgemm_ex(ops.byref(Ac), ops.byref(Ac), ops.byref(Cc), tref, ops.byref(st), sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_ex")
        ops.free_raw(Cc, sh)
    torch.cuda.synchronize()
    nprod, nnzC = st.nprod, st.nnz
    log(f"n_prod={nprod} nnz(C)={nnzC} CR={nprod / max(nnzC, 1):.3f} bins sym={list(st.sym_bin_rows)} "
        f"num={list(st.num_bin_rows)}")

    def timed(cref):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            Cc = ops.opsp_csr()
            code = L.opsp_spgemm_ex(ops.byref(Ac), ops.byref(Ac), ops.byref(Cc), cref, None, sh)
            if code:
                raise ops.OpspError(code, "opsp_spgemm_ex")
            ops.free_raw(Cc, sh)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3 / steps
    ms = timed(tref)
    gflops = 2.0 * nprod / (ms * 1e-3) / 1e9
    log(f"timed {steps} steps: {ms:.3f} ms/step, {gflops:.1f} GFLOPS")
    ms_default = timed(None) if (tuned is not None and builtin) else None
    if ms_default is not None:
        log(f"built-in configuration: {ms_default:.3f} ms/step")

    # per-stage and per-kernel durations: the same calls with HIP events
    # recorded on the call's stream (stage 3 = all numeric kernels, slot 5 =
    # the long-row numeric kernel alone)
    cfg = autotune.load_config(cls) if tuned is not None else ops.Config()
    cfg.stage_timing = 1
    stage = np.zeros(8)
    C_keep = None
    for k in range(steps):
        Cc = ops.opsp_csr()
        s2 = ops.Stats()
        code = L.opsp_spgemm_ex(ops.byref(Ac), ops.byref(Ac), ops.byref(Cc), ops.byref(cfg),
                                ops.byref(s2), sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_ex")
        if k == steps - 1:
            C_keep = Cc
        else:
            ops.free_raw(Cc, sh)
        stage += np.array(list(s2.ms_stage))
    torch.cuda.synchronize()
    stage /= steps
    log("stage ms (setup+bin, symbolic, numbin+scan, numeric, total, long-row numeric kernel):",
        [round(x, 4) for x in stage[:6]])

    M, nnzA = A.rows, A.nnz
    if stage[5] > 0.5 * stage[3]:
        # the long-row kernel dominates: its own bytes over its own time
        crpt = ops._wrap(C_keep.rpt, M + 1, torch.int64, None, dev)
        bytes_, cover = bucket_bytes(ops, torch, dA, crpt, numeric_bounds(ops, tuned))
        del crpt
        kernel = "k_num_global" if cfg.hash_all_rows else "k_num_bucket"
        kms = stage[5]
    else:
        bytes_, cover = numeric_bytes(M, nnzA, nprod, nnzC), {"rows": M, "nprod": nprod,
                                                               "nnzC": nnzC, "nnzA": nnzA}
        kernel, kms = "numeric", stage[3]
    ops.free_raw(C_keep, sh)
    torch.cuda.synchronize()
    achieved = bytes_ / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    roof = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes": int(bytes_), "kernel_ms": round(float(kms), 4), "covers": cover}
    rec = stored_traffic(kernel, name)
    if rec is not None:
        roof["traffic"] = int(rec["bytes_per_launch"])
        roof["traffic_source"] = rec.get("file", "profiles")
        roof["traffic_frac"] = round(rec["bytes_per_launch"] / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    res = {"A": A, "dA": dA, "desc": desc, "ms": ms, "gflops": gflops, "nprod": nprod, "nnzC": nnzC,
           "ms_default": ms_default, "stage": stage, "roofline": roof, "cls": cls,
           "tuned": tuned is not None}
    return res


def time_fp32(ops, torch, np, syn, name, steps, warmup, dev, tuned_cls=True):
    """The same product with FP32 values (opsp_spgemm_f32, inputs rounded to
    float32), timed like the FP64 legs."""
    import ctypes
    from paper_2206_07244_amd import autotune
    desc, builder = syn.WORKLOADS[name]
    A = builder()
    dA = ops.DeviceCSR.from_host(A, dev, dtype=np.float32)
    torch.cuda.synchronize()
    sh = torch.cuda.current_stream().cuda_stream
    Ac = dA._c_fast(A.nnz)
    L = ops.lib()
    tuned = autotune.load_config(workload_class(name)) if tuned_cls else None
    tref = ctypes.byref(tuned) if tuned is not None else None
    st = ops.Stats()

    def once(stats=None):
        Cc = ops.opsp_csr()
        code = L.opsp_spgemm_f32(ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(Cc), tref,
                                 ctypes.byref(stats) if stats is not None else None, sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_f32")
        L.opsp_csr_f32_free(ctypes.byref(Cc), sh)
    once(st)
    for _ in range(warmup):
        once()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / steps
    g = 2.0 * st.nprod / (ms * 1e-3) / 1e9
    log(f"fp32 {name}: {ms:.3f} ms/step, {g:.1f} GFLOPS")
    return {"workload": name, "dtype": "f32", "value": round(g, 3), "unit": "GFLOPS",
            "ms_per_step": round(ms, 4), "nprod": st.nprod, "nnzC": st.nnz}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, np, seconds):
    """The CPU oracle on a bounded, stratified sample of the workload's
    rows: rows ordered by n_prod, every s-th taken, s chosen from a short
    pilot so that the single-threaded run takes about `seconds`; then the
    same rows on all available cores (the oracle's row-parallel form, same
    per-row code).  GFLOPS = 2 * (products of the sampled rows) / time."""
    import oracle
    oracle.build(force=False)
    nprod, _, _, tot = oracle.row_stats(A, A)
    order = np.argsort(nprod, kind="stable")

    def sample(stride):
        return np.sort(order[stride // 2::stride]).astype(np.int64)

    def run(rows, threads):
        t = time.perf_counter()
        oracle.spgemm(A, A, rows=rows, with_scale=False, threads=threads)
        return time.perf_counter() - t
    # pilot: a sparse sample, single-threaded
    stride = max(1, A.rows // 512)
    rows = sample(stride)
    el = run(rows, 1)
    rate = max(float(nprod[rows].sum()), 1.0) / max(el, 1e-3)      # products per second
    want = rate * seconds
    stride = int(max(1, min(A.rows, np.ceil(tot / max(want, 1.0)))))
    rows = sample(stride)
    prod = int(nprod[rows].sum())
    t1 = run(rows, 1)
    threads = oracle.host_threads()
    tn = run(rows, threads)
    g1 = 2.0 * prod / t1 / 1e9
    gn = 2.0 * prod / tn / 1e9
    log(f"cpu oracle: {rows.size} rows ({prod} products): 1 thread {t1:.1f}s {g1:.3f} GFLOPS; "
        f"{threads} threads {tn:.1f}s {gn:.3f} GFLOPS")
    return {"value": round(gn, 4), "unit": "GFLOPS", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}-th row in n_prod order ({rows.size} rows, {prod} of {tot} "
                      f"products), C oracle (symbolic + numeric), row-parallel on {threads} threads",
            "single_thread": {"value": round(g1, 4), "seconds": round(t1, 2)},
            "seconds": round(tn, 2), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--mode", default="plain",
                    choices=["plain", "batched", "learned", "copy", "ablation", "lds"],
                    help="plain: the headline product; batched: 512 uneven products as one "
                         "batch vs 512 plain calls; learned: one-phase product with the trained "
                         "predictor vs the plain two-phase product and the upper-bound rule")
    ap.add_argument("--count", type=int, default=512, help="problems in the batched mode")
    ap.add_argument("--batch-only", action="store_true",
                    help="batched mode: time the tuned batch alone (no built-in configuration, "
                         "no separate plain calls), e.g. under a kernel trace")
    ap.add_argument("--workloads", default="st27_100,bst27_40,band21,rmat20",
                    help="ablation mode: workloads of the tables")
    ap.add_argument("--out", default="", help="ablation mode: also write the tables (markdown) here")
    ap.add_argument("--fp32", default="st27_100",
                    help="plain mode: workload also timed with FP32 values ('' = none)")
    ap.add_argument("--panel", default="", help="learned mode: 'k/P' = the k-th of P row panels "
                                                 "of equal n_prod (for products beyond HBM)")
    ap.add_argument("--no-learned", action="store_true",
                    help="plain mode: skip the one-phase comparison on the same workload")
    ap.add_argument("--no-tuning", action="store_true",
                    help="plain mode: use the built-in bin configuration instead of the "
                         "autotuned one of the workload's class")
    ap.add_argument("--secondary", default="st27_100,bst27_40",
                    help="plain mode: comma-separated workloads reported beside the headline "
                         "('' = none)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "row-panel design is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synthetic as syn
    import paper_2206_07244_amd as ops

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.mode == "batched":
        return bench_batched(args, dev)
    if args.mode == "learned":
        return bench_learned(args, dev)
    if args.mode == "copy":
        return bench_copy(args, dev)
    if args.mode == "ablation":
        return bench_ablation(args, dev)
    if args.mode == "lds":
        return bench_lds(args, dev)

    r = measure_plain(ops, torch, np, syn, args.workload, args.steps, args.warmup, dev,
                      tuned_cls=not args.no_tuning)
    A, dA = r["A"], r.pop("dA")
    nprod, nnzC, ms = r["nprod"], r["nnzC"], r["ms"]
    st = r["stage"]
    out = {
        "metric": METRIC,
        "value": round(r["gflops"], 3),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": r["desc"], "rows": A.rows, "nnzA": A.nnz,
                   "nprod": nprod, "nnzC": nnzC, "path": "plain two-pass",
                   "bins": f"autotuned ({r['cls']})" if r["tuned"] else "built-in"},
        "roofline": r["roofline"],
        "stage_ms": {"setup_bin": round(st[0], 4), "symbolic": round(st[1], 4),
                     "numbin_scan_alloc": round(st[2], 4), "numeric": round(st[3], 4),
                     "total": round(st[4], 4), "long_row_numeric_kernel": round(st[5], 4)},
    }
    if r["ms_default"] is not None:
        out["builtin_config"] = {"value": round(2.0 * nprod / (r["ms_default"] * 1e-3) / 1e9, 3),
                                 "ms_per_step": round(r["ms_default"], 4)}

    def release():
        # C and the staging of the workload just timed stay in the library's
        # cache; hand them back before the next leg allocates
        torch.cuda.synchronize()
        ops.cache_release()
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info()
        log(f"device memory after release: {free / 2**30:.1f} of {total / 2**30:.1f} GiB free; "
            f"library cache {ops.cache_bytes() / 2**30:.2f} GiB, held by callers "
            f"{ops.cache_live_bytes() / 2**30:.2f} GiB")

    if not args.no_learned and os.path.exists(ops.DEFAULT_WEIGHTS):
        release()
        pred = ops.Predictor.load(device=dev)
        try:
            rl = time_learned(ops, torch, dA, dA, pred, args.steps, args.warmup)
        except ops.OpspError as e:
            # the one-phase product holds its capacity arena, the staging
            # buffer and C at once; a product that does not fit that way is
            # reported, not timed
            if e.code != 3:   # OPSP_ERR_ALLOC
                raise
            torch.cuda.synchronize()
            out["learned"] = {"skipped": f"one-phase product does not fit in device memory ({e})"}
            log(f"learned one-phase: skipped, {e}")
            # such products run the one-phase form by row panels: compare
            # the first of LEARNED_PANELS panels of equal n_prod (a zero-copy
            # view of A's rows) in both forms, with the built-in bins
            release()
            _, npd, _ = ops.row_features(dA, dA)
            cum = np.cumsum(npd.cpu().numpy())
            r1 = int(np.searchsorted(cum, int(cum[-1]) / LEARNED_PANELS, side="right"))
            view = ops.DeviceCSR(r1, dA.cols, dA.rpt[:r1 + 1], dA.col, dA.val)
            steps_p = min(args.steps, 5)
            ms_p, stp = time_plain(ops, torch, view, dA, steps_p, 1)
            release()
            rlp = time_learned(ops, torch, view, dA, pred, steps_p, 1)
            del view
            out["learned"]["panel"] = {
                "panel": f"0/{LEARNED_PANELS}", "rows": [0, r1], "nprod": stp.nprod, "steps": steps_p,
                "plain_ms": round(ms_p, 4), "learned_ms": round(rlp["ms"], 4),
                "speedup_vs_plain": round(ms_p / rlp["ms"], 4), **rlp["stats"]}
            log(f"learned one-phase on row panel 0/{LEARNED_PANELS} (rows [0, {r1})): {rlp['ms']:.3f} ms "
                f"against {ms_p:.3f} ms plain ({ms_p / rlp['ms']:.3f}x)")
        else:
            out["learned"] = {"value": round(2.0 * nprod / (rl["ms"] * 1e-3) / 1e9, 3),
                              "ms_per_step": round(rl["ms"], 4),
                              "speedup_vs_plain": round(ms / rl["ms"], 4), **rl["stats"]}
            log(f"learned one-phase: {rl['ms']:.3f} ms/step ({ms / rl['ms']:.3f}x plain)")

    others = [w for w in args.secondary.split(",") if w and w != args.workload]
    if others:
        del dA
        out["secondary"] = []
    for w in others:
        release()
        r2 = measure_plain(ops, torch, np, syn, w, args.steps, args.warmup, dev,
                           tuned_cls=not args.no_tuning, builtin=False)
        out["secondary"].append({"workload": w, "description": r2["desc"],
                                 "value": round(r2["gflops"], 3), "unit": "GFLOPS",
                                 "ms_per_step": round(r2["ms"], 4), "nprod": r2["nprod"],
                                 "nnzC": r2["nnzC"], "roofline": r2["roofline"],
                                 "stage_ms": {k: round(float(v), 4) for k, v in
                                              zip(["setup_bin", "symbolic", "numbin_scan_alloc",
                                                   "numeric", "total"], r2["stage"][:5])}})
        del r2

    if args.fp32:
        release()
        out["fp32"] = time_fp32(ops, torch, np, syn, args.fp32, args.steps, args.warmup, dev,
                                tuned_cls=not args.no_tuning)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, np, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def bench_ablation(args, dev):
    """The paper's ablations (Section 6.3) on one MI355X, with every row taken
    by the hash tables as in the paper (config.hash_all_rows):
      hashing  the symbolic and numeric steps with the single-access probe
               (one compare-and-swap per probe, the product library) and the
               multiple-access probe (read, then swap: the library variant
               built with OPSP_HASH_MULTI_ACCESS), Section 6.3.2;
      ranges   the symbolic step at binning ratios 1, 1.2, 1.5 and the numeric
               step at 1, 1.5, 2, 3 (Section 6.3.3; ratio r puts a row in the
               first table at least r times its n_prod or nnz);
      binning  the share of the binning kernels in the whole product, with the
               setup kernel (into which the first binning pass is fused)
               reported apart (Section 6.3.1), for the paper's hashing and for
               this library's default (range bitmaps and dense rows).
    Stage times are HIP events on the calling stream, mean of --steps calls
    after --warmup."""
    import ctypes
    import numpy as np
    import torch
    import synthetic as syn
    import paper_2206_07244_amd as ops

    sh = torch.cuda.current_stream().cuda_stream
    variants = {"single": ops.lib(), "multi": ops.lib_variant("multi_access")}

    def stages(L, Ac, cfg):
        acc = np.zeros(8)
        for k in range(args.warmup + args.steps):
            Cc = ops.opsp_csr()
            st = ops.Stats()
            cfg.stage_timing = 1
            code = L.opsp_spgemm_ex(ctypes.byref(Ac), ctypes.byref(Ac), ctypes.byref(Cc),
                                    ctypes.byref(cfg), ctypes.byref(st), sh)
            if code:
                raise ops.OpspError(code, "opsp_spgemm_ex")
            code = L.opsp_csr_free(ctypes.byref(Cc), sh)
            if k >= args.warmup:
                acc += np.array(list(st.ms_stage))
        torch.cuda.synchronize()
        # each library keeps its own cache: hand it back before the next
        # configuration (the R-MAT product needs most of the device)
        L.opsp_cache_release()
        return acc / args.steps

    res = {}
    for w in [x for x in args.workloads.split(",") if x]:
        desc, builder = syn.WORKLOADS[w]
        A = builder()
        dA = ops.DeviceCSR.from_host(A, dev)
        Ac = dA._c_fast(A.nnz)
        r = {"description": desc}
        for name, L in variants.items():
            s_ = stages(L, Ac, ops.Config(hash_all_rows=1))
            r[f"hash_{name}"] = {"symbolic_ms": round(s_[1], 4), "numeric_ms": round(s_[3], 4),
                                 "total_ms": round(s_[4], 4)}
            log(f"{w} hashing {name}: sym {s_[1]:.3f} num {s_[3]:.3f} total {s_[4]:.3f} ms")
        r["sym_ratio"] = {}
        for q in (1.0, 1.2, 1.5):
            s_ = stages(variants["single"], Ac, ops.Config(hash_all_rows=1, sym_ratio=q))
            r["sym_ratio"][str(q)] = round(s_[1], 4)
        r["num_ratio"] = {}
        for q in (1.0, 1.5, 2.0, 3.0):
            s_ = stages(variants["single"], Ac, ops.Config(hash_all_rows=1, num_ratio=q))
            r["num_ratio"][str(q)] = round(s_[3], 4)
        log(f"{w} ranges: sym {r['sym_ratio']} num {r['num_ratio']}")
        for tag, cfg in (("paper_hashing", ops.Config(hash_all_rows=1)), ("default", ops.Config())):
            s_ = stages(variants["single"], Ac, cfg)
            setup = s_[6]
            binning = (s_[0] - s_[6]) + s_[2]
            r[f"binning_{tag}"] = {"setup_ms": round(setup, 4), "binning_ms": round(binning, 4),
                                   "total_ms": round(s_[4], 4),
                                   "binning_share": round(binning / s_[4], 4),
                                   "setup_and_binning_share": round((setup + binning) / s_[4], 4)}
        res[w] = r
        del dA, Ac, A
        torch.cuda.synchronize()
        ops.cache_release()
        torch.cuda.empty_cache()

    out = {"mode": "ablation", "steps": args.steps, "warmup": args.warmup, "workloads": res}
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(ablation_markdown(res))


def ablation_markdown(res) -> str:
    """The three ablation tables of bench_ablation as markdown."""
    L = ["### Hashing: single- vs multiple-access probe (Section 6.3.2; every row hashed)", "",
         "| workload | symbolic single ms | symbolic multi ms | speedup | numeric single ms | "
         "numeric multi ms | speedup |", "|---|---|---|---|---|---|---|"]
    for w, r in res.items():
        a, b = r["hash_single"], r["hash_multi"]
        L.append(f"| {w} | {a['symbolic_ms']:.3f} | {b['symbolic_ms']:.3f} | "
                 f"{b['symbolic_ms'] / a['symbolic_ms']:.3f} | {a['numeric_ms']:.3f} | "
                 f"{b['numeric_ms']:.3f} | {b['numeric_ms'] / a['numeric_ms']:.3f} |")
    L += ["", "### Binning ranges (Section 6.3.3; every row hashed): step time and speedup over ratio 1",
          "", "| workload | Sym_1x ms | Sym_1.2x | Sym_1.5x | Num_1x ms | Num_1.5x | Num_2x | Num_3x |",
          "|---|---|---|---|---|---|---|---|"]
    for w, r in res.items():
        sr, nr = r["sym_ratio"], r["num_ratio"]
        s1, n1 = sr["1.0"], nr["1.0"]
        L.append(f"| {w} | {s1:.3f} | {sr['1.2']:.3f} ({s1 / sr['1.2']:.2f}x) | "
                 f"{sr['1.5']:.3f} ({s1 / sr['1.5']:.2f}x) | {n1:.3f} | "
                 f"{nr['1.5']:.3f} ({n1 / nr['1.5']:.2f}x) | {nr['2.0']:.3f} ({n1 / nr['2.0']:.2f}x) | "
                 f"{nr['3.0']:.3f} ({n1 / nr['3.0']:.2f}x) |")
    L += ["", "### Binning share of the whole product (Section 6.3.1)", "",
          "| workload | configuration | setup kernel ms | binning kernels ms | total ms | "
          "binning share | setup + binning share |", "|---|---|---|---|---|---|---|"]
    for w, r in res.items():
        for tag in ("paper_hashing", "default"):
            b = r[f"binning_{tag}"]
            L.append(f"| {w} | {tag.replace('_', ' ')} | {b['setup_ms']:.3f} | {b['binning_ms']:.3f} | "
                     f"{b['total_ms']:.3f} | {100 * b['binning_share']:.2f} % | "
                     f"{100 * b['setup_and_binning_share']:.2f} % |")
    return "\n".join(L) + "\n"


def bench_lds(args, dev):
    """Rate of the LDS atomics the hash and dense kernels issue (the second
    ceiling beside HBM): lane operations per CU per clock at the 2.4 GHz
    peak engine clock, for ds_add_f64, ds_cmpst_rtn_b32, ds_or_b32 and ds_add_f32 with
    lane-consecutive and pseudo-random addresses in a 64 KB table, 512-thread
    workgroups, two per CU (microbench/lds_atomics.hip)."""
    import ctypes
    import torch
    from paper_2206_07244_amd import _build
    L = ctypes.CDLL(_build.MICROBENCH_LIB)
    L.opsp_mb_lds_atomics.restype = ctypes.c_int
    L.opsp_mb_lds_atomics.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_float)]
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    grid, iters, reps = cus * 8, 4096, 5
    res = {}
    for kind, kname in enumerate(["ds_add_f64", "ds_cmpst_rtn_b32", "ds_or_b32", "ds_add_f32"]):
        for pattern, pname in enumerate(["consecutive", "random"]):
            ms = ctypes.c_float()
            code = L.opsp_mb_lds_atomics(kind, pattern, grid, iters, reps, ctypes.byref(ms))
            if code:
                raise RuntimeError(f"microbenchmark failed: hipError {code}")
            ops_ = grid * 512 * iters
            rate = ops_ / (ms.value * 1e-3) / (2.4e9 * cus)
            res[f"{kname}/{pname}"] = {"ms": round(ms.value, 4), "lane_ops_per_cu_per_clock": round(rate, 3),
                                       "G_lane_ops_per_s": round(ops_ / (ms.value * 1e-3) / 1e9, 1)}
            log(f"{kname} {pname}: {ms.value:.3f} ms, {rate:.2f} lane ops per CU per clock")
    print(json.dumps({"mode": "lds", "cus": cus, "grid": grid, "threads": 512, "iters": iters,
                      "results": res}), flush=True)


def bench_copy(args, dev):
    """Calibration of the HBM byte counters: `steps` device-to-device copies
    of a 1 GiB buffer (1 GiB read + 1 GiB written per copy); the counters'
    reading for this run over the known bytes is the scale factor applied to
    the kernels' readings."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / args.steps
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n,
                      "copies": args.steps, "ms_per_copy": round(ms, 4),
                      "GBps": round(2 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)


# Row panels of equal n_prod for the one-phase comparison of a product that
# does not fit one GPU in one piece.
LEARNED_PANELS = 8


def time_learned(ops, torch, dA, dB, pred, steps, warmup):
    """ms per one-phase product (opsp_spgemm_learned, C allocated and freed
    inside the timed region) and the predictor statistics of one call."""
    sh = torch.cuda.current_stream().cuda_stream
    Ac, Bc = dA._c(), dB._c()
    ps = pred.struct()
    L = ops.lib()
    st = ops.Stats()

    def once(stats=None):
        C = ops.opsp_csr()
        code = L.opsp_spgemm_learned(ops.byref(Ac), ops.byref(Bc), ops.byref(C), ops.byref(ps),
                                     None, ops.byref(stats) if stats is not None else None, sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_learned")
        ops.free_raw(C, sh)
    once(st)
    for _ in range(max(warmup, 1)):
        once()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / steps
    cfg = ops.Config(stage_timing=1)
    C = ops.opsp_csr()
    s2 = ops.Stats()
    code = L.opsp_spgemm_learned(ops.byref(Ac), ops.byref(Bc), ops.byref(C), ops.byref(ps),
                                 ops.byref(cfg), ops.byref(s2), sh)
    if code:
        raise ops.OpspError(code, "opsp_spgemm_learned")
    ops.free_raw(C, sh)
    torch.cuda.synchronize()
    nnz = max(st.nnz, 1)
    return {"ms": ms, "stats": {
        "cap_over_nnz": round(st.cap_total / nnz, 4),
        "slot_overflow_rows": st.slot_overflow_rows, "table_overflow_rows": st.table_overflow_rows,
        "retry_rows": st.retry_rows, "arena_entries": st.arena_entries,
        "stage_ms": {"setup_caps_bins": round(s2.ms_stage[0], 4), "numeric": round(s2.ms_stage[1], 4),
                     "scan_retry_alloc": round(s2.ms_stage[2], 4), "copy": round(s2.ms_stage[3], 4),
                     "total": round(s2.ms_stage[4], 4)}}}


def time_plain(ops, torch, dA, dB, steps, warmup):
    sh = torch.cuda.current_stream().cuda_stream
    Ac, Bc = dA._c(), dB._c()
    st = ops.Stats()
    for i in range(max(warmup, 1)):
        Cc = ops.opsp_csr()
        code = ops.lib().opsp_spgemm_ex(ops.byref(Ac), ops.byref(Bc), ops.byref(Cc), None,
                                        ops.byref(st), sh)
        if code:
            raise ops.OpspError(code, "opsp_spgemm_ex")
        ops.free_raw(Cc, sh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        ops.free_raw(ops.spgemm_raw(Ac, Bc, sh), sh)
    torch.cuda.synchronize()
    return (time.perf_counter() - t1) * 1e3 / steps, st


def bench_learned(args, dev):
    """One-phase product with the trained predictor against the plain
    two-phase product and the upper-bound one-phase rule (cap = min(n_prod,
    N)), on the same inputs; optionally on one row panel of equal n_prod."""
    import numpy as np
    import torch
    import synthetic as syn
    import paper_2206_07244_amd as ops

    desc, builder = syn.WORKLOADS[args.workload]
    t0 = time.time()
    A = builder()
    log(f"workload {args.workload}: {A.rows} rows, {A.nnz} nnz ({time.time() - t0:.1f}s)")
    dA = ops.DeviceCSR.from_host(A, dev)
    dB = dA
    panel = None
    if args.panel:
        k, P = (int(x) for x in args.panel.split("/"))
        _, npd, _ = ops.row_features(dA, dA)
        cum = np.cumsum(npd.cpu().numpy())
        tot = int(cum[-1])
        r0 = int(np.searchsorted(cum, tot * k / P, side="right")) if k else 0
        r1 = int(np.searchsorted(cum, tot * (k + 1) / P, side="right")) if k + 1 < P else A.rows
        dA = ops.DeviceCSR(r1 - r0, A.cols, dA.rpt[r0:r1 + 1], dA.col, dA.val)
        panel = {"panel": args.panel, "rows": [r0, r1]}
        log(f"row panel {args.panel}: rows [{r0}, {r1})")
    del A
    pred = ops.Predictor.load(device=dev)
    ms_plain, st = time_plain(ops, torch, dA, dB, args.steps, args.warmup)
    nprod, nnzC = st.nprod, st.nnz
    log(f"plain: {ms_plain:.3f} ms, nprod={nprod}, nnz={nnzC}")
    rl = time_learned(ops, torch, dA, dB, pred, args.steps, args.warmup)
    log(f"learned: {rl['ms']:.3f} ms {rl['stats']}")
    ru = time_learned(ops, torch, dA, dB, ops.Predictor(ops.PRED_UPPER), args.steps, args.warmup)
    log(f"upper-bound rule: {ru['ms']:.3f} ms {ru['stats']}")
    gf = lambda t: round(2.0 * nprod / (t * 1e-3) / 1e9, 3)
    out = {
        "metric": METRIC,
        "value": gf(rl["ms"]),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rl["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "rows": dA.rows,
                   "nprod": nprod, "nnzC": nnzC, "path": "learned one-phase", **(panel or {})},
        "learned": {"ms_per_step": round(rl["ms"], 4), **rl["stats"]},
        "plain": {"value": gf(ms_plain), "ms_per_step": round(ms_plain, 4)},
        "upper_bound_rule": {"value": gf(ru["ms"]), "ms_per_step": round(ru["ms"], 4), **ru["stats"]},
        "speedup_vs_plain": round(ms_plain / rl["ms"], 4),
        "speedup_vs_upper_bound_rule": round(ru["ms"] / rl["ms"], 4),
    }
    print(json.dumps(out), flush=True)


def bench_batched(args, dev):
    """Batched products: `count` pairs A_i (n_i x n_i), B_i with n_i ~ U{1000..64000},
    Poisson(8) distinct uniform columns per row, N(0,1) values; one batch
    execution (two replayed graphs, one host read-back) per step, against the
    same products as `count` sequential plain calls."""
    import numpy as np
    import torch
    import synthetic as syn
    import paper_2206_07244_amd as ops

    t0 = time.time()
    pairs = syn.batch_pairs(args.count, seed=4)
    log(f"batch of {args.count} pairs generated in {time.time() - t0:.1f}s")
    dA = [ops.DeviceCSR.from_host(A, dev) for A, _ in pairs]
    dB = [ops.DeviceCSR.from_host(B, dev) for _, B in pairs]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    from paper_2206_07244_amd import autotune
    tuned = None if args.no_tuning else autotune.load_config("batch")

    def time_batch(cfg):
        """ms per execution of a batch created with `cfg` (graphs replayed)."""
        batch = ops.Batch(dA, dB, config=cfg, stream=stream)
        st = ops.Stats()
        batch.execute(stats=st)
        for _ in range(max(args.warmup, 1)):
            batch.raw_execute(sh)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            batch.raw_execute(sh)
        torch.cuda.synchronize()
        ms_ = (time.perf_counter() - t1) * 1e3 / args.steps
        del batch
        torch.cuda.synchronize()
        return ms_, st

    with torch.cuda.stream(stream):
        ms, st = time_batch(tuned)
        nprod, nnzC = st.nprod, st.nnz
        log(f"batched ({'tuned batch class' if tuned is not None else 'built-in'}): {ms:.3f} ms per "
            f"batch, nprod={nprod}, nnz={nnzC}")
        ms_builtin = None
        if tuned is not None and not args.batch_only:
            ms_builtin, _ = time_batch(None)
            log(f"batched (built-in configuration): {ms_builtin:.3f} ms per batch")

    def time_plain_calls():
        """ms for the same products as `count` separate plain calls."""
        Ac = [a._c_fast(a.nnz) for a in dA]
        Bc = [b._c_fast(b.nnz) for b in dB]
        for a, b in zip(Ac[:8], Bc[:8]):
            ops.free_raw(ops.spgemm_raw(a, b, sh), sh)
        torch.cuda.synchronize()
        reps = 2
        t3 = time.perf_counter()
        for _ in range(reps):
            for a, b in zip(Ac, Bc):
                ops.free_raw(ops.spgemm_raw(a, b, sh), sh)
        torch.cuda.synchronize()
        return (time.perf_counter() - t3) * 1e3 / reps

    ms_plain = None
    if not args.batch_only:
        with torch.cuda.stream(stream):
            ms_plain = time_plain_calls()
        log(f"{args.count} plain calls: {ms_plain:.3f} ms")
    gflops = 2.0 * nprod / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch{args.count}",
                   "description": "independent C_i = A_i B_i, n_i ~ U{1000..64000}, Poisson(8) "
                                  "rows, N(0,1) values, seed 4",
                   "nprod": nprod, "nnzC": nnzC, "path": "batched (two replayed graphs)",
                   "bins": "autotuned (batch)" if tuned is not None else "built-in"},
    }
    if ms_plain is not None:
        out["plain_calls_ms"] = round(ms_plain, 3)
        out["speedup_vs_plain_calls"] = round(ms_plain / ms, 3)
    if ms_builtin is not None:
        out["builtin_config"] = {"ms_per_step": round(ms_builtin, 4),
                                 "value": round(2.0 * nprod / (ms_builtin * 1e-3) / 1e9, 3),
                                 "tuned_speedup": round(ms_builtin / ms, 4)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
