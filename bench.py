#!/usr/bin/env python3
"""EmbedSOM projection throughput on one MI355X.

One step = one full pass of the projection path over one workload: landmark
preparation, the fused screen / exact selection / scores / pairs / 2x2-solve
kernel, and the exact FP64 path for the points it hands over.  Inputs are
resident in HBM before timing starts.  The headline workload is 1M x 32-D
points against 400 landmarks (20 x 20 grid), k = 16; its ``value`` is the BF16
screen + exact FP32 rescore mode, and the plain FP32 mode is reported beside
it.  The same line carries the 1M x 48-D / 1024-landmark / k = 20 workload and
the 10M x 64-D / 1024-landmark / k = 16 frame (both modes; the frame also runs
the k-means landmark update each step), the serving mix, and the FP64 CPU
oracle timed on the host cores.

Timing follows the paper's protocol (kernel time, repeated runs, relative
standard deviation): HIP events are recorded between consecutive steps on
the launching stream, giving per-step times (median, mean, RSD); ``value``
is N over the mean step time of the K steps bracketed by synchronisations.
Before the first mode's warmup steps, the projection runs untimed for
--settle seconds: the GPU's clocks take a few tens of milliseconds under load
to reach their steady state.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/s at 1M×32D, 400 landmarks, k=16: FP32 vs BF16+rescore; p99 latency"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
MFMA_FP32_PEAK_TFLOPS = 157.3
VALU_FP32_PEAK_TFLOPS = 157.3          # published (packed FP32 issue)
VALU_FP32_NONPACKED_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
COORD_TOL = 1e-4

WORKLOADS = {"c2": "c2_fp32_1m", "c3": "c3_bf16_1m", "c4": "c4_large_10m"}
# the tag of each workload's rocprofv3 summaries in profiles/
PROFILE_TAG = {"c2_fp32_1m": "c2_1m", "c3_bf16_1m": "c3_1m", "c4_large_10m": "c4_10m"}


def alu_flops_per_point(g, d, k, cands):
    """Algorithmic VALU work per point of the screened path: one compare per
    screened key, an exact rescore (subtract, multiply, add) of `cands`
    candidates (the design's minimum, k + 2), and about 30 flops per active
    landmark pair (polarised segment projection and the 2x2 accumulation)."""
    return g + 3.0 * cands * d + 30.0 * (k - 1) * (k - 2) / 2.0


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("embed_kernel.h", "embed_inst.hip", "esom_core.hip", "esom_internal.h"):
        with open(os.path.join(ROOT, "paper_2201_00701_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode, workload):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, or None when there is
    none or the kernel sources have changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "embed_main_%s_hbm_counters.txt" % PROFILE_TAG.get(workload, workload))
    try:
        kv = dict(l.split(": ", 1) for l in open(path).read().splitlines()
                  if ": " in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    v = kv.get("traffic_bytes_" + mode)
    return float(v) if v is not None else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(n or 1, 16))


def cpu_baseline_leg(w, rows, one_core_rows=0):
    """The FP64 CPU oracle on a seeded sample of the workload's points, timed on
    all host cores (and on one core for the first `one_core_rows` of the
    sample).  Returns the timing and the oracle's outputs for the sample, which
    the error fields compare the GPU outputs with."""
    import oracle
    oracle.build(force=False)
    threads = host_threads()
    Xs = w.X[rows]
    t = time.perf_counter()
    ref = oracle.embed(Xs, w.L, w.l, w.k, threads=threads)
    dt = time.perf_counter() - t
    res = {"value": len(rows) / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "%d seeded points of the %d (%s), FP64 C oracle, %.2f s wall on %d threads"
                     % (len(rows), len(w.X), w.name, dt, threads)}
    if one_core_rows:
        t = time.perf_counter()
        oracle.embed(Xs[:one_core_rows], w.L, w.l, w.k, threads=1)
        dt1 = time.perf_counter() - t
        res["value_1core"] = one_core_rows / dt1
        res["sample_1core"] = "first %d of that sample, %.2f s wall on 1 thread" % (one_core_rows, dt1)
    return res, ref


def errors_vs_oracle(out_rows, idx_rows, ref, w):
    """Max / mean coordinate error against the FP64 oracle on the sampled rows,
    and neighbour-set mismatches outside the oracle's near ties."""
    import numpy as np
    err = np.abs(out_rows.astype(np.float64) - ref["out"]).max(axis=1)
    k = w.k
    res = {"max_abs": float(err.max()), "mean_abs": float(err.mean()),
           "tol": COORD_TOL * w.span, "points": int(len(err))}
    if idx_rows is not None:
        dk, dk1 = np.sqrt(ref["d2"][:, k - 1]), np.sqrt(ref["d2"][:, k])
        tie = (dk1 - dk) < 1e-6 * dk1
        same = np.all(np.sort(idx_rows, 1) == np.sort(ref["idx"][:, :k], 1), axis=1)
        res["set_mismatch"] = int(np.sum(~same & ~tie))
        res["near_ties"] = int(tie.sum())
    return res


def time_steps(torch, step, steps):
    """Runs `steps` steps with an event between consecutive ones on the current
    stream; returns (total ms between synchronisations, per-step ms list)."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]), per


def step_stats(per):
    import numpy as np
    a = np.array(per)
    return {"ms_step_median": float(np.median(a)), "ms_step_mean": float(a.mean()),
            "rsd_pct": float(100.0 * a.std(ddof=1) / a.mean()) if len(a) > 1 else 0.0}


def roofline_for(mode, n, g, d, k, ms_main, st, workload):
    import math
    gpad = 64 * math.ceil(g / 64)
    dpad = 16 * math.ceil(d / 16)
    traffic = measured_traffic(mode, workload)
    if mode == "fp32":
        ach = 2.0 * n * g * d / (ms_main * 1e-3) / 1e12
        # FP32 MFMA runs the candidate pass (the threshold pass is BF16), over
        # the padded landmark and dimension counts
        issued = 2.0 * n * gpad * dpad / (ms_main * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / MFMA_FP32_PEAK_TFLOPS, "traffic": traffic,
                "issued_tflops": issued, "issued_frac": issued / MFMA_FP32_PEAK_TFLOPS}
    cands = st["n_candidates"] / max(st["n_points"], 1)
    ach = alu_flops_per_point(g, d, k, k + 2) * n / (ms_main * 1e-3) / 1e12
    mf = 2.0 * n * g * d / (ms_main * 1e-3) / 1e12
    # BF16 MFMA issued: the threshold pass and the split candidate pass (three
    # products per element), over the padded counts
    mfi = 4.0 * 2.0 * n * gpad * dpad / (ms_main * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / VALU_FP32_PEAK_TFLOPS, "traffic": traffic,
            "peak_nonpacked": VALU_FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": ach / VALU_FP32_NONPACKED_TFLOPS,
            "mfma_bf16_tflops": mf, "mfma_bf16_frac": mf / MFMA_BF16_PEAK_TFLOPS,
            "mfma_bf16_issued_tflops": mfi, "mfma_bf16_issued_frac": mfi / MFMA_BF16_PEAK_TFLOPS,
            "candidates_per_point": cands}


def run_workload(torch, esom, w, modes, args, frame_update=False, keep_rows=None):
    """Times each mode on workload w; returns per-mode results (and, when
    keep_rows is given, the GPU outputs and neighbours of those rows)."""
    import numpy as np
    n, d = w.X.shape
    g, k = len(w.L), w.k
    X = torch.from_numpy(w.X).cuda()
    L0 = torch.from_numpy(w.L).cuda()
    L = L0.clone()
    l = torch.from_numpy(w.l).cuda()
    out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    knn = torch.empty((n, k), dtype=torch.int32, device="cuda") if frame_update else None
    cnt = torch.empty(g, dtype=torch.int32, device="cuda") if frame_update else None
    ctx = esom.Context(0)
    ctx.set_timing(True)
    results, kept = {}, {}
    t_settle = time.time()
    while time.time() - t_settle < args.settle:
        ctx.embed(X, L, l, k=k, mode=modes[0], out=out)
        torch.cuda.synchronize()
    for mode in modes:
        def embed_step():
            ctx.embed(X, L, l, k=k, mode=mode, out=out)

        def frame_step():
            # every frame starts from the same landmarks, so all steps do equal work
            L.copy_(L0)
            esom.esom_embed(ctx.handle, X.data_ptr(), n, d, d, L.data_ptr(), l.data_ptr(), g,
                            esom.esom_default_params(k=k, mode=mode), out.data_ptr(),
                            knn.data_ptr(), 0, torch.cuda.current_stream().cuda_stream)
            esom.esom_landmark_update(ctx.handle, X.data_ptr(), n, d, d, L.data_ptr(), l.data_ptr(),
                                      g, 0, 0.1, 0.0, knn.data_ptr(), k, cnt.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)

        for _ in range(args.warmup):
            embed_step()
        torch.cuda.synchronize()
        ctx.stats(reset=True)
        ms_total, per = time_steps(torch, embed_step, args.steps)
        st = ctx.stats(reset=True)
        ms_step = ms_total / args.steps
        ms_main = st["ms_main"] / max(st["n_timed"], 1)
        res = {"value": n / (ms_step * 1e-3), "unit": "points/s", "ms_per_step": ms_step}
        res.update(step_stats(per))
        res.update({"ms_prep": st["ms_prep"] / max(st["n_timed"], 1), "ms_main_kernel": ms_main,
                    "ms_exact_path": st["ms_exact"] / max(st["n_timed"], 1),
                    "exact_path_points_per_step": st["n_fallback"] / args.steps,
                    "candidates_per_point": st["n_candidates"] / max(st["n_points"], 1),
                    "hbm_gbs_main": (4.0 * d + 8.0) * n / (ms_main * 1e-3) / 1e9})
        res["roofline"] = roofline_for(mode, n, g, d, k, ms_main, st, w.name)
        if keep_rows is not None:
            kept[mode] = out.cpu().numpy()[keep_rows]
        if frame_update:
            # the frame: embed with the neighbour list, then the k-means update
            # (alpha 0.1) reusing each point's nearest landmark
            for _ in range(2):
                frame_step()
            torch.cuda.synchronize()
            ctx.stats(reset=True)
            fsteps = max(3, args.steps // 2)
            ms_f, perf = time_steps(torch, frame_step, fsteps)
            ctx.stats(reset=True)
            fr = {"ms_per_frame": ms_f / fsteps, "points_per_s": n / (ms_f / fsteps * 1e-3),
                  "update": "k-means, alpha 0.1, nearest landmark reused from the embed"}
            fr.update(step_stats(perf))
            # the update alone
            L.copy_(L0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            near = knn[:, 0]
            e0.record()
            for _ in range(fsteps):
                ctx.landmark_update(X, L, l, kind="kmeans", alpha=0.1, nearest=near)
            e1.record()
            torch.cuda.synchronize()
            fr["ms_update"] = e0.elapsed_time(e1) / fsteps
            L.copy_(L0)
            res["frame"] = fr
        results[mode] = res
        print("bench: %s mode %s %.3f ms/step (median %.3f, RSD %.2f%%; main kernel %.3f ms) %.3g points/s"
              % (w.name, mode, ms_step, res["ms_step_median"], res["rsd_pct"], ms_main, res["value"]),
              file=sys.stderr, flush=True)
    ctx.close()
    del X, L, L0, l, out, knn
    torch.cuda.empty_cache()
    return results, kept


def ablations(torch, esom, synth, reps=3):
    """The paper's kernel families (k-NN Base / Shared / GridInsert / Bitonic,
    projection Base / Shared / Aligned / Registers) beside the fused kernel on
    the paper-shaped workload: n = 2^20 points uniform on [0, 1)^d, d in
    {16, 32}, 256 landmarks (16 x 16 grid), k = 16.  Milliseconds per call from
    HIP events (the median of `reps` calls after one warm-up call)."""
    import numpy as np
    res = {}
    for d in (16, 32):
        w = synth.paper_shaped(d)
        n = len(w.X)
        X = torch.from_numpy(w.X).cuda()
        L = torch.from_numpy(w.L).cuda()
        l = torch.from_numpy(w.l).cuda()
        k = w.k

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return float(np.median(ts))

        ctx = esom.Context(0)
        out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        r = {"n": n, "d": d, "g": len(w.L), "k": k,
             "fused_fp32_ms": timed(lambda: ctx.embed(X, L, l, k=k, mode="fp32", out=out)),
             "fused_bf16_ms": timed(lambda: ctx.embed(X, L, l, k=k, mode="bf16", out=out))}
        ctx.close()
        knn, proj = {}, {}
        for algo in ("base", "shared", "gridinsert", "bitonic"):
            knn[algo] = timed(lambda: esom.ablation_knn(algo, X, L, k))
        idx, d2 = esom.ablation_knn("bitonic", X, L, k)
        for algo in ("base", "shared", "aligned", "registers"):
            proj[algo] = timed(lambda: esom.ablation_project(algo, X, L, l, idx, d2, out=out))
        r["knn_ms"] = knn
        r["projection_ms"] = proj
        best = min(knn.values()) + min(proj.values())
        r["best_pair_ms"] = best
        r["fused_fp32_points_per_s"] = n / (r["fused_fp32_ms"] * 1e-3)
        r["best_pair_points_per_s"] = n / (best * 1e-3)
        res["paper_uniform_d%d" % d] = r
        print("bench: ablations d=%d: fused fp32 %.3f ms, bf16 %.3f ms; knn %s; projection %s"
              % (d, r["fused_fp32_ms"], r["fused_bf16_ms"],
                 ", ".join("%s %.3f" % kv for kv in knn.items()),
                 ", ".join("%s %.3f" % kv for kv in proj.items())), file=sys.stderr, flush=True)
        del X, L, l, out, idx, d2
        torch.cuda.empty_cache()
    return res


def serve_mix(n_requests=2000, warmup=200, rate=200.0, budget=8 << 30, slots=4, seed=5,
              base_n=1_000_000):
    """Serving mix: Poisson arrivals; N log-uniform in [1e3, 1e6]; D in {16, 32, 48};
    g in {100, 400, 1024} (10x10, 20x20, 32x32 grids); k in {8, 16, 20}; 10% of the
    requests re-embed a resident dataset after moving 1-5 of its 2-D landmarks by
    N(0, 0.5^2).  New points are uploaded from pinned host memory within the
    request.  Latency = result in host memory minus scheduled arrival."""
    import threading

    import numpy as np
    import torch

    from paper_2201_00701_amd import esom, synth

    rng = np.random.default_rng(seed)
    Ds, Gs, Ks = (16, 32, 48), (100, 400, 1024), (8, 16, 20)
    grid = {100: 10, 400: 20, 1024: 32}
    base, LM = {}, {}
    for D in Ds:
        X = synth.mixture(base_n, D, 30, seed=seed * 100 + D)
        pin = torch.empty((base_n, D), dtype=torch.float32, pin_memory=True).numpy()
        pin[:] = X
        base[D] = pin
        for g in Gs:
            LM[(D, g)] = synth.landmarks_from_data(X, g, seed=seed * 100 + D + g)
    srv = esom.Server(0, budget, slots)
    resident = {}
    for D in Ds:
        g = int(rng.choice(Gs))
        k = int(rng.choice(Ks))
        n = 100_000
        resident[D] = {"id": srv.put(np.ascontiguousarray(base[D][:n])), "g": g, "k": k, "n": n,
                       "l": synth.grid2d(g, grid[g]).copy(),
                       "out": np.empty((n, 2), np.float32)}
    total = warmup + n_requests
    arrivals = np.cumsum(rng.exponential(1.0 / rate, total))
    plan = []
    for i in range(total):
        if rng.random() < 0.1:
            D = int(rng.choice(Ds))
            plan.append(("edit", D, int(rng.integers(1, 6))))
        else:
            N = int(round(np.exp(rng.uniform(np.log(1e3), np.log(1e6)))))
            plan.append(("new", int(rng.choice(Ds)), int(rng.choice(Gs)), int(rng.choice(Ks)), N,
                         int(rng.integers(0, base_n - N + 1))))
    rids = [None] * total
    infos = [None] * total
    outs = {}
    done_evt = threading.Event()

    def waiter():
        for i in range(total):
            while rids[i] is None:
                time.sleep(0.0002)
            infos[i] = srv.wait(rids[i], -1)
        done_evt.set()

    th = threading.Thread(target=waiter, daemon=True)
    off = srv.stats()["now_ms"] - time.perf_counter() * 1e3
    t_start = time.perf_counter() + 0.05
    th.start()
    for i, item in enumerate(plan):
        t_arr = t_start + arrivals[i]
        while True:
            dt = t_arr - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.001))
        if item[0] == "edit":
            _, D, m = item
            r = resident[D]
            moved = rng.choice(r["g"], m, replace=False)
            r["l"][moved] += rng.normal(0, 0.5, (m, 2)).astype(np.float32)
            rids[i] = srv.submit(LM[(D, r["g"])], np.ascontiguousarray(r["l"]), k=r["k"],
                                 mode="bf16", dataset=r["id"], out=r["out"])
        else:
            _, D, g, k, N, o = item
            X = base[D][o:o + N]
            outs[i] = np.empty((N, 2), np.float32)
            rids[i] = srv.submit(LM[(D, g)], synth.grid2d(g, grid[g]), k=min(k, g), mode="bf16",
                                 X=X, out=outs[i])
    done_evt.wait()
    st = srv.stats()
    srv.close()
    lat, pts = [], 0
    for i in range(warmup, total):
        lat.append(infos[i]["done_ms"] - ((t_start + arrivals[i]) * 1e3 + off))
        pts += infos[i]["n"]
    lat = np.array(lat)
    first = (t_start + arrivals[warmup]) * 1e3 + off
    last = max(infos[i]["done_ms"] for i in range(warmup, total))
    return {"requests": n_requests, "warmup_requests": warmup, "rate_req_s": rate,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "points_per_s": pts / ((last - first) * 1e-3),
            "cache_hits": int(sum(infos[i]["cache_hit"] for i in range(warmup, total))),
            "graph_replays": int(sum(infos[i]["graph_replay"] for i in range(warmup, total))),
            "slots": slots, "budget_gib": budget / float(1 << 30), "peak_gib": st["peak_bytes"] / float(1 << 30),
            "admission_waits": int(st["admission_waits"]), "max_queued": int(st["max_queued"]),
            "rejected": int(st["rejected"]), "failed": int(st["failed"]), "mode": "bf16"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle", type=float, default=0.3,
                    help="seconds of untimed projection before the warmup steps (clock ramp)")
    ap.add_argument("--workloads", default="c2,c3,c4",
                    help="comma list of c2 (headline), c3, c4; the first is the headline")
    ap.add_argument("--modes", default="bf16,fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the paper's kernel families on the paper-shaped workload")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--tight-budget-mib", type=int, default=384,
                    help="HBM budget of the second serving run (admission binds)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (the reference kernel for "
                         "scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the projection is data-parallel over points, and the "
              "library runs on a single MI355X (how it would shard is a design note, not code); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_00701_amd import esom, synth

    modes = args.modes.split(",")
    names = [WORKLOADS[x] for x in args.workloads.split(",")]
    per_workload = {}
    for wi, name in enumerate(names):
        t0 = time.time()
        w = synth.make(name)
        n, d = w.X.shape
        print("bench: workload %s n=%d d=%d g=%d k=%d (generated in %.1f s)"
              % (name, n, d, len(w.L), w.k, time.time() - t0), file=sys.stderr, flush=True)
        rows = None
        if not args.no_cpu_baseline:
            rows = np.arange(n) if n <= 1_000_000 else synth.subsample(n, 1_000_000, seed=19)
        res, kept = run_workload(torch, esom, w, modes, args, frame_update=(name == "c4_large_10m"),
                                 keep_rows=rows)
        if rows is not None:
            cpu, ref = cpu_baseline_leg(w, rows, one_core_rows=200_000 if wi == 0 else 0)
            for mode in modes:
                res[mode]["error_vs_oracle"] = errors_vs_oracle(kept[mode], None, ref, w)
            res["cpu_baseline"] = cpu
            print("bench: %s oracle %.3g points/s on %d threads; max error %s"
                  % (name, cpu["value"], cpu["cores"],
                     ", ".join("%s %.3g" % (m, res[m]["error_vs_oracle"]["max_abs"]) for m in modes)),
                  file=sys.stderr, flush=True)
        res["config"] = "N=%d, D=%d, L=%d (%d x %d grid), k=%d" % (
            n, d, len(w.L), int(round(len(w.L) ** 0.5)), int(round(len(w.L) ** 0.5)), w.k)
        per_workload[name] = res
        del w, kept

    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    head_name = names[0]
    hw = per_workload[head_name]
    head = "bf16" if "bf16" in modes else modes[0]
    line = {
        "metric": METRIC,
        "value": hw[head]["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hw[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s, %s" % (
            head_name, hw["config"], "BF16 screen + FP32 rescore" if head == "bf16" else "FP32"),
            "mode": head},
        "roofline": hw[head]["roofline"],
        "modes": {m: hw[m] for m in modes},
        "workloads": {nm: r for nm, r in per_workload.items() if nm != head_name},
    }
    if "cpu_baseline" in hw:
        line["cpu_baseline"] = hw["cpu_baseline"]
    if not args.no_ablations:
        line["ablations"] = ablations(torch, esom, synth)
    if not args.no_serve:
        print("bench: serving mix (%d requests)" % args.serve_requests, file=sys.stderr, flush=True)
        line["serving"] = serve_mix(n_requests=args.serve_requests)
        print("bench: serving p50 %.2f ms p99 %.2f ms, %d graph replays" % (
            line["serving"]["p50_ms"], line["serving"]["p99_ms"], line["serving"]["graph_replays"]),
              file=sys.stderr, flush=True)
        # the same mix under a budget small enough that admission waits for memory
        line["serving_tight_budget"] = serve_mix(n_requests=args.serve_requests,
                                                 budget=args.tight_budget_mib << 20)
        t = line["serving_tight_budget"]
        print("bench: serving (%d MiB budget) p50 %.2f ms p99 %.2f ms, %d admission waits, "
              "max queue %d" % (args.tight_budget_mib, t["p50_ms"], t["p99_ms"], t["admission_waits"],
                                t["max_queued"]), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
