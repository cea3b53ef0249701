"""Benchmark of the SwiftWRF render path on one MI355X.

Workload: N = 100,000 synthetic 2D Gaussians, 90 x 360 spectra (1 deg/px),
deformation MLP 89 -> 4 x 256 -> 7. A step renders one batch of B transmitter
positions end to end (PE -> MLP -> deform/preprocess -> scan -> keys -> radix
sort -> tile ranges -> blend) with the inputs resident in HBM. The headline
value is the batched throughput (spectra/s); the plain one-query-per-launch
FP32 path is timed beside it on the same GPU, and the oracle on the host CPU.

Prints one JSON line (see the repository's design notes for every field).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spectra/s at N=100k, 90x360 (batched vs plain); p50/p99 query latency us"
FLOP_PER_PAIR = 2 * (26 * 256 + 3 * 256 * 256 + 256 * 7)  # MLP per (query, Gaussian) pair
PEAK = {"bf16": 2500.0, "fp32": 157.3}  # dense MFMA TFLOP/s: BF16, FP32 (v_mfma_f32_16x16x4_f32)
FP32_VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # FP32 FMA TFLOP/s on the vector ALUs without packed instructions
HBM_PEAK_GBS = 8000.0
# FP32 lane-operations per second without FMA doubling or packing: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# VALU lane-op slots per (pixel, list entry) evaluation of the blend: 2 sub, 4 mul/fma (whitened offset), 2 (q),
# 1 compare, 1 mul + v_exp_f32 at quarter rate (4), 1 mul, 1 min, 1 compare, 2 (1 - a, T'), 1 compare, 2 (C), 1
# (index) ~ 20
BLEND_OPS_PER_EVAL = 20
# MLP kernel HBM bytes per pair that the algorithm needs: BF16 gamma(mu) (64 B) and 7 FP32 scene parameters (28 B)
# read, one 52 B pair record written; the weight stream is per tile and L2-resident.
MLP_ALGO_BYTES_PER_PAIR = 64 + 28 + 52
MLP_SOURCES = ("paper_2506_12787_amd/csrc/mlp_bf16.hip", "paper_2506_12787_amd/csrc/mlp_common.h",
               "paper_2506_12787_amd/csrc/swf_device.h")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mlp_bf16_n100k_90x360_b64_hbm_traffic.md")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--batch", type=int, default=64)
    p.add_argument("--n", type=int, default=100_000)
    p.add_argument("--height", type=int, default=90)
    p.add_argument("--width", type=int, default=360)
    p.add_argument("--mlp", choices=("bf16", "fp32"), default="bf16")
    p.add_argument("--plain-queries", type=int, default=16)
    p.add_argument("--fp32-steps", type=int, default=3,
                   help="timed batched steps with the FP32 MLP beside the BF16 headline (0: skip)")
    p.add_argument("--pairs-per-wave", type=int, default=0, help="BF16 MLP pairs per wave (48, the default, 32 or 64)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--quick", action="store_true", help="timed steps only (for profiler runs)")
    p.add_argument("--serve-requests", type=int, default=3000, help="requests per serving measurement")
    p.add_argument("--serve-sweep", action="store_true",
                   help="8 resident scenes, Poisson arrivals at a rate sweep (prints one JSON line per rate)")
    p.add_argument("--hbm-budget-gb", type=float, default=2.0,
                   help="serving sweep: bound on the transient workspace of all slots (GB), so admission binds")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="after the timed steps, run a plain FP32 copy kernel (x*1) over this many MiB three times: "
                        "the reference kernel that scales HBM byte counters")
    p.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                   help="summarise rocprofv3 counter CSVs (FETCH_SIZE / WRITE_SIZE runs of a --copy-probe-mib run) "
                        "into HBM bytes per launch of the MLP kernel, then exit")
    p.add_argument("--copy-mib", type=int, default=1024, help="copy size used by the counted run (for --pmc-summary)")
    p.add_argument("--pmc-table", nargs="+", metavar="DIR",
                   help="print mean counter values per dispatch of the kernels named by --kernels from these "
                        "rocprofv3 counter directories")
    p.add_argument("--kernels", default="mlp_bf16,bin_hist,bin_scatter,blend_forward",
                   help="comma-separated name fragments for --pmc-table")
    p.add_argument("--workload", choices=("headline", "large", "train", "beamscan", "rssi", "wrap", "protocol", "paper"), default="headline",
                   help="large: N=500k Gaussians (log-scales in [log 0.5, log 20] px), 360x1440 spectra, batch 256; "
                        "BF16 and FP32 MLP; prints its own JSON line (at most 5 timed steps, 1 warm-up). "
                        "train: training steps at N=50k, batch 16, 90x360 (forward with the blend state kept, L1 "
                        "loss, hand-written backward, Adam on Gaussians and MLP); prints its own JSON line. "
                        "beamscan: beam-scan spectra from multipath lists (batch 256, 90x360). rssi: the RSSI head "
                        "(16x16, 50 Gaussians, batch 1024). wrap: the headline batch with periodic azimuth. protocol: the "
                        "paper's training protocol (fine stage) with beam-scan targets. paper: the paper's own model (10k "
                        "Gaussians, GMM sum, 8x156 FP32 MLP, batch 64)")
    return p.parse_args()


def mlp_sources_hash():
    h = hashlib.sha256()
    for f in MLP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload_key(a):
    ppw = a.pairs_per_wave or 48
    return f"n{a.n}_h{a.height}_w{a.width}_b{a.batch}_{a.mlp}_ppw{ppw}"


def read_counters(dirs):
    """{(kernel name, counter): [value per dispatch]} from rocprofv3 counter-collection CSVs."""
    per = {}
    for d in dirs:
        for root, _, files in os.walk(d):
            for f in files:
                if not f.endswith("counter_collection.csv"):
                    continue
                with open(os.path.join(root, f), newline="") as fh:
                    for r in csv.DictReader(fh):
                        k = (r["Kernel_Name"], r["Counter_Name"])
                        disp = per.setdefault(k, {})
                        disp[(f, r["Dispatch_Id"])] = disp.get((f, r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def pmc_summary(a):
    """HBM bytes per launch of the MLP kernel from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by what
    the same counter reads for the plain copy kernel of known size run in the same process."""
    c = read_counters(a.pmc_summary)
    mean = lambda v: sum(v) / len(v)
    names = {k for k, _ in c}
    mlp = [n for n in names if f"mlp_{a.mlp}_kernel" in n]
    cp = [n for n in names if "elementwise" in n]
    if len(mlp) != 1 or not cp:
        sys.exit(f"pmc-summary: need one mlp_{a.mlp}_kernel and a copy kernel, found {sorted(names)}")
    mlp = mlp[0]
    # the probe is the elementwise kernel with the largest reads
    cp = max(cp, key=lambda n: mean(c.get((n, "FETCH_SIZE"), [0.0])))
    copy_bytes = a.copy_mib * 2 ** 20
    out = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        if (mlp, ctr) not in c or (cp, ctr) not in c:
            sys.exit(f"pmc-summary: counter {ctr} missing")
        kib_copy = mean(c[(cp, ctr)])
        kib_mlp = mean(c[(mlp, ctr)])
        scale = copy_bytes / (kib_copy * 1024.0)
        out[ctr] = {"mlp_kib_per_dispatch": kib_mlp, "mlp_dispatches": len(c[(mlp, ctr)]),
                    "copy_kib_per_dispatch": kib_copy, "copy_dispatches": len(c[(cp, ctr)]),
                    "copy_bytes": copy_bytes, "scale": scale, "mlp_bytes": kib_mlp * 1024.0 * scale}
    pairs = a.n * a.batch
    traffic = out["FETCH_SIZE"]["mlp_bytes"] + out["WRITE_SIZE"]["mlp_bytes"]
    algo = MLP_ALGO_BYTES_PER_PAIR * pairs
    print(f"kernel: {mlp}")
    print(f"copy kernel: {cp}")
    for ctr, v in out.items():
        print(f"{ctr}: mlp {v['mlp_kib_per_dispatch']:.1f} KiB/dispatch ({v['mlp_dispatches']} dispatches); copy "
              f"{v['copy_kib_per_dispatch']:.1f} KiB/dispatch for {v['copy_bytes']} B ({v['copy_dispatches']} "
              f"dispatches) -> scale {v['scale']:.4f} -> {v['mlp_bytes'] / 1e6:.1f} MB")
    print(f"algorithmic bytes per launch: {algo} ({MLP_ALGO_BYTES_PER_PAIR} B x {pairs} pairs)")
    print(f"traffic / algorithmic: {traffic / algo:.3f}")
    print(f"workload: {workload_key(a)}")
    print(f"sources: {mlp_sources_hash()}")
    print(f"traffic_bytes_per_launch: {traffic:.0f}")


def pmc_table(a):
    """Mean counter value per dispatch for every kernel whose name contains one of --kernels, from rocprofv3
    counter-collection CSVs; FETCH_SIZE / WRITE_SIZE also as bytes, scaled by the copy kernel of known size when
    the same runs hold it."""
    c = read_counters(a.pmc_table)
    mean = lambda v: sum(v) / len(v)
    names = sorted({k for k, _ in c})
    cp = [n for n in names if "elementwise" in n]
    scale = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [(n, mean(c[(n, ctr)])) for n in cp if (n, ctr) in c]
        if vals:
            scale[ctr] = a.copy_mib * 2 ** 20 / (max(v for _, v in vals) * 1024.0)
    pats = [x for x in a.kernels.split(",") if x]
    print("| Kernel | Counter | Mean per dispatch | Dispatches | Bytes per dispatch (copy-scaled) |")
    print("|---|---|---|---|---|")
    for n in names:
        if not any(pt in n for pt in pats):
            continue
        for (kn, ctr), v in sorted(c.items()):
            if kn != n:
                continue
            b = f"{mean(v) * 1024.0 * scale[ctr] / 1e6:.1f} MB" if ctr in scale else ""
            print(f"| {n[:70]} | {ctr} | {mean(v):.6g} | {len(v)} | {b} |")


def measured_traffic(a):
    """HBM bytes per MLP launch from the committed counter summary, if it was taken on this workload and on the
    current kernel sources; otherwise None."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            kv = dict(line.strip().split(": ", 1) for line in fh if line.count(": ") >= 1 and
                      line.split(": ", 1)[0] in ("workload", "sources", "traffic_bytes_per_launch"))
    except OSError:
        return None
    if kv.get("workload") != workload_key(a) or kv.get("sources") != mlp_sources_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def measured_peaks(ctx):
    """Rates this GPU sustains in plain loops (after the timed region): BF16 MFMA, FP32 FMA and LDS reads from the
    library's probes, HBM from a 1 GiB device copy timed with events (2 GiB moved)."""
    import torch
    pk = ctx.measure_peaks()
    src = torch.ones(2 ** 28, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    pk["hbm_gbs"] = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return pk


def add_measured(rec_roof, achieved, peak_measured):
    rec_roof["measured_peak"] = peak_measured
    rec_roof["frac_of_measured"] = achieved / peak_measured if peak_measured else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(g, Ws, bs, H, W, txs, budget_s, one_thread_spectra=2):
    """The FP64 oracle timed on the host: whole spectra (MLP + brute-force
    compositing over all Gaussians in depth order) until the budget is used,
    on every host thread, then `one_thread_spectra` whole spectra on one thread
    (compositor and BLAS both limited to one)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import model as M
    s = M.Scene.from_arrays(g, H, W)
    mlp = M.MLP([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs])
    pix = M.full_grid(H, W)
    threads = M.set_threads(0)
    blas_threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    t0 = time.perf_counter()
    done = 0
    while True:
        M.render_query(s, mlp, txs[done % len(txs)].astype(np.float64), pix=pix, margins=None)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    one = None
    if one_thread_spectra > 0:
        M.set_threads(1)
        with threadpool_limits(1):
            t1 = time.perf_counter()
            for k in range(one_thread_spectra):
                M.render_query(s, mlp, txs[k % len(txs)].astype(np.float64), pix=pix, margins=None)
            dt1 = time.perf_counter() - t1
        M.set_threads(threads)
        one = {"value": one_thread_spectra / dt1, "unit": "spectra/s", "cores": 1,
               "sample": f"{one_thread_spectra} full spectra, {dt1:.1f} s"}
    return {"value": done / dt, "unit": "spectra/s", "cores": threads, "kind": "oracle",
            "blas_threads": blas_threads, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": one,
            "sample": f"{done} full {H}x{W} spectra at N={len(g['mean_x'])} (FP64 MLP + brute-force compositing), "
                      f"{dt:.1f} s"}


class _Pool:
    """Reusable host output buffers for serving requests (grows on demand)."""

    def __init__(self, shapes, per_shape):
        self.free = {sh: [np.zeros(sh, np.float32) for _ in range(per_shape)] for sh in set(shapes)}

    def get(self, sh):
        return self.free[sh].pop() if self.free[sh] else np.zeros(sh, np.float32)

    def put(self, sh, a):
        self.free[sh].append(a)


def serve_run(ctx, plan, shapes, rate=None, depth=256):
    """Serve `plan` = [(scene_id, tx)] through the serving loop. rate=None:
    closed loop with `depth` outstanding requests (saturation); else Poisson
    arrivals at `rate` per second, latency measured from the scheduled arrival.
    Returns (throughput, latencies_us, stats list)."""
    import threading
    pool = _Pool(list(shapes.values()), min(depth, 64) + 8)
    lock = threading.Condition()
    inflight = []
    lat, stats = [], []
    done = [0]
    n = len(plan)

    def waiter():
        while done[0] < n:
            with lock:
                while not inflight:
                    lock.wait()
                tk, sid, buf = inflight.pop(0)
            st = ctx.serve_wait(tk)
            lat.append(st["total_us"])
            stats.append(st)
            with lock:
                pool.put(shapes[sid], buf)
                done[0] += 1
                lock.notify_all()

    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = ctx.clock()
    if rate:
        arrivals = t0 + 0.05 + np.cumsum(np.random.default_rng(11).exponential(1.0 / rate, n))
    for i, (sid, tx) in enumerate(plan):
        with lock:
            while done[0] + depth <= i:
                lock.wait()
            buf = pool.get(shapes[sid])
        arr = 0.0
        if rate:
            arr = float(arrivals[i])
            while ctx.clock() < arr:
                pass
        tk = ctx.serve_submit(sid, tx, buf, arr)
        with lock:
            inflight.append((tk, sid, buf))
            lock.notify_all()
    th.join()
    elapsed = ctx.clock() - (t0 + (0.05 if rate else 0.0))
    return n / elapsed, lat, stats


def serve_sweep(a):
    """8 resident scenes (N in {5k, 20k, 100k}, 90x360 or 180x720), random scene
    per request, Poisson arrivals at fractions of the measured saturation rate."""
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    scenes = [(5000, 90, 360), (5000, 180, 720), (20000, 90, 360), (20000, 180, 720), (100000, 90, 360),
              (100000, 180, 720), (20000, 90, 360), (100000, 90, 360)]
    ctx = B.Context(0)
    sids, shapes = [], {}
    for i, (n, H, W) in enumerate(scenes):
        sid = ctx.upload_scene(synth.gaussians(n, H, W, seed=1003 + 10 * i), H, W,
                               mlp=synth.mlp_weights(seed=3003 + 10 * i))
        sids.append(sid)
        shapes[sid] = (H, W)
    rng = np.random.default_rng(5003)
    R = a.serve_requests
    txs = synth.tx_positions(R, seed=2003)
    plan = [(sids[int(k)], txs[j]) for j, k in enumerate(rng.integers(0, len(scenes), R))]
    # plain path: the same request mix, one FP32 query per launch, synchronously
    import torch
    q = min(R, 64)
    t_dev = torch.from_numpy(np.stack([t for _, t in plan[:q]])).cuda()
    outs = {sid: torch.empty((1,) + shapes[sid], device="cuda") for sid in sids}
    for k in range(min(q, 8)):
        ctx.render(plan[k][0], t_dev[k:k + 1], flags=B.MLP_FP32, out=outs[plan[k][0]])
    torch.cuda.synchronize()
    lat_plain = []
    t0 = time.perf_counter()
    for k in range(q):
        s0 = time.perf_counter()
        ctx.render(plan[k][0], t_dev[k:k + 1], flags=B.MLP_FP32, out=outs[plan[k][0]])
        torch.cuda.synchronize()
        lat_plain.append(1e6 * (time.perf_counter() - s0))
    plain = q / (time.perf_counter() - t0)
    print(json.dumps({"serve_sweep": "plain", "throughput": plain, "p50_us": pct(lat_plain, 50),
                      "p99_us": pct(lat_plain, 99), "queries": q,
                      "note": "one FP32 query per launch over the same scene mix"}), flush=True)
    budget = int(a.hbm_budget_gb * 1e9)
    # per-scene batches (one graph per scene and bucket), then batches across scenes (graphs keyed by capacities)
    for mode in ("per_scene", "mixed"):
        ctx.serve_start(max_batch=64, n_slots=3, flags=B.MLP_BF16, hbm_budget=budget, mixed=mode == "mixed")
        serve_run(ctx, plan, shapes)  # warm-up: one pass of the plan captures the graphs its batches need
        warm = ctx.serve_counters()
        sat, lat, st = serve_run(ctx, plan, shapes)
        print(json.dumps({"serve_sweep": "saturation", "mode": mode, "rate": None, "throughput": sat,
                          "over_plain": sat / plain, "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
                          "mean_batch": float(np.mean([s["batch"] for s in st])), "hbm_budget_bytes": budget}),
              flush=True)
        for f in (0.1, 0.25, 0.5, 0.75, 0.9, 1.1):
            thr, lat, st = serve_run(ctx, plan, shapes, rate=f * sat, depth=1 << 30)
            print(json.dumps({"serve_sweep": "poisson", "mode": mode, "rate_fraction": f, "rate": f * sat,
                              "throughput": thr, "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
                              "mean_batch": float(np.mean([s["batch"] for s in st]))}), flush=True)
        cnt = ctx.serve_counters()
        cnt["graph_builds_after_warmup"] = cnt["graph_builds"] - warm["graph_builds"]
        print(json.dumps({"serve_sweep": "counters", "mode": mode, **cnt}), flush=True)
        ctx.serve_stop()
    ctx.close()


def timed_renders(ctx, sid, tx_dev, flags, out, steps, warmup):
    """Renders tx_dev[0:warmup] untimed, then tx_dev[warmup:warmup+steps] timed with stage events;
    returns (elapsed_s, per-step ms, stage table)."""
    import torch
    for i in range(warmup):
        ctx.render(sid, tx_dev[i], flags=flags, out=out)
    torch.cuda.synchronize()
    ctx.stage_timing(True)
    ctx.stage_times()  # reset
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        ctx.render(sid, tx_dev[warmup + i], flags=flags, out=out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.stage_timing(False)
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return max(wall, sum(step_ms) / 1e3), step_ms, {k: v[0] / max(v[1], 1) for k, v in stages.items()
                                                    if not k.endswith("_backward")}


def bench_large(a):
    """Large scene: N = 500k, 360 x 1440, batch 256, BF16 (timed steps) and FP32 (one timed step) MLP."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth

    H, W, N, Bq = 360, 1440, 500_000, 256
    steps, warmup = max(1, min(a.steps, 5)), min(a.warmup, 1)
    g = synth.gaussians(N, H, W, seed=1004, scale_range=(0.5, 20.0))
    Ws, bs = synth.mlp_weights(seed=3004)
    nbat = warmup + steps
    txs = synth.tx_positions(nbat * Bq, seed=2004)
    ctx = B.Context(0, mlp_pairs_per_wave=a.pairs_per_wave)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx_dev = torch.from_numpy(txs).cuda().view(nbat, Bq, 3)
    out = torch.empty((Bq, H, W), device="cuda", dtype=torch.float32)
    el, step_ms, st = timed_renders(ctx, sid, tx_dev, B.MLP_BF16, out, steps, warmup)
    work = ctx.blend_work()
    value = steps * Bq / el
    bf16_last = out.clone()
    el32, step32, st32 = timed_renders(ctx, sid, tx_dev[nbat - 1:], B.MLP_FP32, out, 1, 0)
    # same batch (the last timed one) in both precisions
    err = float((bf16_last - out).abs().max() / out.abs().max().clamp_min(1e-30))
    pairs = N * Bq
    T_tiles = -(-W // 16) * -(-H // 16)
    seg = 256 if T_tiles <= 256 else 512  # binning segment: one 8- or 9-bit digit
    segs = -(-T_tiles // seg)
    keys = work["entries"]
    hist_entries = Bq * segs * seg * -(-N // (1024 if seg == 256 else 8192))
    list_bytes = pairs * 24 + keys * 4 + hist_entries * 12 + Bq * T_tiles * 8
    list_ms = st["scan"] + st["emit_keys"] + st["radix_sort"] + st["tile_ranges"]
    flops = float(FLOP_PER_PAIR) * pairs
    rec = {
        "metric": "spectra/s at N=500k, 360x1440, batch 256 (large scene)", "value": value, "unit": "spectra/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "large scene: N=500000 Gaussians, log-scales U(log 0.5, log 20) px, 360x1440 spectra "
                               "(0.25 deg/px), batch 256 TX positions, MLP 89-4x256-7",
                   "n_gaussians": N, "height": H, "width": W, "batch": Bq},
        "fp32_mlp": {"value": Bq / el32, "ms_per_step": 1e3 * el32, "mlp_ms": st32["mlp_preprocess"],
                     "bf16_speedup": value / (Bq / el32),
                     "bf16_vs_fp32_normwise_max_err": err},
        "stages_ms_per_step": st,
        "roofline": {"kernel": "mlp_bf16_deform_preprocess", "bound": "mfma",
                     "achieved": flops / (st["mlp_preprocess"] * 1e-3) / 1e12, "peak": PEAK["bf16"],
                     "unit": "TFLOP/s", "frac": flops / (st["mlp_preprocess"] * 1e-3) / 1e12 / PEAK["bf16"],
                     "traffic": None, "avg_launch_ms": st["mlp_preprocess"]},
        "stage_rooflines": {
            "lists": {"bound": "hbm", "achieved": list_bytes / (list_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": list_bytes / (list_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "algorithmic_bytes": list_bytes, "ms": list_ms, "list_entries": keys, "segments": segs,
                      "note": "binning: rect+count read twice (24 B/pair), 4 B/list entry written, histogram scan "
                              "12 B/entry, ranges 8 B/tile"},
            "blend": {"bound": "alu", "evaluations": work["evaluations"], "ops_per_evaluation": BLEND_OPS_PER_EVAL,
                      "achieved": work["evaluations"] * BLEND_OPS_PER_EVAL / (st["blend"] * 1e-3) / 1e12,
                      "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                      "frac": work["evaluations"] * BLEND_OPS_PER_EVAL / (st["blend"] * 1e-3) / VALU_PEAK_LANE_OPS,
                      "ms": st["blend"]}},
        "latency_us": {"batched_p50": 1e3 * pct(step_ms, 50), "batched_p99": 1e3 * pct(step_ms, 99)},
    }
    pk = measured_peaks(ctx)
    add_measured(rec["roofline"], rec["roofline"]["achieved"], pk["mfma_bf16_tflops"])
    add_measured(rec["stage_rooflines"]["lists"], rec["stage_rooflines"]["lists"]["achieved"], pk["hbm_gbs"])
    add_measured(rec["stage_rooflines"]["blend"], rec["stage_rooflines"]["blend"]["achieved"], pk["fma_tops"])
    rec["measured_peaks"] = pk
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_train(a):
    """Training steps: N = 50k Gaussians, batch 16 TX positions, 90 x 360; BF16 MLP, FP32 rasterizer, L1 loss,
    hand-written backward, Adam in the library (the hyperparameter table's learning rates)."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth

    N, H, W, Bq = 50_000, 90, 360, 16
    steps, warmup = a.steps, a.warmup
    g = synth.gaussians(N, H, W, seed=1002)
    g_true = synth.gaussians(N, H, W, seed=4002)
    Ws, bs = synth.mlp_weights(seed=3002)
    ctx = B.Context(0, mlp_pairs_per_wave=a.pairs_per_wave)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    nbat = warmup + steps
    tx_dev = torch.from_numpy(synth.tx_positions(nbat * Bq, seed=2002)).cuda().view(nbat, Bq, 3)
    # targets: the separately seeded ground-truth set rendered at the same TX positions (by this library, whose
    # renders the parity tests hold to the oracle; the bench does not run the oracle outside its CPU baseline)
    gsid = ctx.upload_scene(g_true, H, W, mlp=(Ws, bs))
    targets = [ctx.render(gsid, tx_dev[i], flags=B.MLP_BF16).clone() for i in range(nbat)]
    gp = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in B.PARAMS[:7]}
    Wd = [torch.from_numpy(w).cuda() for w in Ws]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    params = [gp[k] for k in B.PARAMS[:7]] + Wd + bd
    grads = [torch.zeros_like(t) for t in params]
    mom = [torch.zeros_like(t) for t in params]
    vel = [torch.zeros_like(t) for t in params]
    lrs = [1e-2] * 7 + [8e-3] * (len(Wd) + len(bd))
    gd = dict(zip(B.PARAMS[:7], grads[:7]))
    gd["weight"] = grads[7:7 + len(Wd)]
    gd["bias"] = grads[7 + len(Wd):]
    losses = []
    count = [0]
    reused = []

    def step(i, probe=False, det=False, fp32=False):
        mf = B.MLP_FP32 if fp32 else B.MLP_BF16
        out, aux = ctx.render(sid, tx_dev[i], flags=mf | B.KEEP_AUX)
        loss, grad = ctx.l1_loss(out, targets[i])
        for t in grads:
            t.zero_()
        ctx.render_backward(sid, tx_dev[i], mf | (B.DETERMINISTIC if det else 0), grad, aux, gd)
        if probe:  # (waits) whether the backward took its forward's kept records and lists
            reused.append(bool(ctx.device_status()["flags"] & B.DEV_BWD_REUSED))
        count[0] += 1
        ctx.adam_step(params, grads, mom, vel, lrs, count[0])
        ctx.update_scene(sid, gaussians=gp, mlp=(Wd, bd))
        return loss

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        losses.append(step(warmup + i))
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    el = max(wall, sum(step_ms) / 1e3)
    lv = [float(l) for l in losses]
    # per-stage times: a few more steps with the library's stage events on (after the timed region)
    n_inst = min(steps, 5)
    ctx.stage_timing(True)
    ctx.stage_times()  # reset
    for i in range(n_inst):
        step(warmup + i)
    torch.cuda.synchronize()
    stages = {k: v[0] / n_inst for k, v in ctx.stage_times().items() if v[1] > 0}
    ctx.stage_timing(False)
    step(warmup, probe=True)
    # the same steps with the deterministic backward (fixed-order gradient sums)
    nd = min(steps, 10)
    step(warmup, det=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(nd):
        step(warmup + i, det=True)
    torch.cuda.synchronize()
    det_ms = 1e3 * (time.perf_counter() - t1) / nd
    # the same steps at the paper's precision: FP32 MLP forward and backward (FP32 matrix cores), with their stages
    step(warmup, fp32=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(nd):
        step(warmup + i, fp32=True)
    torch.cuda.synchronize()
    fp32_ms = 1e3 * (time.perf_counter() - t2) / nd
    ctx.stage_timing(True)
    ctx.stage_times()  # reset
    for i in range(n_inst):
        step(warmup + i, fp32=True)
    torch.cuda.synchronize()
    stages32 = {k: v[0] / n_inst for k, v in ctx.stage_times().items() if v[1] > 0}
    ctx.stage_timing(False)
    # MLP backward FLOPs per pair: weight gradients and input gradients of the output layer (7 x 256) and of the
    # three 256 x 256 layers, 2 FLOP per multiply-add each (layer 1's gradients are per Gaussian and per query)
    bwd_flop = Bq * N * 2 * 2 * (7 * 256 + 3 * 256 * 256)
    t_bwd = stages.get("mlp_backward", 0.0)
    ach = bwd_flop / (t_bwd * 1e-3) / 1e12 if t_bwd > 0 else None
    # HBM bytes the MLP backward must move per pair (BF16 activations and gradients, 512 B per 256-row): dy read
    # (7 FP32); the output layer reads the last activations and writes their gradient; the two upper 256 x 256
    # layers read their output gradient and input activations and write their input gradient; the lowest one
    # reads its output gradient and input activations (the first layer's gradient is reduced into per-Gaussian
    # and per-query sums, never stored)
    bwd_bytes = Bq * N * (28 + 2 * 512 + 2 * 3 * 512 + 2 * 512)
    gbs = bwd_bytes / (t_bwd * 1e-3) / 1e9 if t_bwd > 0 else None
    rec = {
        "metric": "training steps/s at N=50k, batch 16, 90x360", "value": steps / el, "unit": "steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "training step: N=50000 Gaussians, batch 16 TX positions, 90x360, BF16 MLP "
                               "89-4x256-7, FP32 rasterizer, L1 loss, hand-written backward, Adam (Gaussians 1e-2, "
                               "MLP 8e-3) in the library", "n_gaussians": N, "batch": Bq, "height": H, "width": W},
        "spectra_per_s": steps * Bq / el,
        "loss_first": lv[0], "loss_last": lv[-1],
        "latency_us": {"step_p50": 1e3 * pct(step_ms, 50), "step_p99": 1e3 * pct(step_ms, 99)},
        "stages_ms_per_step": stages,
        "roofline": {"kernel": "mlp_backward (BF16 layer GEMMs with FP32 accumulation, ReLU masks, column sums)",
                     "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": None if gbs is None else gbs / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_step": bwd_bytes, "avg_ms": t_bwd,
                     "mfma": {"achieved": ach, "peak": PEAK["bf16"], "unit": "TFLOP/s",
                              "frac": None if ach is None else ach / PEAK["bf16"], "flop_per_step": bwd_flop},
                     "note": "5,148 B per pair: the rows the backward must read and write once each (BF16); the "
                             "kernels read each layer's gradient and activations twice (weight and input gradient "
                             "in separate passes), 7,220 B per pair"},
        "backward_reused_forward": reused[0],
        "deterministic_ms_per_step": det_ms,
        "fp32": {"ms_per_step": fp32_ms, "stages_ms_per_step": stages32,
                 "note": "FP32 MLP forward and backward (the paper's precision), the same loop otherwise"},
        "note": "targets: a separately seeded ground-truth Gaussian set rendered by this library at the same TX "
                "positions; stage times from 5 more steps with stage events on; the backward takes the records, "
                "lists and BF16 activations its forward render kept (backward_reused_forward)",
    }
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_protocol(a):
    """The paper's training protocol in its fine stage (Sec. 4.4): N = 50k Gaussians, batch 16 positions, 90 x 360,
    anneal-smoothed positions, BF16 deformation, hybrid l1 + SSIM loss, frozen canonical positions, Adam (1e-2 /
    8e-3); targets are beam-scan spectra of multipath lists at the same positions (Sec. 3.1)."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    from paper_2506_12787_amd.train import Trainer

    N, H, W, Bq = 50_000, 90, 360, 16
    steps, warmup = a.steps, a.warmup
    ctx = B.Context(0, mlp_pairs_per_wave=a.pairs_per_wave)
    nbat = warmup + steps
    paths, counts, txh = synth.multipath(nbat * Bq, seed=6002)
    tx_all = torch.from_numpy(txh).cuda().view(nbat, Bq, 3)
    targets = ctx.beamscan(torch.from_numpy(paths).cuda(), torch.from_numpy(counts).cuda(), H, W).view(nbat, Bq, H, W)
    tr = Trainer(ctx, synth.gaussians(N, H, W, seed=1002), H, W, synth.mlp_weights(seed=3002),
                 n_positions=nbat * Bq, coarse_iters=2, bf16=True, seed=7)
    losses = []
    for i in range(2):  # the coarse stage (static Gaussians), untimed
        tr.step(tx_all[i % nbat], targets[i % nbat].contiguous())
    el, ms = _event_time(lambda: losses.append(tr.step(tx_all[len(losses) % nbat],
                                                       targets[len(losses) % nbat].contiguous())),
                         steps, warmup)
    lv = [float(l[0]) for l in losses]
    rec = {"metric": "training steps/s of the paper's protocol (fine stage), N=50k, batch 16, 90x360",
           "value": steps / el, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * el / steps, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "training protocol fine stage: N=50000 Gaussians, batch 16 positions, 90x360, "
                                  "anneal smoothing (gamma 1, tau 10k), BF16 MLP 89-4x256-7, hybrid loss 0.7 l1 + "
                                  "0.3 (1 - SSIM), frozen canonical positions, Adam 1e-2 / 8e-3; targets: beam-scan "
                                  "spectra of 25-path multipath lists", "n_gaussians": N, "batch": Bq,
                      "height": H, "width": W},
           "spectra_per_s": steps * Bq / el, "loss_first": lv[0], "loss_last": lv[-1],
           "latency_us": {"step_p50": 1e3 * pct(ms, 50), "step_p99": 1e3 * pct(ms, 99)}}
    ctx.close()
    print(json.dumps(rec), flush=True)


def _event_time(fn, steps, warmup):
    """Runs fn() warmup times, then times `steps` calls with HIP events on the current stream; returns
    (elapsed seconds = max(wall, event sum), per-call ms)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return max(wall, sum(ms) / 1e3), ms


def bench_beamscan(a):
    """Beam-scan spectra from multipath lists (Sec. 3.1): a batch of 256 receivers' worth of mirror-image path
    lists (25 paths: line of sight and wall reflections up to second order), 4 x 4 array at half-wavelength
    spacing, 90 x 360 spectra."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, Bq, side = 90, 360, 256, 4
    paths, counts, _ = synth.multipath(Bq, seed=6003)
    ctx = B.Context(0)
    p, c = torch.from_numpy(paths).cuda(), torch.from_numpy(counts).cuda()
    out = torch.empty((Bq, H, W), device="cuda")
    el, ms = _event_time(lambda: ctx.beamscan(p, c, H, W, side=side, out=out), a.steps, a.warmup)
    K = side * side
    # the contraction of the beam-scan equation: K complex multiply-adds per (pixel, query), 8 FLOP each
    flop = 8.0 * K * Bq * H * W
    avg = sum(ms) / len(ms)
    rec = {"metric": "beam-scan spectra/s (90x360, 4x4 array, 25-path lists, batch 256)", "value": a.steps * Bq / el,
           "unit": "spectra/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps,
           "higher_is_better": True, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": "beam-scan spectrum synthesis from mirror-image multipath lists (line of sight + "
                                  "wall reflections up to order 2, 25 paths) in a 6x6x3 m room, 4x4 array, D = "
                                  "lambda/2, 90x360 spectra, batch 256", "batch": Bq, "height": H, "width": W,
                      "array_side": side, "paths": int(paths.shape[1])},
           "roofline": {"kernel": "beamscan spectrum (channel_kernel + spectrum_kernel)", "bound": "alu",
                        "achieved": flop / (avg * 1e-3) / 1e12, "peak": FP32_VALU_PEAK, "unit": "TFLOP/s",
                        "frac": flop / (avg * 1e-3) / 1e12 / FP32_VALU_PEAK, "traffic": None,
                        "avg_call_ms": avg, "flop_per_call": flop,
                        "output_GBs": Bq * H * W * 4 / (avg * 1e-3) / 1e9,
                        "note": "8 K FLOP per (pixel, query): the steering-vector contraction; the per-pixel sincospi "
                                "(shared by 8 queries) and the per-query FP64 channel are not counted"}}
    if not a.no_cpu_baseline:
        from oracle import beamscan as Bs
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < min(a.cpu_seconds, 10.0):
            Bs.spectrum(paths[n % Bq].astype(np.float64), int(counts[n % Bq]), H, W, side)
            n += 1
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": n / dt, "unit": "spectra/s", "cores": 1, "kind": "oracle",
                               "cpu_model": cpu_model(), "sample": f"{n} full spectra (numpy FP64), {dt:.1f} s"}
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_rssi(a):
    """RSSI head (Sec. 7.2): 16 x 16 spectra of 50 Gaussians pooled to one value per query, batch 1024."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, N, Bq = 16, 16, 50, 1024
    g = synth.gaussians(N, H, W, seed=1005, scale_range=(0.7, 4.0))
    Ws, bs = synth.mlp_weights(seed=3005)
    ctx = B.Context(0)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    nb = a.warmup + a.steps
    tx = torch.from_numpy(synth.tx_positions(nb * Bq, seed=2005)).cuda().view(nb, Bq, 3)
    it = [0]

    def call(flags):
        ctx.render_rssi(sid, tx[it[0] % nb], flags=flags)
        it[0] += 1

    rec = {"metric": "RSSI queries/s (16x16 spectra, 50 Gaussians, batch 1024)", "unit": "queries/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "RSSI head: deformable render of a 16x16 spectrum from 50 Gaussians, global average "
                                  "pooling, batch 1024 TX positions, MLP 89-4x256-7", "n_gaussians": N, "height": H,
                      "width": W, "batch": Bq}}
    for name, flags in (("bf16", B.MLP_BF16), ("fp32", B.MLP_FP32)):
        ctx.stage_timing(True)
        ctx.stage_times()
        el, ms = _event_time(lambda: call(flags), a.steps, a.warmup)
        st = {k: v[0] / max(v[1], 1) for k, v in ctx.stage_times().items() if v[1] > 0}
        ctx.stage_timing(False)
        leg = {"value": a.steps * Bq / el, "ms_per_step": 1e3 * el / a.steps, "p50_ms": pct(ms, 50),
               "p99_ms": pct(ms, 99), "stages_ms_per_step": st}
        if name == "bf16":
            rec.update(value=leg["value"], ms_per_step=leg["ms_per_step"], stages_ms_per_step=st,
                       latency_us={"batch_p50": 1e3 * leg["p50_ms"], "batch_p99": 1e3 * leg["p99_ms"]})
            flops = float(FLOP_PER_PAIR) * N * Bq
            mlp_ms = st.get("mlp_preprocess", 0.0)
            rec["roofline"] = {"kernel": "mlp_bf16_deform_preprocess", "bound": "mfma",
                               "achieved": flops / (mlp_ms * 1e-3) / 1e12 if mlp_ms else None, "peak": PEAK["bf16"],
                               "unit": "TFLOP/s", "traffic": None, "avg_launch_ms": mlp_ms,
                               "note": "51k pairs per batch: the MLP launch is too small to fill the chip"}
            if mlp_ms:
                rec["roofline"]["frac"] = rec["roofline"]["achieved"] / PEAK["bf16"]
        else:
            rec["fp32"] = leg
    if not a.no_cpu_baseline:
        from oracle import model as M
        from oracle import rssi as R
        s = M.Scene.from_arrays(g, H, W)
        mlp = M.MLP([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs])
        txh = tx[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < min(a.cpu_seconds, 10.0):
            R.rssi_query(s, mlp, txh[n % Bq])
            n += 1
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": n / dt, "unit": "queries/s", "cores": M.set_threads(0), "kind": "oracle",
                               "cpu_model": cpu_model(), "sample": f"{n} queries (FP64 MLP + render + pooling), "
                                                                   f"{dt:.1f} s"}
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_wrap(a):
    """The headline batch (N = 100k, 90 x 360, batch 64, BF16) with periodic azimuth (lists by binning: one
    segment of tiles)."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, N, Bq = 90, 360, 100_000, 64
    g = synth.gaussians(N, H, W, seed=1003)
    ctx = B.Context(0)
    sid = ctx.upload_scene(g, H, W, mlp=synth.mlp_weights(seed=3003))
    nbat = a.warmup + a.steps
    tx_dev = torch.from_numpy(synth.tx_positions(nbat * Bq, seed=2003)).cuda().view(nbat, Bq, 3)
    out = torch.empty((Bq, H, W), device="cuda")
    rec = {"metric": "spectra/s at N=100k, 90x360, batch 64, periodic azimuth", "unit": "spectra/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "batched deformable render with azimuth wrap-around, N=100000, 90x360, batch 64, "
                                  "BF16 MLP 89-4x256-7", "n_gaussians": N, "height": H, "width": W, "batch": Bq}}
    for name, flags in (("wrap", B.MLP_BF16 | B.WRAP_AZIMUTH), ("plane", B.MLP_BF16)):
        el, step_ms, st = timed_renders(ctx, sid, tx_dev, flags, out, a.steps, a.warmup)
        work = ctx.blend_work()
        lists_ms = st["scan"] + st["emit_keys"] + st["radix_sort"] + st["tile_ranges"]
        leg = {"value": a.steps * Bq / el, "ms_per_step": 1e3 * el / a.steps, "stages_ms_per_step": st,
               "list_entries": work["entries"], "lists_ms": lists_ms}
        if name == "wrap":
            pairs = N * Bq
            nk = work["entries"]
            T_tiles = -(-W // 16) * -(-H // 16)
            if T_tiles <= 256:
                # binned (one segment): the binning's byte model of the default line
                lb = pairs * 24 + nk * 4 + Bq * 256 * -(-N // 1024) * 12 + Bq * T_tiles * 8
                kern = "list building by binning (histogram, column and tile scans, placement, ranges)"
            else:
                # scan 8 B/pair, emit 12 B/pair read + 8 B/key written, 2 radix passes x 16 B/key + ranges 4 B/key
                lb = pairs * 20 + nk * (8 + 2 * 16 + 4)
                kern = "list building (scan, key emission, 2-pass radix sort, ranges)"
            rec.update(value=leg["value"], ms_per_step=leg["ms_per_step"], stages_ms_per_step=st,
                       list_entries=nk)
            rec["roofline"] = {"kernel": kern,
                               "bound": "hbm", "achieved": lb / (lists_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": lb / (lists_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "traffic": None, "algorithmic_bytes": lb, "ms": lists_ms}
        else:
            rec["plane"] = leg
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_paper(a):
    """The paper's own model (Sec. 4.1/4.2/6.1): N = 10k Gaussians (the paper's count), 90 x 360, batch 64 positions,
    FP32 paper MLP (8 x 156 with skips), order-free GMM sum of complex responses; the plain one-query path beside."""
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth
    H, W, N, Bq = 90, 360, 10_000, 64
    g = synth.paper_gaussians(N, seed=1006)
    Ws, bs = synth.paper_mlp_weights(seed=3006, out_scale=0.3)
    ctx = B.Context(0)
    sid = ctx.upload_paper_scene(g, H, W, mlp=(Ws, bs))
    nbat = a.warmup + a.steps
    tx = torch.from_numpy(synth.tx_positions(nbat * Bq, seed=2006)).cuda().view(nbat, Bq, 3)
    out = torch.empty((Bq, H, W), device="cuda")
    it = [0]

    def call():
        ctx.render_paper(sid, tx[it[0] % nbat], flags=B.MLP_FP32, out=out, channels=False)
        it[0] += 1

    ctx.stage_timing(True)
    ctx.stage_times()
    el, ms = _event_time(call, a.steps, a.warmup)
    st = {k: v[0] / max(v[1], 1) for k, v in ctx.stage_times().items() if v[1] > 0}
    ctx.stage_timing(False)
    flop_pair = 2 * sum(o * i for o, i in synth.PAPER_LAYER_SHAPES)
    flops = float(flop_pair) * N * Bq
    mlp_ms = st["mlp_preprocess"]
    rec = {"metric": "paper-model spectra/s at N=10k, 90x360, batch 64 (FP32)", "value": a.steps * Bq / el,
           "unit": "spectra/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": "the paper's model: 10000 Cholesky Gaussians with tanh centres and complex "
                                  "responses, order-free GMM sum, deformation MLP 81-8x156 (input skips at layers "
                                  "3, 5, 7)-5 in FP32, 90x360 spectra, batch 64 positions", "n_gaussians": N,
                      "height": H, "width": W, "batch": Bq},
           "stages_ms_per_step": st,
           "latency_us": {"batch_p50": 1e3 * pct(ms, 50), "batch_p99": 1e3 * pct(ms, 99)},
           "roofline": {"kernel": "paper_mlp_kernel (FP32 MLP on v_mfma_f32_16x16x4_f32 + deform + preprocess)",
                        "bound": "mfma", "achieved": flops / (mlp_ms * 1e-3) / 1e12, "peak": PEAK["fp32"],
                        "unit": "TFLOP/s", "frac": flops / (mlp_ms * 1e-3) / 1e12 / PEAK["fp32"],
                        "traffic": None, "flop_per_pair": flop_pair, "avg_launch_ms": mlp_ms,
                        "note": "algorithmic FLOPs of the unpadded 156-wide layers (the kernel pads the widths to "
                                "160 and the inputs to 96: 6% more); FP32 operands and accumulation, the paper's "
                                "precision"}}
    # plain: one query per launch
    o1 = torch.empty((1, H, W), device="cuda")
    for i in range(2):
        ctx.render_paper(sid, tx[0, i:i + 1].contiguous(), flags=B.MLP_FP32, out=o1, channels=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(16):
        s0 = time.perf_counter()
        ctx.render_paper(sid, tx[1, i:i + 1].contiguous(), flags=B.MLP_FP32, out=o1, channels=False)
        torch.cuda.synchronize()
        lat.append(1e6 * (time.perf_counter() - s0))
    plain = 16 / (time.perf_counter() - t0)
    rec["plain"] = {"value": plain, "unit": "spectra/s", "p50_us": pct(lat, 50), "p99_us": pct(lat, 99)}
    rec["batched_over_plain"] = rec["value"] / plain
    if not a.no_cpu_baseline:
        from oracle import paper as P
        txh = tx[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < min(a.cpu_seconds, 12.0):
            P.render_query(g, H, W, mlp=(Ws, bs), tx=txh[n % Bq])
            n += 1
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": n / dt, "unit": "spectra/s", "cores": os.cpu_count(), "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"{n} full spectra (numpy FP64 MLP and GMM sum), {dt:.1f} s"}
    ctx.close()
    print(json.dumps(rec), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if a.pmc_summary:
        pmc_summary(a)
        return
    if a.pmc_table:
        pmc_table(a)
        return
    if a.serve_sweep:
        serve_sweep(a)
        return
    if a.workload == "large":
        bench_large(a)
        return
    if a.workload == "train":
        bench_train(a)
        return
    if a.workload in ("beamscan", "rssi", "wrap", "protocol", "paper"):
        {"beamscan": bench_beamscan, "rssi": bench_rssi, "wrap": bench_wrap, "protocol": bench_protocol,
         "paper": bench_paper}[a.workload](a)
        return
    import torch
    from paper_2506_12787_amd import binding as B
    from paper_2506_12787_amd import synth

    H, W, N, Bq = a.height, a.width, a.n, a.batch
    g = synth.gaussians(N, H, W, seed=1003)
    Ws, bs = synth.mlp_weights(seed=3003)
    nbat = a.warmup + a.steps
    txs = synth.tx_positions(nbat * Bq, seed=2003)
    ctx = B.Context(0, mlp_pairs_per_wave=a.pairs_per_wave)
    sid = ctx.upload_scene(g, H, W, mlp=(Ws, bs))
    tx_dev = torch.from_numpy(txs).cuda().view(nbat, Bq, 3)
    out = torch.empty((Bq, H, W), device="cuda", dtype=torch.float32)
    flags = B.MLP_BF16 if a.mlp == "bf16" else B.MLP_FP32

    for i in range(a.warmup):
        ctx.render(sid, tx_dev[i], flags=flags, out=out)
    torch.cuda.synchronize()
    ctx.stage_timing(True)
    ctx.stage_times()  # reset
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(a.steps):
        ctx.render(sid, tx_dev[a.warmup + i], flags=flags, out=out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.stage_timing(False)
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(a.steps)]
    gpu_ms = sum(step_ms)
    elapsed = max(wall, gpu_ms / 1e3)
    value = a.steps * Bq / elapsed
    ms_per_step = 1e3 * elapsed / a.steps

    mlp_ms, mlp_n = stages["mlp_preprocess"]
    avg_mlp_ms = mlp_ms / max(mlp_n, 1)
    flops = float(FLOP_PER_PAIR) * N * Bq
    achieved = flops / (avg_mlp_ms * 1e-3) / 1e12
    peak = PEAK[a.mlp]
    roofline = {"kernel": f"mlp_{a.mlp}_deform_preprocess", "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(a) if a.mlp == "bf16" else None,
                "algorithmic_bytes_per_launch": MLP_ALGO_BYTES_PER_PAIR * N * Bq,
                "avg_launch_ms": avg_mlp_ms, "flop_per_launch": flops}

    # per-stage rooflines of the list building and the blend, from the last timed batch's work counts
    work = ctx.blend_work()
    st_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
    T_tiles = -(-a.width // 16) * -(-a.height // 16)
    seg = 256 if T_tiles <= 256 else 512  # binning segment: one 8- or 9-bit digit
    segs = -(-T_tiles // seg)
    binned = Bq <= 65535 and T_tiles <= 4096
    pairs = N * Bq
    if binned:
        hist_entries = Bq * segs * seg * -(-N // (1024 if seg == 256 else 8192))
        bin_bytes = pairs * 24 + work["entries"] * 4 + hist_entries * 12 + Bq * T_tiles * 8
        bin_ms = st_ms["scan"] + st_ms["radix_sort"] + st_ms["tile_ranges"]
        bin_note = ("binning: rect+count read twice (24 B/pair), 4 B/list entry written, histogram scan 12 B/entry, "
                    "ranges 8 B/tile")
    else:
        bin_bytes = pairs * 12 + work["entries"] * (8 + 20 + 4) + pairs * 20
        bin_ms = st_ms["scan"] + st_ms["emit_keys"] + st_ms["radix_sort"] + st_ms["tile_ranges"]
        bin_note = "emit + radix sort + ranges (per-pass traffic not itemised)"
    blend_ms = st_ms["blend"]
    stage_rooflines = {
        "lists": {"bound": "hbm", "achieved": bin_bytes / (bin_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": bin_bytes / (bin_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "algorithmic_bytes": bin_bytes, "ms": bin_ms, "list_entries": work["entries"], "note": bin_note},
        "blend": {"bound": "alu", "achieved": work["evaluations"] * BLEND_OPS_PER_EVAL / (blend_ms * 1e-3) / 1e12,
                  "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                  "frac": work["evaluations"] * BLEND_OPS_PER_EVAL / (blend_ms * 1e-3) / VALU_PEAK_LANE_OPS,
                  "evaluations": work["evaluations"], "ops_per_evaluation": BLEND_OPS_PER_EVAL, "ms": blend_ms,
                  "staged_records": work["staged"],
                  "executed_lane_evaluations": work["executed"],
                  "executed_over_needed": work["executed"] / max(work["evaluations"], 1),
                  "gather_GBs": work["staged"] * 44 / (blend_ms * 1e-3) / 1e9},
    }

    pk = measured_peaks(ctx)
    if a.mlp == "bf16":
        add_measured(roofline, achieved, pk["mfma_bf16_tflops"])
    add_measured(stage_rooflines["lists"], stage_rooflines["lists"]["achieved"], pk["hbm_gbs"])
    add_measured(stage_rooflines["blend"], stage_rooflines["blend"]["achieved"], pk["fma_tops"])

    rec = {
        "metric": METRIC, "value": value, "unit": "spectra/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.mlp, "data": "synthetic",
        "config": {"workload": f"batched deformable render, N={N} Gaussians, {H}x{W} spectra, batch {Bq} TX "
                               f"positions, {a.mlp.upper()} MLP 89-4x256-7",
                   "n_gaussians": N, "height": H, "width": W, "batch": Bq, "mlp": a.mlp},
        "latency_us": {"batched_p50": 1e3 * pct(step_ms, 50), "batched_p99": 1e3 * pct(step_ms, 99),
                       "note": "closed-loop: every query of a batch completes with its batch"},
        "stages_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items() if not k.endswith("_backward")},
        "roofline": roofline,
        "stage_rooflines": stage_rooflines,
        "measured_peaks": dict(pk, note="plain loops on this GPU after the timed region: BF16 MFMA chains in "
                                        "registers, FP32 FMA, conflict-free LDS reads, a 1 GiB device copy"),
    }
    if a.copy_probe_mib:
        src = torch.ones(a.copy_probe_mib * 2 ** 18, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not a.quick and a.mlp == "bf16" and a.fp32_steps > 0:
        # the same batched render with the FP32 MLP (the paper's arithmetic), so that the batching gain and the
        # precision gain separate
        nb32 = min(nbat, a.fp32_steps + 1)
        el32, step32, st32 = timed_renders(ctx, sid, tx_dev, B.MLP_FP32, out, nb32 - 1, 1)
        v32 = (nb32 - 1) * Bq / el32
        mlp32 = st32["mlp_preprocess"]
        ach32 = flops / (mlp32 * 1e-3) / 1e12
        rec["fp32_batched"] = {
            "value": v32, "unit": "spectra/s", "dtype": "fp32", "batch": Bq, "steps": nb32 - 1,
            "ms_per_step": 1e3 * el32 / (nb32 - 1), "stages_ms_per_step": st32,
            "roofline": {"kernel": "mlp_fp32_deform_preprocess", "bound": "mfma", "achieved": ach32,
                         "peak": PEAK["fp32"], "unit": "TFLOP/s", "frac": ach32 / PEAK["fp32"],
                         "avg_launch_ms": mlp32, "flop_per_launch": flops}}
        rec["bf16_over_fp32_batched"] = value / v32
    if not a.quick:
        # plain one-query-per-launch FP32 path
        q = a.plain_queries
        txp = torch.from_numpy(synth.tx_positions(q + 2, seed=2103)).cuda()
        o1 = torch.empty((1, H, W), device="cuda", dtype=torch.float32)
        for i in range(2):
            ctx.render(sid, txp[i:i + 1], flags=B.MLP_FP32, out=o1)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for i in range(q):
            s0 = time.perf_counter()
            ctx.render(sid, txp[2 + i:3 + i], flags=B.MLP_FP32, out=o1)
            torch.cuda.synchronize()
            lat.append(1e6 * (time.perf_counter() - s0))
        pw = time.perf_counter() - t0
        plain = q / pw
        rec["plain"] = {"value": plain, "unit": "spectra/s", "dtype": "fp32", "batch": 1,
                        "p50_us": pct(lat, 50), "p99_us": pct(lat, 99)}
        rec["batched_over_plain"] = value / plain
        if "fp32_batched" in rec:
            rec["fp32_batched_over_plain"] = rec["fp32_batched"]["value"] / plain
        # serving loop on the same scene: captured graphs, continuous batching
        # batches across scenes (here all of one scene): a batch renders its own queries only, no padding
        ctx.serve_start(max_batch=Bq, n_slots=3, flags=flags, mixed=True)
        R = a.serve_requests
        stx = synth.tx_positions(R, seed=2203)
        plan = [(sid, stx[i]) for i in range(R)]
        shapes = {sid: (H, W)}
        serve_run(ctx, plan[:4 * Bq], shapes)  # warm-up (graph capture)
        sat, lat_s, st_s = serve_run(ctx, plan, shapes, depth=4 * Bq)
        rate = 0.7 * sat
        thr_p, lat_p, st_p = serve_run(ctx, plan, shapes, rate=rate, depth=1 << 30)
        cnt = ctx.serve_counters()
        ctx.serve_stop()
        rec["serving"] = {
            "saturation_spectra_per_s": sat, "saturation_p50_us": pct(lat_s, 50), "saturation_p99_us": pct(lat_s, 99),
            "poisson_rate_per_s": rate, "poisson_throughput": thr_p, "poisson_p50_us": pct(lat_p, 50),
            "poisson_p99_us": pct(lat_p, 99), "poisson_mean_batch": float(np.mean([s["batch"] for s in st_p])),
            "requests_per_point": R, "slots": 3, "max_batch": Bq, "graphs": True, "fallbacks": cnt["fallbacks"],
            "mode": "mixed" if cnt["mixed_launches"] == cnt["launches"] else "per_scene",
            "note": "latency from scheduled arrival to the result in the caller's host buffer"}
        rec["latency_us"]["serving_p50"] = pct(lat_p, 50)
        rec["latency_us"]["serving_p99"] = pct(lat_p, 99)
        if not a.no_cpu_baseline:
            rec["cpu_baseline"] = cpu_baseline(g, Ws, bs, H, W, txs[:8], a.cpu_seconds)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
