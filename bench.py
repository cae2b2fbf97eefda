#!/usr/bin/env python
"""Throughput of the denoiser's hot path on one MI355X.

One step = one whole pass of the pipeline (Morton sort, octree, voxel filter,
kNN, density, percentile/median, score, top-lambda, compaction) over one
synthetic 120k-point LiDAR frame at k=32, leaf cap 1024, with the input already
resident in HBM. Prints ONE JSON line on stdout; progress goes to stderr.

The line also carries the batched form ("batched vs plain"): 64 uneven LiDAR
frames (6.2M points) in one pipeline pass, leaf cap and kNN chunk picked by the
autotuner, replayed from a captured HIP graph, beside the same frames run one
plain call at a time, and the served form ("served"): a Poisson stream from 16
sensors at 10 Hz through the continuous-batching server (p50/p99 latency),
plus a saturating burst of 128 frames through the same server.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-batch] [--no-serve]
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X: 256 CU x 2.4 GHz x 256 flop/clk (packed FMA)
FP32_PACKED_NO_FMA_TOPS = 78.6      # two fp32 ops per lane-cycle (packed add/mul, no FMA)
FP32_EXACT_CEILING_TOPS = 39.3       # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, one op per lane-cycle
FLOPS_PER_PAIR = 8                   # 3 sub + 3 mul + 2 add per (query, candidate) pair


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def knn_traffic(name="knn_lidar_120k_traffic.json"):
    """HBM bytes per kNN launch from a committed PMC summary, if it was taken
    on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2512_10386_amd", "csrc", "knn.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("knn_source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(xyz, params, workload, budget_s=12.0, single_budget_s=10.0):
    """The CPU oracle, as it stands, on the host cores: whole frames until the
    time budget is used (at least one); then the same with one thread, in a
    child process started with OMP_NUM_THREADS=1."""
    import subprocess
    from oracle import oracle as O
    O.build()
    reps, t0 = 0, time.perf_counter()
    threads = 1
    while True:
        r = O.denoise(xyz, **params)
        threads = r["threads"]
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 30:
            break
    rec = {"value": round(xyz.shape[0] * reps / el / 1e6, 4), "unit": "Mpoints/s",
           "cores": int(threads), "kind": "oracle",
           "sample": f"{reps} full frames of the same workload ({xyz.shape[0]} points each), "
                     f"{el:.1f} s wall"}
    child = (
        "import sys, time, json\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle import oracle as O\n"
        "from paper_2512_10386_amd import synth\n"
        f"xyz, _, p = synth.make({workload!r})\n"
        "reps, t0 = 0, time.perf_counter()\n"
        "while True:\n"
        "    r = O.denoise(xyz, **p); reps += 1; el = time.perf_counter() - t0\n"
        f"    if el >= {single_budget_s} or reps >= 10: break\n"
        "print(json.dumps(dict(reps=reps, el=el, n=int(xyz.shape[0]), threads=int(r['threads']))))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True,
                             timeout=single_budget_s * 6 + 60)
        one = json.loads(out.stdout.strip().splitlines()[-1])
        rec["single_thread"] = {"value": round(one["n"] * one["reps"] / one["el"] / 1e6, 4), "unit": "Mpoints/s",
                                "cores": one["threads"],
                                "sample": f"{one['reps']} full frames, {one['el']:.1f} s wall"}
    except (subprocess.SubprocessError, ValueError, IndexError, KeyError) as e:
        rec["single_thread"] = {"error": str(e)[:200]}
    return rec


def bench_batch(steps, cap=0, chunk=0, plain_loop=True):
    """The 64-frame batch: autotune (unless cap is given), graph replay, eager
    batch, and the same frames as plain calls (unless plain_loop is False)."""
    import numpy as np
    import torch
    from paper_2512_10386_amd import synth
    from paper_2512_10386_amd.binding import BatchDenoiser, Denoiser, gdn_set_timing, gdn_timing

    frames, _, params = synth.make("lidar_batch_64")
    sizes = [len(f) for f in frames]
    off = np.zeros(len(frames) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    n, nf = int(off[-1]), len(frames)
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(np.concatenate(frames)).to(dev)
    offd = torch.from_numpy(off).to(dev)
    log(f"[bench] batch: {nf} frames, {n} points (min {min(sizes)}, max {max(sizes)})")
    if cap:
        bd = BatchDenoiser(0, **dict(params, leaf_cap=cap, knn_chunk=chunk))
        table = {}
        log(f"[bench] batch at leaf_cap {cap}, knn_chunk {chunk} (no autotune)")
    else:
        bd = BatchDenoiser(0, **params)
        table = bd.autotune(xyz, offd, caps=synth.LIDAR_BATCH_CAPS, chunks=(8192, 16384, 32768), reps=2)
        cap, chunk = bd.params.leaf_cap, bd.params.knn_chunk
        log(f"[bench] autotune -> leaf_cap {cap}, knn_chunk {chunk}")
    out = bd.alloc(n, nf)
    for _ in range(3):
        bd.graph(xyz, offd, out)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        bd.graph(xyz, offd, out)
    t1.record()
    torch.cuda.synchronize()
    ms_graph = t0.elapsed_time(t1) / steps
    # eager batch calls, then again with the library's kNN-kernel events
    t0.record()
    for _ in range(steps):
        bd(xyz, offd, out)
    t1.record()
    torch.cuda.synchronize()
    ms_eager = t0.elapsed_time(t1) / steps
    gdn_set_timing(bd.ctx, True)
    for _ in range(steps):
        bd(xyz, offd, out)
    torch.cuda.synchronize()
    per = [gdn_timing(bd.ctx, b) for b in range(steps)]
    gdn_set_timing(bd.ctx, False)
    knn_ms = statistics.fmean(k for _, k in per)
    bd.check_status(n)
    counts = bd.dump("COUNTS", n).cpu().numpy()
    pairs = int(counts[2])
    ms_plain = None
    if plain_loop:
        # the same frames as plain single-frame calls, back to back
        pd = Denoiser(0, **dict(params, leaf_cap=cap, knn_chunk=chunk))
        xs = [xyz[int(off[f]):int(off[f + 1])] for f in range(nf)]
        outs = []
        for x in xs:
            outs.append(pd(x))
        torch.cuda.synchronize()
        t0.record()
        reps = max(1, steps // 4)
        for _ in range(reps):
            for x, o in zip(xs, outs):
                pd(x, o)
        t1.record()
        torch.cuda.synchronize()
        ms_plain = t0.elapsed_time(t1) / reps
        pd.close()
    bd.close()
    mp = lambda ms: round(n / (ms * 1e-3) / 1e6, 2) if ms else None
    res = {"workload": "lidar_batch_64", "frames": nf, "points": n, "k": params["k"],
           "leaf_cap": cap, "knn_chunk": chunk, "steps": steps,
           "ms_per_batch_graph": round(ms_graph, 4), "ms_per_batch_eager": round(ms_eager, 4),
           "ms_plain_loop": round(ms_plain, 4) if ms_plain else None,
           "mpoints_s_graph": mp(ms_graph), "mpoints_s_eager": mp(ms_eager), "mpoints_s_plain_loop": mp(ms_plain),
           "knn_kernel_ms": round(knn_ms, 4), "pairs": pairs,
           "knn_tflops_algorithmic": round(pairs * FLOPS_PER_PAIR / (knn_ms * 1e-3) / 1e12, 3),
           "autotune_ms": {f"{c}/{h}": round(v, 3) for (c, h), v in table.items()}}
    achieved = pairs * FLOPS_PER_PAIR / (knn_ms * 1e-3) / 1e12
    res["roofline"] = {"kernel": "knn_group_kernel", "bound": "alu", "achieved": round(achieved, 3),
                       "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                       "traffic": knn_traffic("knn_lidar_batch64_traffic.json") if cap == 256 else None,
                       "pairs_per_launch": pairs, "flops_per_pair": FLOPS_PER_PAIR, "kernel_ms": round(knn_ms, 5),
                       "exact_fp32_ceiling": FP32_EXACT_CEILING_TOPS,
                       "frac_of_exact_ceiling": round(achieved / FP32_EXACT_CEILING_TOPS, 4)}
    log(f"[bench] batch: graph {ms_graph:.3f} ms ({res['mpoints_s_graph']} Mpts/s), eager {ms_eager:.3f} ms, "
        f"plain loop {ms_plain or 0:.3f} ms ({res['mpoints_s_plain_loop']} Mpts/s), kNN {knn_ms:.3f} ms")
    return res


SERVE_SLOT_POINTS = 4 << 20   # points per slot batch (the large-input kernels run above 2^20)
SERVE_SLOT_FRAMES = 64


def bench_serve(seconds):
    """The served stream: 16 sensors at 10 Hz (Poisson arrivals) sending frames
    of 20k-130k points through the continuous-batching server, with the frames
    already on the device and again arriving in pinned host memory (copied on a
    copy stream); then the same server saturated with a burst of 128 frames."""
    import numpy as np
    import torch
    from paper_2512_10386_amd import synth
    from paper_2512_10386_amd.serve import Server, simulate

    frames, _, params = synth.make("lidar_stream_pool")
    dev = torch.device("cuda", 0)
    devs = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames]
    hosts = [torch.from_numpy(np.ascontiguousarray(f)).pin_memory() for f in frames]
    srv = Server(0, hbm_budget=32 << 30, max_slots=4, slot_points=SERVE_SLOT_POINTS, slot_frames=SERVE_SLOT_FRAMES,
                 **params)
    log(f"[bench] serve: {len(frames)}-frame pool, {srv.n_slots} slots of {srv.bytes_per_slot / 2**20:.0f} MiB")
    warm = min(2.0, seconds / 5)
    r = simulate(srv, devs, n_sensors=16, rate_hz=10.0, duration_s=seconds + warm, warmup_s=warm, seed=5, log=log)
    log(f"[bench] serve: {r['frames']} frames, p50 {r['p50_ms']:.3f} ms, p99 {r['p99_ms']:.3f} ms, "
        f"{r['mpoints_s']:.2f} Mpts/s (offered)")
    rh = simulate(srv, hosts, n_sensors=16, rate_hz=10.0, duration_s=seconds + warm, warmup_s=warm, seed=6, log=log)
    log(f"[bench] serve from host memory: {rh['frames']} frames, p50 {rh['p50_ms']:.3f} ms, "
        f"p99 {rh['p99_ms']:.3f} ms")
    # saturation: 128 frames submitted at once, time until the last is done
    order = [i % len(devs) for i in range(128)]
    outs = [srv.alloc(devs[i].shape[0]) for i in order]
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        for i, o in zip(order, outs):
            srv.submit(devs[i], o)
        left = len(order)
        while left:
            fin, _, _ = srv.poll()
            left -= len(fin)
            if time.perf_counter() - t0 > 60:
                raise RuntimeError("server burst did not finish")
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    pts = sum(devs[i].shape[0] for i in order)
    srv.close()
    # the same 128 frames as one batch replayed from a graph: the batched
    # path's rate on exactly this work
    from paper_2512_10386_amd.binding import BatchDenoiser
    off = np.zeros(len(order) + 1, np.int64)
    off[1:] = np.cumsum([devs[i].shape[0] for i in order])
    xb = torch.cat([devs[i] for i in order])
    ob = torch.from_numpy(off).to(dev)
    bd = BatchDenoiser(0, **dict(params, knn_chunk=32768))
    ob_out = bd.alloc(xb.shape[0], len(order))
    for _ in range(3):
        bd.graph(xb, ob, ob_out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        bd.graph(xb, ob, ob_out)
    e1.record()
    torch.cuda.synchronize()
    ms_ref = e0.elapsed_time(e1) / 10
    bd.close()
    r.update({"workload": "lidar_stream_16x10hz", "sensors": 16, "rate_hz": 10.0, "k": params["k"],
              "leaf_cap": params["leaf_cap"], "pool_frames": len(frames), "slot_points": SERVE_SLOT_POINTS,
              "slot_frames": SERVE_SLOT_FRAMES,
              "pool_points_min": min(f.shape[0] for f in frames), "pool_points_max": max(f.shape[0] for f in frames),
              "burst_frames": len(order), "burst_points": pts, "burst_ms": round(best * 1e3, 3),
              "burst_mpoints_s": round(pts / best / 1e6, 2),
              "burst_as_one_graph_batch_ms": round(ms_ref, 3),
              "burst_vs_batched": round(ms_ref / (best * 1e3), 3),
              "from_host": {"frames": rh["frames"], "p50_ms": round(rh["p50_ms"], 4), "p99_ms": round(rh["p99_ms"], 4),
                            "max_ms": round(rh["max_ms"], 4),
                            "how": "each frame in pinned host memory, copied on a copy stream, submitted when copied"}})
    for key in ("p50_ms", "p99_ms", "max_ms", "mpoints_s"):
        r[key] = round(r[key], 4)
    log(f"[bench] serve burst: {len(order)} frames in {best * 1e3:.2f} ms ({r['burst_mpoints_s']} Mpts/s); "
        f"as one graph batch {ms_ref:.2f} ms")
    return r


def bench_ablation(reps):
    """Module switches of Tables 8/9 on the 20k scanned-object stand-in:
    F1, PSNR, CD and GPU ms per frame for each combination."""
    from paper_2512_10386_amd import synth
    from paper_2512_10386_amd.evaluate import ablation
    xyz, label, params = synth.make("sphere_plane_20k")
    rows = ablation(xyz, label, params, reps=reps)
    for r in rows:
        log(f"[bench] ablation {r['name']:>20}: F1 {r['f1']:.4f} PSNR {r['psnr_db']:.2f} dB "
            f"CD {r['cd']:.3e} {r['ms']:.3f} ms")
    def num(v):  # JSON has no inf/NaN: a PSNR of +inf (nothing clean lost) is reported as null
        return (round(v, 6) if math.isfinite(v) else None) if isinstance(v, float) else v
    return {"workload": "sphere_plane_20k", "points": int(xyz.shape[0]), "k": params["k"],
            "rows": [{k: num(v) for k, v in r.items()} for r in rows]}


def bench_fit(steps):
    """Score fit on the three 200k-point frames (one batch): time of one
    loss + gradient evaluation, and a short Adam run from the defaults with
    F1 of the fitted threshold rule against the plain top-lambda rule."""
    import numpy as np
    import torch
    from paper_2512_10386_amd import synth
    from paper_2512_10386_amd.binding import BatchDenoiser
    from paper_2512_10386_amd.fit import ScoreFit, f1_scores, fit_params
    xs, ls, params = synth.make("fit_200k")
    off = np.zeros(len(xs) + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in xs])
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(np.concatenate(xs)).to(dev)
    lab_np = np.concatenate(ls)
    lab = torch.from_numpy(lab_np).to(dev)
    offd = torch.from_numpy(off).to(dev)
    sf = ScoreFit(xyz, lab, frame_off=offd, temperature=0.5, **params)
    torch.cuda.synchronize()
    score = sf.res.score.cpu().numpy()
    p2 = score >= 0
    tau0 = float(np.median(np.log(score[p2])))
    for _ in range(3):
        sf.loss_grad(1.0, 1.0, 2.0, tau0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        sf.loss_grad(1.0, 1.0, 2.0, tau0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    theta, losses = fit_params(sf, [1.0, 1.0, 2.0, tau0], steps=steps, lr=0.05)
    plain_keep = sf.res.keep.cpu().numpy()
    sf.close()
    bd = BatchDenoiser(0, **dict(params, alpha=theta[0], sigma=theta[1], gamma=theta[2], log_threshold=theta[3]))
    fitted_keep = bd(xyz, offd).keep.cpu().numpy()
    bd.close()
    f_plain = f1_scores(plain_keep, lab_np)[2]
    f_fit = f1_scores(fitted_keep, lab_np)[2]
    log(f"[bench] fit: loss+grad {ms:.3f} ms over {int(off[-1])} points; loss {losses[0]:.4f} -> {losses[-1]:.4f}; "
        f"F1 plain {f_plain:.4f} fitted {f_fit:.4f}")
    return {"workload": "fit_200k", "points": int(off[-1]), "frames": len(xs), "k": params["k"],
            "ms_loss_grad": round(ms, 4), "adam_steps": steps, "loss_first": round(losses[0], 6),
            "loss_last": round(losses[-1], 6), "theta_alpha_sigma_gamma_tau": [round(v, 5) for v in theta],
            "f1_plain_top_lambda": round(f_plain, 5), "f1_fitted_threshold": round(f_fit, 5)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="lidar_120k")
    ap.add_argument("--latency-frames", type=int, default=1000, help="solo frames timed for p50/p99")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (64-frame) leg")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-cap", type=int, default=0, help="batch leaf cap (skips the autotuner)")
    ap.add_argument("--batch-chunk", type=int, default=32768, help="batch kNN chunk with --batch-cap")
    ap.add_argument("--no-plain-loop", action="store_true", help="skip the batch frames as plain calls")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream leg")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-extras", action="store_true", help="skip the ablation and fit legs")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(frames are independent, so several GPUs would each take whole frames).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_10386_amd import synth
    from paper_2512_10386_amd.binding import Denoiser, gdn_set_timing, gdn_timing

    xyz, label, params = synth.make(args.workload)
    n = xyz.shape[0]
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(xyz).to(dev)
    den = Denoiser(0, **params)
    out = den(x)
    torch.cuda.synchronize()
    counts = den.dump("COUNTS", n).cpu().numpy()
    status = int(den.dump("STATUS", n).cpu().numpy()[0])
    n_leaves, n_p1, pairs, n_kept = (int(c) for c in counts)
    log(f"[bench] {args.workload}: n={n} leaves={n_leaves} |P1|={n_p1} pairs={pairs} kept={n_kept} status={status}")
    if status != 0:
        log("[bench] device status word is non-zero")

    if args.copy_calib_mib:
        a = torch.empty(args.copy_calib_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        den(x, out)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")

    # timed region: K back-to-back frames (the library's own per-call events
    # are off here: each event record drains the queue for a few us)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t_start.record()
    for _ in range(args.steps):
        den(x, out)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = t_start.elapsed_time(t_end)
    ms_per_step = ms_total / args.steps
    # the kNN kernel's duration: the same frames again with HIP events around
    # that kernel on the library's stream
    gdn_set_timing(den.ctx, True)
    n_knn = min(max(args.steps, 1), 256)
    for _ in range(n_knn):
        den(x, out)
    torch.cuda.synchronize()
    per_call = [gdn_timing(den.ctx, b) for b in range(n_knn)]
    knn_ms = statistics.fmean(k for _, k in per_call)
    call_ms = statistics.fmean(t for t, _ in per_call)
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step (host wall {wall:.3f} s); "
        f"with kNN events: kNN kernel {knn_ms:.4f} ms, call {call_ms:.4f} ms")
    gdn_set_timing(den.ctx, False)

    den.check_status(n)

    # frame latency: each frame submitted alone and waited for (host clock
    # from the call to the end of a synchronize), over --latency-frames frames
    lat = []
    for _ in range(args.latency_frames):
        s = time.perf_counter()
        den(x, out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - s) * 1e3)
    lat = np.array(lat)
    p50 = p99 = None
    if len(lat):
        p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
        log(f"[bench] latency over {len(lat)} solo frames: p50 {p50:.4f} ms p99 {p99:.4f} ms max {lat.max():.4f} ms")

    flops = pairs * FLOPS_PER_PAIR
    achieved = flops / (knn_ms * 1e-3) / 1e12
    roofline = {
        "kernel": "knn_group_kernel",
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
        "traffic": knn_traffic(),
        "pairs_per_launch": pairs,
        "flops_per_pair": FLOPS_PER_PAIR,
        "kernel_ms": round(knn_ms, 5),
        "packed_no_fma_ceiling": FP32_PACKED_NO_FMA_TOPS,
        "exact_fp32_ceiling": FP32_EXACT_CEILING_TOPS,
        "frac_of_exact_ceiling": round(achieved / FP32_EXACT_CEILING_TOPS, 4),
    }

    value = n / (ms_per_step * 1e-3) / 1e6
    rec = {
        "metric": "Mpoints/s denoised at k=32 (kNN+score) + p99 frame latency; batched vs plain",
        "value": round(value, 4),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "points": n, "k": params["k"],
                   "leaf_cap": params["leaf_cap"], "frames_per_step": 1, "path": "plain single-frame",
                   "score_dtype": "f64", "leaves": n_leaves, "p1_points": n_p1, "kept": n_kept},
        "latency_ms": {"p50": round(p50, 4) if p50 else None, "p99": round(p99, 4) if p99 else None,
                       "frames": int(len(lat)),
                       "how": "solo frames, host clock from the call to the end of a device synchronize"},
        "roofline": roofline,
    }
    if not args.no_batch:
        rec["batched"] = bench_batch(args.batch_steps, args.batch_cap, args.batch_chunk, not args.no_plain_loop)
    if not args.no_serve:
        rec["served"] = bench_serve(args.serve_seconds)
    if not args.no_extras:
        rec["ablation"] = bench_ablation(10)
        rec["fit"] = bench_fit(60)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(xyz, params, args.workload)
        log(f"[bench] cpu baseline {rec['cpu_baseline']}")
    print(json.dumps(rec, allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
