"""Throughput benchmark of the lane-detection hot path on one MI355X.

One step = ld_detect over a batch of synthetic 1242x375 frames already resident in HBM
(grey u8 + f32 subpixel disparity, 4 curved lanes, ~10% obstacle pixels, 16 sequences of
64 frames).  Prints one JSON line: frames/s and ms per step (timed with no per-kernel
events), the roofline of the dominant kernel (its algorithmic bytes or operations per launch
over its average launch time, HIP events on the launch stream, in a separate pass), the
whole path's fraction of the HBM roofline, other batch sizes, the 1920x1080 u16 throughput
stream, single-frame latency p50/p99, the learned-pruned path, a serving run, and the CPU
oracle timed on the host's cores (one core and all cores, median of five runs each).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 32-bit VALU lanes per clock x 2.4 GHz = 39.3 T ops/s
METRIC = "frames/s @1242x375 on 1 MI355X, plain vs learned-pruned; p99 latency; % HBM"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _gen(args):
    from paper_1807_02752_amd import synth
    seed, start, count = args
    g, d, _ = synth.make_batch("c2", seed, count, start)
    return g, d


def make_workload(n_seq: int, per_seq: int, procs: int, first_seq: int = 0):
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(s, i, min(16, per_seq - i)) for s in range(first_seq, first_seq + n_seq) for i in range(0, per_seq, 16)]
    greys, disps = [], []
    with ProcessPoolExecutor(max_workers=procs) as ex:
        for g, d in ex.map(_gen, jobs):
            greys.append(g)
            disps.append(d)
    return np.concatenate(greys), np.concatenate(disps)


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "lane_path_1242x375_hbm_bytes.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic_json:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in ("ld.hip", "ld_device.h"):
        h.update(open(os.path.join(ROOT, "paper_1807_02752_amd", "csrc", f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"].get(kernel)


SERVE_CLASSES = [(640, 192, 0, 96, 16), (1242, 375, 0, 128, 16), (1920, 1080, 0, 255, 16)]
SERVE_STREAMS, SERVE_FPS, SERVE_POOL = 32, 30.0, 4


def _gen_serving(args):
    from paper_1807_02752_amd import synth
    stream, cls = args
    W, H, _, dm, _ = SERVE_CLASSES[cls]
    return [synth.make_scaled_c1(W, H, dm, seed=100 + stream, idx=i)[:2] for i in range(SERVE_POOL)]


def make_serving_pool(procs: int):
    """32 camera streams, each of a resolution class drawn uniformly (seeded), with a few
    u8 frames of the scaled 320x96 generator per stream, cycled by the arrivals."""
    from concurrent.futures import ProcessPoolExecutor
    rng = np.random.default_rng(7)
    classes = rng.integers(0, len(SERVE_CLASSES), SERVE_STREAMS).tolist()
    with ProcessPoolExecutor(max_workers=procs) as ex:
        frames = list(ex.map(_gen_serving, list(enumerate(classes))))
    return classes, frames


def serving_leg(args, pool, net=None):
    """Continuous batching: every stream submits frames as Poisson arrivals at 30 fps for
    serve_seconds of wall time while the host polls; latency is arrival to host-visible
    result.  With `net` the engines run the pruned path (plain fallback per frame)."""
    import torch
    from paper_1807_02752_amd import ld
    classes, frames = pool
    dev = [[(torch.from_numpy(gr).cuda(), torch.from_numpy(dp).cuda()) for gr, dp in fr] for fr in frames]
    cfg = ld.server_config(SERVE_CLASSES, n_streams=SERVE_STREAMS, inflight=2, max_queue=1024, use_graphs=True,
                           cnn=net)
    srv = ld.Server(cfg)
    rng = np.random.default_rng(11)
    T = args.serve_seconds
    arrivals = []
    for s in range(SERVE_STREAMS):
        t = rng.exponential(1.0 / SERVE_FPS)
        while t < T:
            arrivals.append((t, s))
            t += rng.exponential(1.0 / SERVE_FPS)
    arrivals.sort()
    # warm-up: one frame of every class through the server (graph capture happens here)
    for c in range(len(SERVE_CLASSES)):
        s = classes.index(c) if c in classes else None
        if s is not None:
            srv.submit(s, c, *dev[s][0])
    while sum(srv.pending()) > 0:
        srv.poll()
    lat, done, k = [], 0, 0
    count = {s: 0 for s in range(SERVE_STREAMS)}
    t0 = time.perf_counter()
    while k < len(arrivals) or sum(srv.pending()) > 0:
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k][0] <= now:
            s = arrivals[k][1]
            gr, dp = dev[s][count[s] % SERVE_POOL]
            count[s] += 1
            st, _ = srv.submit(s, classes[s], gr, dp)
            assert st == ld.LD_OK, st
            k += 1
        for r in srv.poll():
            lat.append((r["t_done"] - r["t_submit"]) * 1e3)
            done += 1
    wall = time.perf_counter() - t0
    pc, mem = srv.engines()
    srv.close()
    lat = np.array(lat)
    return {"streams": SERVE_STREAMS, "offered_fps": len(arrivals) / T, "achieved_fps": done / wall,
            "requests": done, "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "classes": [f"{w}x{h}" for w, h, *_ in SERVE_CLASSES], "streams_per_class": [classes.count(c) for c in range(3)],
            "engines_per_class": pc[:3], "engine_bytes": mem, "graphs": True, "pruning": net is not None}


def learned_leg(args, det, g, d, lanes, plain_lanes, tgreys, tdisps, plain_ms):
    """Train the pruning network on the GPU (frames of other sequences, labels from the plain
    search), then time ld_detect_pruned on the same batch and compare its lanes with the plain
    search's."""
    import torch
    from paper_1807_02752_amd import ld
    from paper_1807_02752_amd import train as tr
    B = g.shape[0]
    t0 = time.time()
    G, D = torch.from_numpy(tgreys).cuda(), torch.from_numpy(tdisps).cuda()
    net, losses = tr.train(G, D, 128, steps=args.train_steps, batch=16, lr=3e-3, pos_weight=4.0, seed=0)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    del G, D
    log(f"trained {args.train_steps} steps in {train_s:.1f}s, loss {losses[:10].mean():.4f} -> {losses[-10:].mean():.4f}")
    lp = det.lanes_buffer()
    ms = time_steps(lambda: det.detect_pruned(net, g, d, lp), args.steps, args.warmup)
    det.profile(True)                  # kernel times in a pass of their own
    for _ in range(args.steps):
        det.detect_pruned(net, g, d, lp)
    kt = det.kernel_times()
    det.profile(False)
    L = ld.Detector.parse_lanes(lp)
    diff = tot = 0
    for a, b in zip(plain_lanes, L):
        sa, sb = set(a["u_start"][: a["n"]].tolist()), set(b["u_start"][: b["n"]].tolist())
        diff += len(sa ^ sb)
        tot += len(sa)
    fb = [det.read(ld.LD_STATE_PRUNE, b)[1] for b in range(B)]
    cfg = net.config
    res = {"value": B / (ms / 1e3), "unit": "frames/s", "ms_per_step": ms, "speedup_vs_plain": plain_ms / ms,
           "lane_disagreement": diff / max(tot, 1), "lanes_compared": tot,
           "fallback_frac": float(np.mean([(x & 3) != 0 for x in fb])),
           # per step, all launches of a kernel summed (k_energy and k_peaks run a second time,
           # for the frames that fell back to the plain search, usually with every frame masked)
           "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items() if v[1]},
           "network": {"n_bands": cfg.n_bands, "theta": round(cfg.theta, 3), "delta_x": cfg.delta_x,
                       "dilate": cfg.dilate, "seed_ransac": cfg.seed_ransac, "params": ld.LD_CNN_PARAMS},
           "train": {"steps": args.train_steps, "batch": 16, "frames": int(tgreys.shape[0]), "seconds": round(train_s, 2),
                     "loss_first10": float(losses[:10].mean()), "loss_last10": float(losses[-10:].mean())}}
    log(f"pruned: {ms:.3f} ms/step ({plain_ms / ms:.2f}x plain), disagreement {res['lane_disagreement']:.4f}, "
        f"fallback {res['fallback_frac']:.3f}")
    return res, net


def host_cores():
    """Cores this process may run on: the affinity set, capped by the cgroup CPU quota."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            n = max(1, min(n, int(int(q) // int(per))))
    except (OSError, ValueError):
        pass
    return n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(greys, disps, seconds: float):
    """The oracle, as it stands, on the host cores: one core (frames in sequence) and all
    cores (one thread per core, frames split over the threads; ctypes releases the GIL during
    each call).  Each figure is the median of five runs over a bounded sample of the timed
    workload, sized so that the ten runs take about `seconds` of wall time."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()
    oracle.detect(greys[0], disps[0], 128)               # warm-up (page-in, library load)
    t0 = time.perf_counter()
    oracle.detect(greys[1], disps[1], 128, frame_idx=1)
    t1 = time.perf_counter() - t0
    cores = host_cores()
    per_run = max(1, int(seconds / 10 / t1))             # frames one core does in one run
    one, allc = [], []
    for r in range(5):
        idx = [(r * per_run + i) % len(greys) for i in range(per_run)]
        t0 = time.perf_counter()
        for i in idx:
            oracle.detect(greys[i], disps[i], 128, frame_idx=i)
        one.append(len(idx) / (time.perf_counter() - t0))
    n_all = per_run * cores
    with ThreadPoolExecutor(max_workers=cores) as ex:
        for r in range(5):
            idx = [(r * n_all + i) % len(greys) for i in range(n_all)]
            t0 = time.perf_counter()
            list(ex.map(lambda i: oracle.detect(greys[i], disps[i], 128, frame_idx=i), idx))
            allc.append(len(idx) / (time.perf_counter() - t0))
    return {"value": float(np.median(allc)), "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"median of 5 runs of {n_all} frames of the 1242x375 workload on {cores} threads "
                      f"(one per core); single core: median of 5 runs of {per_run} frames in sequence",
            "single_core": {"value": float(np.median(one)), "unit": "frames/s", "cores": 1,
                            "ms_per_frame": 1e3 / float(np.median(one))},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


# Algorithmic work per frame of each kernel, for its roofline (units: bytes for "hbm", 32-bit
# lane operations for "alu").  The HBM figures are the compulsory reads of the input images
# (the disparity once for the histogram, the grey image once for the gradient); the kernels
# between them move only intermediates, priced at zero bytes, and are bound by their
# arithmetic instead.
def kernel_work(k, W, H, R, es, p):
    N = W * H
    if k == "k_vdisp_hist":
        return "hbm", N * es, f"{N * es} B per frame (disparity read once)"
    if k == "k_edges":
        return "hbm", N * 1, f"{N} B per frame (grey read once)"
    if k == "k_vpx_fit":
        ops = R * 2 * W * (2 * p.tau_x_max + 1) * 2
        return "alu", ops, f"{ops:.4g} ops per frame (row DP: R x 2W x 11 taps x add+min)"
    if k == "k_energy":
        ops = R * (W * 16 + 2 * W * 6)
        return "alu", ops, (f"{ops:.4g} ops per frame (per road row: 16 per pixel for q scatter, 7-row and 3-column "
                            f"box sums and M_1; 6 per candidate for the track fma, rounding, range test, gather-add)")
    if k == "k_vdisp_fit":
        ops = (128 + 1) * H * (p.tau_y_max + 1) * 2
        return "alu", ops, f"{ops:.4g} ops per frame (v-disparity DP: D x H x 7 taps x add+min)"
    if k == "k_vpx_ransac":
        ops = R * 64 * 2 * 16
        return "alu", ops, f"{ops:.4g} ops per frame (64 quartic hypotheses x R points x ~16 ops, two rounds)"
    ops = 2 * W * 4
    return "alu", ops, f"{ops:.4g} ops per frame (2W candidates x compare/select)"


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def c3_leg(args):
    """Throughput stream of 1920x1080 frames: u16 disparity in 1/16 px up to 255 px, 6 lanes
    (inner 4 dashed), 15% obstacle pixels, grey gain redrawn every 50 frames.  `c3_distinct`
    frames are generated and tiled to `c3_frames` (each position keeps its own frame index,
    hence its own RANSAC draws)."""
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_1807_02752_amd import ld
    n = args.c3_distinct
    jobs = [(0, i, min(10, n - i)) for i in range(0, n, 10)]
    with ProcessPoolExecutor(max_workers=args.procs) as ex:
        parts = list(ex.map(_gen_c3, jobs))
    greys = np.concatenate([q[0] for q in parts])
    disps = np.concatenate([q[1] for q in parts])
    reps = (args.c3_frames + n - 1) // n
    g = torch.from_numpy(greys).cuda().repeat(reps, 1, 1)[: args.c3_frames].contiguous()
    d = torch.from_numpy(disps).cuda().repeat(reps, 1, 1)[: args.c3_frames].contiguous()
    del greys, disps
    B, H, W = g.shape
    det = ld.Detector(W, H, B, ld.LD_DISP_U16Q4, 255)
    lanes = det.lanes_buffer()
    ms = time_steps(lambda: det.detect(g, d, lanes), max(2, args.steps // 4), 1)
    L = ld.Detector.parse_lanes(lanes)
    det.close()
    fps = B / (ms / 1e3)
    alg = W * H * 3
    return {"workload": f"{B} frames 1920x1080, u16 disparity (1/16 px, d_max 255), 6 lanes, 15% obstacles, gain "
                        f"changes every 50 frames ({n} generated, tiled)", "frames_per_step": B,
            "value": fps, "unit": "frames/s", "ms_per_step": ms, "alg_bytes_per_frame": alg,
            "hbm_frac": alg * fps / (HBM_PEAK_GBS * 1e9), "lanes_per_frame": float(L["n"].mean())}


def _gen_c3(args):
    from paper_1807_02752_amd import synth
    seed, start, count = args
    g, d, _ = synth.make_batch("c3", seed, count, start)
    return g, d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sequences", type=int, default=16)
    ap.add_argument("--per-seq", type=int, default=64)
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--train-steps", type=int, default=300, help="training steps of the pruning network (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="length of the serving run (0: skip)")
    ap.add_argument("--c3-frames", type=int, default=1000, help="frames of the 1920x1080 stream (0: skip)")
    ap.add_argument("--c3-distinct", type=int, default=250, help="distinct 1920x1080 frames generated")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (4 launches) to calibrate HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every box here has a single MI355X, and the path shards by "
              "camera stream with no exchange (see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib > 0:
        n = args.copy_calib << 18
        src = torch.arange(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            torch.mul(src, 1.0, out=dst)       # one elementwise kernel: reads and writes 4n bytes
        torch.cuda.synchronize()
        log(f"copy calibration: 4 launches of {4 * n} B read + {4 * n} B written")
        return
    from paper_1807_02752_amd import ld

    t0 = time.time()
    greys, disps = make_workload(args.sequences, args.per_seq, args.procs)
    B, H, W = greys.shape
    if args.train_steps > 0:     # training frames: other sequences than the timed workload
        tgreys, tdisps = make_workload(16, 16, args.procs, first_seq=1000)
    serve_pool = make_serving_pool(args.procs) if args.serve_seconds > 0 else None
    log(f"generated {B} frames {W}x{H} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = torch.from_numpy(greys).to(dev)
    d = torch.from_numpy(disps).to(dev)
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    lanes = det.lanes_buffer()

    # headline: whole steps with no per-kernel events
    ms_per_step = time_steps(lambda: det.detect(g, d, lanes), args.steps, args.warmup)
    fps = B / (ms_per_step / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {fps:.0f} frames/s")

    # per-kernel launch times in a separate pass (HIP events on the launch stream)
    det.profile(True)
    for _ in range(args.steps):
        det.detect(g, d, lanes)
    ktimes = det.kernel_times()
    det.profile(False)
    lanes_np = ld.Detector.parse_lanes(lanes)
    infos = np.stack([det.read(ld.LD_STATE_INFO, b) for b in range(min(B, 64))])
    R_mean = float(infos[:, 6].mean())
    kern = {k: {"ms_per_launch": v[0] / max(v[1], 1), "launches": int(v[1])} for k, v in ktimes.items() if v[1]}
    dom = max(kern, key=lambda k: kern[k]["ms_per_launch"])
    t_dom = kern[dom]["ms_per_launch"] / 1e3
    p = det.params
    bound, per_unit, desc = kernel_work(dom, W, H, R_mean, 4, p)
    if bound == "hbm":
        roof = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": per_unit * B / t_dom / 1e9}
    else:
        roof = {"bound": "alu", "unit": "TOP/s", "peak": ALU_PEAK_TOPS, "achieved": per_unit * B / t_dom / 1e12}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom)
    roof.update({"kernel": dom, "per_unit": desc, "units_per_launch": B, "launch_ms": kern[dom]["ms_per_launch"]})
    per_kernel_roof = {}
    for k, v in kern.items():
        bnd, pu, _ = kernel_work(k, W, H, R_mean, 4, p)
        t = v["ms_per_launch"] / 1e3
        ach = pu * B / t / (1e9 if bnd == "hbm" else 1e12)
        per_kernel_roof[k] = {"ms": round(v["ms_per_launch"], 4), "bound": bnd,
                              "frac": round(ach / (HBM_PEAK_GBS if bnd == "hbm" else ALU_PEAK_TOPS), 4)}

    # other batch sizes (the first frames of the same workload)
    batches = {}
    for nb in (64, 256):
        det.set_active(nb)
        ms = time_steps(lambda: det.detect(g, d, lanes), args.steps, 2)
        batches[str(nb)] = {"ms_per_step": ms, "frames_per_s": nb / (ms / 1e3)}
    det.set_active(B)

    # single-frame latency (batch of one, synchronous per frame)
    lat = []
    det1 = ld.Detector(W, H, 1, ld.LD_DISP_F32, 128) if args.latency_frames > 0 else None
    lanes1 = det1.lanes_buffer() if det1 else None
    for i in range(min(args.latency_frames, B)):
        gi, di = g[i:i + 1], d[i:i + 1]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        det1.detect(gi, di, lanes1)
        det1.sync()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat[5:] if len(lat) > 10 else lat) if lat else np.array([np.nan])
    if det1:
        det1.close()

    alg_bytes = W * H * (1 + 4)
    path_achieved = alg_bytes * fps / 1e9
    out = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32+f64", "data": "synthetic",
        "config": {"workload": "1242x375 frames, f32 subpixel disparity 0..128, 4 curved lanes, ~10% obstacle pixels, "
                               "16 sequences x 64 frames", "frames_per_step": B, "width": W, "height": H, "d_max": 128,
                   "variant": "plain"},
        "roofline": roof,
        "hbm_frac": path_achieved / HBM_PEAK_GBS,
        "roofline_path": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": path_achieved,
                          "frac": path_achieved / HBM_PEAK_GBS,
                          "per_unit": f"{alg_bytes} B per frame (grey once + f32 disparity once)"},
        "kernels": per_kernel_roof,
        "batch_sizes": batches,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "batch": 1},
        "road_rows_mean": R_mean,
        "lanes_per_frame": float(lanes_np["n"].mean()),
        "learned_pruned": None,
    }
    det.close()
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    net = None
    if args.train_steps > 0:
        out["learned_pruned"], net = learned_leg(args, det, g, d, lanes, lanes_np, tgreys, tdisps, ms_per_step)
    det.close()
    del g, d
    torch.cuda.empty_cache()
    if args.c3_frames > 0:
        out["c3_stream"] = c3_leg(args)
        torch.cuda.empty_cache()
    if serve_pool is not None:
        out["serving"] = serving_leg(args, serve_pool, net)
    if net is not None:
        net.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(greys, disps, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
