"""Throughput benchmark of the lane-detection hot path on one MI355X.

One step = ld_detect over a batch of synthetic 1242x375 frames already resident in HBM
(grey u8 + f32 subpixel disparity, 4 curved lanes, ~10% obstacle pixels, 16 sequences of
64 frames).  Prints one JSON line: frames/s, ms per step, the roofline of the dominant
kernel (HIP events on the launch stream), single-frame latency p50/p99, and the CPU oracle
timed on the host's cores on a bounded sample of the same frames.
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
    for _ in range(args.warmup):
        det.detect_pruned(net, g, d, lp)
    torch.cuda.synchronize()
    det.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        det.detect_pruned(net, g, d, lp)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
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


def cpu_baseline(greys, disps, seconds: float, threads: int):
    """The oracle, as it stands, on the host cores: frames split over `threads` threads
    (ctypes releases the GIL during each call)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()
    t0 = time.perf_counter()
    oracle.detect(greys[0], disps[0], 128)
    per_frame = time.perf_counter() - t0
    n = int(max(threads, min(len(greys), seconds / max(per_frame, 1e-3))))
    idx = list(range(n))

    def work(i):
        oracle.detect(greys[i], disps[i], 128, frame_idx=i)
        return i

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, idx))
    wall = time.perf_counter() - t0
    return {"value": n / wall, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} frames of the 1242x375 workload, {threads} threads, {wall:.1f} s wall",
            "single_thread_ms_per_frame": per_frame * 1e3}


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
    for _ in range(args.warmup):
        det.detect(g, d, lanes)
    torch.cuda.synchronize()
    log("warmup done")

    det.profile(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        det.detect(g, d, lanes)
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ktimes = det.kernel_times()
    det.profile(False)
    ms_per_step = total_ms / args.steps
    fps = B * args.steps / (total_ms / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {fps:.0f} frames/s")

    # per-kernel averages and the dominant kernel's roofline
    lanes_np = ld.Detector.parse_lanes(lanes)
    infos = np.stack([det.read(ld.LD_STATE_INFO, b) for b in range(min(B, 64))])
    R_mean = float(infos[:, 6].mean())
    kern = {k: {"ms_per_launch": v[0] / max(v[1], 1), "launches": int(v[1])} for k, v in ktimes.items()}
    dom = max(kern, key=lambda k: kern[k]["ms_per_launch"])
    t_dom = kern[dom]["ms_per_launch"] / 1e3
    p = det.params
    if dom == "k_vdisp_hist":
        per_unit, units = W * H * 4, B
        roof = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "achieved": per_unit * units / t_dom / 1e9, "per_unit": f"{per_unit} B per frame (disparity read)"}
    elif dom == "k_edges":
        per_unit = (R_mean + 2) * W * 1 + R_mean * W * 4
        roof = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "achieved": per_unit * B / t_dom / 1e9, "per_unit": f"{per_unit:.0f} B per frame (road rows of grey + disparity)"}
    elif dom == "k_vpx_fit":
        ops = R_mean * 2 * W * (2 * p.tau_x_max + 1) * 2
        roof = {"bound": "alu", "unit": "TOP/s", "peak": ALU_PEAK_TOPS, "achieved": ops * B / t_dom / 1e12,
                "per_unit": f"{ops:.3g} ops per frame (row DP: R x 2W x 11 taps x add+min)"}
    elif dom == "k_energy":
        ops = R_mean * (W * 16 + 2 * W * 6)
        roof = {"bound": "alu", "unit": "TOP/s", "peak": ALU_PEAK_TOPS, "achieved": ops * B / t_dom / 1e12,
                "per_unit": f"{ops:.3g} ops per frame (M_0/M_1 rows + 2W track gathers per road row)"}
    else:   # k_vdisp_fit / k_peaks
        ops = (128 + 1) * H * (p.tau_y_max + 1) * 2
        roof = {"bound": "alu", "unit": "TOP/s", "peak": ALU_PEAK_TOPS, "achieved": ops * B / t_dom / 1e12,
                "per_unit": f"{ops:.3g} ops per frame (v-disparity DP: D x H x 7 taps x add+min)"}
    roof["kernel"] = dom
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom)
    roof["launch_ms"] = kern[dom]["ms_per_launch"]

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
    out = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32+f64", "data": "synthetic",
        "config": {"workload": "1242x375 frames, f32 subpixel disparity 0..128, 4 curved lanes, ~10% obstacle pixels, "
                               "16 sequences x 64 frames", "frames_per_step": B, "width": W, "height": H, "d_max": 128,
                   "variant": "plain"},
        "roofline": roof,
        "hbm_frac": alg_bytes * fps / (HBM_PEAK_GBS * 1e9),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "batch": 1},
        "kernels_ms_per_launch": {k: round(v["ms_per_launch"], 4) for k, v in kern.items()},
        "road_rows_mean": R_mean,
        "lanes_per_frame": float(lanes_np["n"].mean()),
        "learned_pruned": None,
    }
    net = None
    if args.train_steps > 0:
        out["learned_pruned"], net = learned_leg(args, det, g, d, lanes, lanes_np, tgreys, tdisps, ms_per_step)
    if serve_pool is not None:
        out["serving"] = serving_leg(args, serve_pool, net)
    if net is not None:
        net.close()
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(greys, disps, args.cpu_seconds, threads)
    det.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
