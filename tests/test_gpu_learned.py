"""GPU parity of the learned part: the network's forward pass, loss, gradient and Adam step
against the FP64 oracle of oracle/cnn.py (BF16 rounding emulated at the same points), the
training labels, and the narrowed search (ld_detect_pruned) against oracle.detect_pruned fed
with the decisions the GPU network took.

Tolerances.  Forward: the GPU accumulates BF16 x BF16 products in FP32 where the oracle sums
exactly-rounded FP64; an intermediate BF16 rounding can fall on the other side of a tie, so
single probabilities may move by up to a few 1e-3; |dP| <= 2e-2 everywhere and <= 2e-3 for
99.9 % of the pixels.  Gradients: |dg| <= 5e-3 max|g| per parameter tensor.  Adam (FP32):
|dw| <= 1e-6 + 1e-5 |w|.  Decisions of the narrowed search downstream of the network are
bit-exact given the network's decisions.
"""
import numpy as np
import pytest

import oracle
from oracle import cnn
from paper_1807_02752_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from test_gpu_parity import ETOL, _fit_equal, _lanes_match  # noqa: E402


def _ld():
    from paper_1807_02752_amd import ld
    return ld


def random_params(seed):
    p = cnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2"):
        p[k] = rng.normal(0, 0.05, size=p[k].shape)
    p["b3"] = np.array([0.3])
    return cnn.flat(p).astype(np.float32)


def bright_params(noise=0.0, seed=0):
    """A hand-set network that marks bright pixels: z = 20 ReLU(I/255 - 0.6) - 1 (centre taps)."""
    p = {k: np.zeros(s) for k, s in cnn.ORDER}
    p["w1"][1, 1, 0, 0] = 1.0
    p["b1"][0] = -0.6
    p["w2"][1, 1, 0, 0] = 1.0
    p["w3"][1, 1, 0, 0] = 20.0
    p["b3"][0] = -1.0
    v = cnn.flat(p)
    if noise:
        v = v + np.random.default_rng(seed).normal(0, noise, v.size)
    return v.astype(np.float32)


def frames_c2(n, seed=0, start=0):
    g, d, _ = synth.make_batch("c2", seed, n, start)
    return g, d


def _oracle_bands(grey, disp, d_max, n_bands, frame_idx):
    r = oracle.detect(grey, disp, d_max, frame_idx=frame_idx)
    H = grey.shape[0]
    tops = [cnn.band_top(r.v_h, H, n_bands, k) if not (r.flags & 1) else -1 for k in range(n_bands)]
    return r, tops


def test_forward_matches_oracle():
    ld = _ld()
    greys, disps = frames_c2(2, seed=3)
    B, H, W = greys.shape
    nb = 2
    params = random_params(5)
    net = ld.Cnn(params, n_bands=nb)
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    prob = torch.full((B, nb, 16, W), -1.0, dtype=torch.float32, device="cuda")
    det.vdisp(d)
    net.forward(det, g, d, prob)
    det.sync()
    P = prob.cpu().numpy()
    pd = cnn.unflat(params.astype(np.float64))
    errs = []
    for b in range(B):
        r, tops = _oracle_bands(greys[b], disps[b], 128, nb, b)
        bits = det.read(ld.LD_STATE_LANE_BITS, b).reshape(4, 16, W)
        for k, top in enumerate(tops):
            assert top >= 0
            x = cnn.band_features(greys[b], disps[b], r.f, top)
            z3 = cnn.forward(x, pd)[-1][..., 0]
            want = cnn.sigmoid(z3)
            e = np.abs(P[b, k] - want)
            errs.append(e.ravel())
            assert e.max() <= 2e-2, (b, k, e.max())
            # decisions: z >= logit(0.5) = 0 except within a margin of the threshold
            clear = np.abs(z3) > 0.05
            assert np.array_equal(bits[k][clear], (z3[clear] >= 0).astype(np.uint8))
    errs = np.concatenate(errs)
    assert np.quantile(errs, 0.999) <= 2e-3, np.quantile(errs, 0.999)
    det.close()
    net.close()


def _labels_for(rng, B, nb, W):
    lab = (rng.random((B, nb, 16, W)) < 0.2).astype(np.uint8)
    lab[rng.random((B, nb, 16, W)) < 0.1] = 255
    return lab


def _oracle_grad(greys, disps, params, labels, nb, pos_weight, inv_norm):
    pd = cnn.unflat(params.astype(np.float64))
    total = {k: np.zeros(s) for k, s in cnn.ORDER}
    loss = 0.0
    for b in range(greys.shape[0]):
        r, tops = _oracle_bands(greys[b], disps[b], 128, nb, b)
        for k, top in enumerate(tops):
            x = cnn.band_features(greys[b], disps[b], r.f, top)
            cache = cnn.forward(x, pd)
            y = labels[b, k].astype(np.float64)
            mask = (labels[b, k] != 255).astype(np.float64)
            y = np.where(mask > 0, y, 0.0)
            n = max(1.0, mask.sum())
            l, dz = cnn.loss_and_grad_logits(cache[-1], y, mask, pos_weight)
            loss += l * n * inv_norm
            gr = cnn.backward(x, pd, cache, dz * n * inv_norm)
            for kk in total:
                total[kk] += gr[kk]
    return loss, total


def test_gradient_and_adam_match_oracle():
    ld = _ld()
    greys, disps = frames_c2(2, seed=4)
    B, H, W = greys.shape
    nb = 2
    params = random_params(7)
    net = ld.Cnn(params, n_bands=nb, max_batch=B, max_width=W)
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    labels = _labels_for(np.random.default_rng(9), B, nb, W)
    lab = torch.from_numpy(labels).cuda()
    inv_norm = 1.0 / float((labels != 255).sum())
    pw = 4.0
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(ld.LD_CNN_PARAMS, dtype=torch.float32, device="cuda")
    det.vdisp(d)
    net.train_step(det, g, d, lab, pw, inv_norm, 0.0, loss, grad)
    det.sync()
    gg = grad.cpu().numpy().astype(np.float64)
    lref, gref = _oracle_grad(greys, disps, params, labels, nb, pw, inv_norm)
    assert abs(float(loss.item()) - lref) <= 1e-4 * abs(lref), (loss.item(), lref)
    gu = cnn.unflat(gg)
    for k in gref:
        scale = np.abs(gref[k]).max()
        assert scale > 0, k
        err = np.abs(gu[k] - gref[k]).max()
        assert err <= 5e-3 * scale, (k, err, scale)
    # unchanged weights at lr = 0, then two Adam steps against the oracle's update rule
    assert np.array_equal(net.get_params(), params)
    lr = 1e-3
    m = {k: np.zeros(s) for k, s in cnn.ORDER}
    v = {k: np.zeros(s) for k, s in cnn.ORDER}
    cur = cnn.unflat(params.astype(np.float64))
    for t in (1, 2):
        net.train_step(det, g, d, lab, pw, inv_norm, lr, None, grad)
        det.sync()
        gstep = cnn.unflat(grad.cpu().numpy().astype(np.float64))
        cur = cnn.adam_step(cur, m, v, gstep, t, lr=lr)
        got = cnn.unflat(net.get_params().astype(np.float64))
        for k in cur:
            assert np.all(np.abs(got[k] - cur[k]) <= 1e-6 + 1e-5 * np.abs(cur[k])), k
        cur = got     # continue from the FP32 masters
    det.close()
    net.close()


def test_training_step_is_deterministic():
    ld = _ld()
    greys, disps = frames_c2(2, seed=6)
    B, H, W = greys.shape
    params = random_params(3)
    labels = torch.from_numpy(_labels_for(np.random.default_rng(2), B, 2, W)).cuda()
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    outs = []
    for _ in range(2):
        net = ld.Cnn(params, n_bands=2, max_batch=B, max_width=W)
        det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
        det.vdisp(d)
        for _ in range(3):
            net.train_step(det, g, d, labels, 4.0, 1e-5, 1e-3)
        det.sync()
        outs.append(net.get_params())
        det.close()
        net.close()
    assert np.array_equal(outs[0], outs[1])


def test_checkpoint_resume_continues_training_exactly(tmp_path):
    """ld_cnn_save after three Adam steps, then a fourth step; a network restored by
    ld_cnn_load takes the same fourth step: the weights match bit for bit (and they would not
    if the moments or the step count were lost: the restored step differs from a fresh one)."""
    ld = _ld()
    greys, disps = frames_c2(2, seed=6)
    B, H, W = greys.shape
    params = random_params(5)
    labels = torch.from_numpy(_labels_for(np.random.default_rng(3), B, 2, W)).cuda()
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    det.vdisp(d)
    net = ld.Cnn(params, n_bands=2, max_batch=B, max_width=W, theta=0.4)
    for _ in range(3):
        net.train_step(det, g, d, labels, 4.0, 1e-5, 1e-3)
    path = str(tmp_path / "net.ckpt")
    net.save(path)
    saved = net.get_params()
    header, arrays = ld.read_checkpoint(path)
    assert header["step"] == 3 and header["params"] == ld.LD_CNN_PARAMS
    assert abs(header["config"]["theta"] - 0.4) < 1e-7 and header["config"]["n_bands"] == 2
    assert np.array_equal(arrays["master"], saved)
    assert np.abs(arrays["adam_v"]).max() > 0
    net.train_step(det, g, d, labels, 4.0, 1e-5, 1e-3)
    det.sync()
    cont = net.get_params()
    net.close()
    back = ld.Cnn.load(path)
    assert back.config.n_bands == 2 and abs(back.config.theta - 0.4) < 1e-7
    assert np.array_equal(back.get_params(), saved)
    back.train_step(det, g, d, labels, 4.0, 1e-5, 1e-3)
    det.sync()
    assert np.array_equal(back.get_params(), cont)
    back.close()
    fresh = ld.Cnn(saved, n_bands=2, max_batch=B, max_width=W)   # same weights, no moments, step 0
    fresh.train_step(det, g, d, labels, 4.0, 1e-5, 1e-3)
    det.sync()
    assert not np.array_equal(fresh.get_params(), cont)
    fresh.close()
    det.close()


def test_labels_from_plain_curves():
    ld = _ld()
    greys, disps = frames_c2(3, seed=1)
    B, H, W = greys.shape
    nb = 2
    net = ld.Cnn(None, n_bands=nb)
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    lanes = det.lanes_buffer()
    curves = torch.empty((B, 16, H), dtype=torch.float32, device="cuda")
    det.detect(g, d, lanes, curves_out=curves)
    lab = torch.empty((B, nb, 16, W), dtype=torch.uint8, device="cuda")
    net.labels(det, lanes, curves, lab, radius=2.0, radius_per_disp=0.139)
    det.sync()
    L = ld.Detector.parse_lanes(lanes)
    cv = curves.cpu().numpy()
    got = lab.cpu().numpy()
    u = np.arange(W, dtype=np.float32)
    for b in range(B):
        info = det.read(ld.LD_STATE_INFO, b)
        f = det.read(ld.LD_STATE_TABLES, b).reshape(6, H)[0]
        for k in range(nb):
            top = cnn.band_top(int(info[1]), H, nb, k)
            for r in range(16):
                v = top + r
                rad = np.float32(2.0) + np.float32(0.139) * np.float32(f[v])
                want = np.zeros(W, bool)
                for l in range(L["n"][b]):
                    c = cv[b, l, v]
                    want |= np.abs(u - np.float32(c)) <= rad
                assert np.array_equal(got[b, k, r], want.astype(np.uint8)), (b, k, r)
        assert got[b].max() == 1
    det.close()
    net.close()


def _run_pruned(greys, disps, d_max, params, nb=2, **cfg):
    ld = _ld()
    B, H, W = greys.shape
    fmt = {np.dtype(np.uint8): 0, np.dtype(np.float32): 1, np.dtype(np.uint16): 2}[disps.dtype]
    net = ld.Cnn(params, n_bands=nb, **cfg)
    det = ld.Detector(W, H, B, fmt, d_max)
    g, d = torch.from_numpy(greys).cuda(), torch.from_numpy(disps).cuda()
    lanes = det.lanes_buffer()
    curves = torch.empty((B, 16, H), dtype=torch.float32, device="cuda")
    det.detect_pruned(net, g, d, lanes, curves_out=curves)
    det.sync()
    out = {"lanes": ld.Detector.parse_lanes(lanes), "curves": curves.cpu().numpy(), "frames": []}
    for b in range(B):
        out["frames"].append({
            "info": det.read(ld.LD_STATE_INFO, b), "gamma": det.read(ld.LD_STATE_GAMMA, b)[0],
            "mx": det.read(ld.LD_STATE_MX_PATH, b), "energy": det.read(ld.LD_STATE_ENERGY, b),
            "bits": det.read(ld.LD_STATE_LANE_BITS, b), "prune": det.read(ld.LD_STATE_PRUNE, b),
            "mask": det.read(ld.LD_STATE_CAND_MASK, b), "trace": det.read(ld.LD_STATE_TRACE, b).reshape(2, 64, 3),
        })
    cfgv = net.config
    det.close()
    net.close()
    return out, cfgv


def _compare_pruned(out, cfgv, b, grey, disp, d_max, nb):
    fr = out["frames"][b]
    r = oracle.detect_pruned(grey, disp, d_max, fr["bits"], n_bands=nb, delta_x=cfgv.delta_x, dilate=cfgv.dilate,
                             min_votes=cfgv.min_votes, seed_ransac=cfgv.seed_ransac, frame_idx=b)
    assert np.array_equal(fr["prune"], r.prune), (b, fr["prune"].tolist(), r.prune.tolist())
    assert fr["info"][0] == r.flags, (b, fr["info"][0], r.flags)
    L = out["lanes"][b]
    assert L["flags"] == r.flags
    if r.flags & 1:
        return r
    assert np.array_equal(fr["mx"], r.mx_path)
    _fit_equal(fr["gamma"], r.gamma, 4)
    assert np.array_equal(fr["trace"][1, : r.gamma.rounds], r.trace_gamma)
    if r.flags & 2:
        return r
    assert np.array_equal(fr["mask"], r.cand_mask)
    eg, er = fr["energy"], r.energy
    scale = np.abs(er).max()
    assert np.all(np.abs(eg - er) <= ETOL * np.maximum(np.abs(er), scale) + 1e-12)
    assert _lanes_match(L["u_start"][: L["n"]], r, er, grey.shape[1])
    return r


@pytest.mark.parametrize("cfg", [{}, {"dilate": 3, "seed_ransac": 1, "delta_x": 48}])
def test_pruned_path_matches_oracle_on_c2(cfg):
    greys, disps = frames_c2(4, seed=2)
    out, cfgv = _run_pruned(greys, disps, 128, bright_params(), **cfg)
    kinds = set()
    for b in range(greys.shape[0]):
        r = _compare_pruned(out, cfgv, b, greys[b], disps[b], 128, 2)
        kinds.add(int(r.prune[1]))
    assert 0 in kinds            # the narrowed search itself ran to the end


def test_pruned_bench_launch_sampled_frames():
    # the benchmark's learned-pruned launch: 1024 frames of 1242x375 (f32 disparity) through
    # ld_detect_pruned in one call with one band; eight batch positions drawn with a fixed seed
    # against the oracle's narrowed search fed with the GPU network's decisions.  64 synthetic
    # frames (4 sequences x 16) are tiled to 1024, each position with its own frame index.
    ld = _ld()
    parts = [frames_c2(16, seed=s) for s in range(4)]
    G = np.concatenate([p[0] for p in parts] * 16)
    D = np.concatenate([p[1] for p in parts] * 16)
    B, H, W = G.shape
    assert (B, H, W) == (1024, 375, 1242)
    net = ld.Cnn(bright_params(), n_bands=1)
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    lanes = det.lanes_buffer()
    det.detect_pruned(net, torch.from_numpy(G).cuda(), torch.from_numpy(D).cuda(), lanes)
    det.sync()
    L = ld.Detector.parse_lanes(lanes)
    rng = np.random.default_rng(1807)
    picks = sorted(int(x) for x in rng.choice(B, 8, replace=False))
    frames = {}
    for b in picks:
        frames[b] = {
            "info": det.read(ld.LD_STATE_INFO, b), "gamma": det.read(ld.LD_STATE_GAMMA, b)[0],
            "mx": det.read(ld.LD_STATE_MX_PATH, b), "energy": det.read(ld.LD_STATE_ENERGY, b),
            "bits": det.read(ld.LD_STATE_LANE_BITS, b), "prune": det.read(ld.LD_STATE_PRUNE, b),
            "mask": det.read(ld.LD_STATE_CAND_MASK, b), "trace": det.read(ld.LD_STATE_TRACE, b).reshape(2, 64, 3),
        }
    cfgv = net.config
    det.close()
    net.close()
    kinds = set()
    for b in picks:
        print("pruned bench launch: frame", b, flush=True)
        r = _compare_pruned({"lanes": L, "frames": frames}, cfgv, b, G[b], D[b], 128, 1)
        kinds.add(int(r.prune[1]))
    assert 0 in kinds            # the narrowed search itself ran to the end on some of them


def test_pruned_path_fallbacks_match_oracle():
    # a network that marks nothing: no seed, full search everywhere
    greys, disps = frames_c2(2, seed=5)
    zero = np.zeros(3057, np.float32)
    zero[-1] = -5.0
    out, cfgv = _run_pruned(greys, disps, 128, zero)
    for b in range(2):
        r = _compare_pruned(out, cfgv, b, greys[b], disps[b], 128, 2)
        assert r.prune[1] & 1 and r.flags & 16
    # a noisy network on three bands, a narrow window and no dilation: mixed outcomes
    out, cfgv = _run_pruned(greys, disps, 128, bright_params(noise=0.05, seed=1), nb=3, delta_x=6, dilate=0,
                            seed_ransac=1)
    for b in range(2):
        _compare_pruned(out, cfgv, b, greys[b], disps[b], 128, 3)


def test_pruned_path_other_formats_and_degenerate():
    dm = 48
    g1, d1, _ = synth.make_c1(0)
    out, cfgv = _run_pruned(g1[None], d1[None], dm, bright_params())
    _compare_pruned(out, cfgv, 0, g1, d1, dm, 2)
    g3, d3 = synth.make_frame("c3", 0, 0)[:2]
    out, cfgv = _run_pruned(g3[None], d3[None], 255, bright_params())
    _compare_pruned(out, cfgv, 0, g3, d3, 255, 2)
    for kind in ("all_invalid", "flat_image", "obstacle_only", "random"):
        g, d = synth.degenerate(kind)
        out, cfgv = _run_pruned(g[None], d[None], 32, bright_params())
        _compare_pruned(out, cfgv, 0, g, d, 32, 2)


def _gen(args):
    seed, start, count = args
    g, d, _ = synth.make_batch("c2", seed, count, start)
    return g, d


def _pool_frames(seeds, per_seq):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=8) as ex:
        parts = list(ex.map(_gen, [(s, 0, per_seq) for s in seeds]))
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def lane_disagreement(lanes_a, lanes_b):
    """Lanes present in one result and not the other (by start column), over all lanes of a."""
    diff = tot = 0
    for a, b in zip(lanes_a, lanes_b):
        sa, sb = set(a["u_start"][: a["n"]].tolist()), set(b["u_start"][: b["n"]].tolist())
        diff += len(sa ^ sb)
        tot += len(sa)
    return diff / max(tot, 1)


def test_trained_network_gain():
    """Train from random weights on frames labelled by the plain method, then run the narrowed
    search on held-out sequences: it must agree with the plain search on >= 99.5 % of the
    lanes; the speed of both and the fallback rate are reported."""
    from paper_1807_02752_amd import train as tr
    ld = _ld()
    gtr, dtr = _pool_frames(range(100, 116), 16)      # 256 training frames
    gte, dte = _pool_frames(range(200, 208), 16)      # 128 held-out frames
    G, D = torch.from_numpy(gtr).cuda(), torch.from_numpy(dtr).cuda()
    net, losses = tr.train(G, D, 128, steps=300, batch=16, lr=3e-3, pos_weight=4.0, seed=0)
    print(f"loss first 10 {losses[:10].mean():.4f} last 10 {losses[-10:].mean():.4f}")
    assert losses[-10:].mean() < 0.5 * losses[:10].mean()
    B, H, W = gte.shape
    g, d = torch.from_numpy(gte).cuda(), torch.from_numpy(dte).cuda()
    det = ld.Detector(W, H, B, ld.LD_DISP_F32, 128)
    lp, ll = det.lanes_buffer(), det.lanes_buffer()
    times = {}
    for name, fn in (("plain", lambda: det.detect(g, d, lp)), ("pruned", lambda: det.detect_pruned(net, g, d, ll))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 5
    P = ld.Detector.parse_lanes(lp)
    L = ld.Detector.parse_lanes(ll)
    dis = lane_disagreement(P, L)
    fb = np.mean([(det.read(ld.LD_STATE_PRUNE, b)[1] & 3) != 0 for b in range(B)])
    kept = np.mean([det.read(ld.LD_STATE_PRUNE, b)[14] for b in range(B)])
    print(f"plain {times['plain']:.3f} ms, pruned {times['pruned']:.3f} ms per {B} frames; "
          f"disagreement {dis:.4f}; fallback {fb:.3f}; kept candidates {kept:.0f} of {2 * W}")
    # the same network with candidate pruning on (reported, not held to the bar)
    net_c = ld.Cnn(net.get_params(), n_bands=1, dilate=8)
    det.detect_pruned(net_c, g, d, ll)
    torch.cuda.synchronize()
    print(f"with candidate pruning (dilate 8): disagreement {lane_disagreement(P, ld.Detector.parse_lanes(ll)):.4f}")
    assert dis <= 0.005
    assert fb < 0.5
    det.close()
    net.close()
    net_c.close()
