"""GPU parity of the stereo disparity (ld_stereo, Sec. 2.1) against the oracle: the left map,
the right map and the checked map equal byte for byte (the costs are exact integers and one
FP64 quotient in the same order on both sides), on synthetic road pairs, ragged shifted
textures, several block sizes and propagation bounds, flat and tiny images, and the
1024-frame launch; then lanes from the estimated disparity against the oracle's path on the
oracle's disparity."""
import numpy as np
import pytest

import oracle
from paper_1807_02752_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ld():
    from paper_1807_02752_amd import ld
    return ld


def _stereo_gpu(L, R, d_max, rho=3, tau=1, tr=3, pad=0):
    ld = _ld()
    B, H, W = L.shape
    det = ld.Detector(W, H, B, ld.LD_DISP_U8, d_max)
    lb = torch.zeros((B, H, W + pad), dtype=torch.uint8, device="cuda")
    rb = torch.zeros((B, H, W + pad), dtype=torch.uint8, device="cuda")
    lb[:, :, :W] = torch.from_numpy(L).cuda()
    rb[:, :, :W] = torch.from_numpy(R).cuda()
    out = torch.full((B, H, W + pad), 99, dtype=torch.uint8, device="cuda")
    lf = torch.full((B, H, W), 99, dtype=torch.uint8, device="cuda")
    rt = torch.full((B, H, W), 99, dtype=torch.uint8, device="cuda")
    det.stereo(lb[:, :, :W], rb[:, :, :W], out[:, :, :W], lf, rt, rho=rho, tau=tau, tr_lrc=tr)
    det.sync()
    det.close()
    o = out.cpu().numpy()
    if pad:
        assert np.all(o[:, :, W:] == 99)
    return o[:, :, :W], lf.cpu().numpy(), rt.cpu().numpy()


def _check(L, R, d_max, got, **kw):
    for b in range(L.shape[0]):
        want = oracle.stereo(L[b], R[b], d_max=d_max, **kw)
        for name, g, w in zip(("checked", "left", "right"), got, want[:3]):
            assert np.array_equal(g[b], w), (b, name, np.argwhere(g[b] != w)[:5])


def test_road_pairs_small_and_kitti_size():
    for cfg, d_max, n in (("c1", 48, 3), ("c2", 128, 2)):
        pairs = [synth.make_stereo(cfg, 4, i) for i in range(n)]
        L = np.stack([p[0] for p in pairs])
        R = np.stack([p[1] for p in pairs])
        got = _stereo_gpu(L, R, d_max)
        _check(L, R, d_max, got)


@pytest.mark.parametrize("H,W,rho,tau,pad", [(37, 70, 3, 1, 0), (29, 53, 1, 0, 3), (40, 91, 5, 2, 7), (11, 64, 3, 1, 0)])
def test_shifted_textures_ragged_and_parameters(H, W, rho, tau, pad):
    rng = np.random.default_rng(H * W + rho)
    L = rng.integers(0, 256, (2, H, W)).astype(np.uint8)
    R = rng.integers(0, 256, (2, H, W)).astype(np.uint8)
    for b in range(2):
        for v in range(H):
            d = 3 + (v * (b + 1)) // 9
            R[b, v, :W - d] = np.clip(L[b, v, d:].astype(int) + rng.integers(-6, 7, W - d), 0, 255)
    got = _stereo_gpu(L, R, 24, rho=rho, tau=tau, pad=pad)
    _check(L, R, 24, got, rho=rho, tau=tau)


@pytest.mark.parametrize("W,d_max", [(200, 150), (640, 150), (90, 40)])
def test_pixels_without_matched_neighbours_in_later_rows(W, d_max):
    """A flat band (blocks of zero variance are not matched) leaves the row above it with no
    matched neighbour below: those pixels search all of 1..d_max again, a wave per pixel when
    few (several candidates a lane for d_max above 64) and a lane per pixel when many."""
    rng = np.random.default_rng(W + d_max)
    H = 60
    L = rng.integers(0, 256, (2, H, W)).astype(np.uint8)
    R = rng.integers(0, 256, (2, H, W)).astype(np.uint8)
    for b in range(2):
        for v in range(H):
            d = 5 + (v * (b + 2)) // 11
            R[b, v, :W - d] = np.clip(L[b, v, d:].astype(int) + rng.integers(-4, 5, W - d), 0, 255)
        L[b, 20:31] = 100
        R[b, 20:31] = 100
    got = _stereo_gpu(L, R, d_max)
    _check(L, R, d_max, got)
    assert not got[1][:, 24:27].any()          # the flat rows are not matched
    assert got[1][:, 16, 3:-3].any()           # the rows above them are matched again


def test_flat_tiny_and_invalid():
    ld = _ld()
    flat = np.full((1, 20, 30), 77, np.uint8)
    got = _stereo_gpu(flat, flat, 16)
    assert not any(g.any() for g in got)
    tiny = np.random.default_rng(0).integers(0, 256, (1, 8, 10)).astype(np.uint8)   # no 11x11 block fits
    got = _stereo_gpu(tiny, tiny, 4, rho=5)
    assert not any(g.any() for g in got)
    det = ld.Detector(64, 40, 1, ld.LD_DISP_U8, 32)
    a = torch.zeros((1, 40, 64), dtype=torch.uint8, device="cuda")
    P, s = ld._ptr, ld._stream()
    for rho, tau, tr in [(0, 1, 3), (6, 1, 3), (3, -1, 3), (3, 1, -1)]:
        assert ld.ld_stereo(det.handle, P(a), 64, P(a), 64, rho, tau, tr, P(a), 64, P(a), P(a), s) == ld.LD_E_INVAL
    assert ld.ld_stereo(det.handle, P(a), 63, P(a), 64, 3, 1, 3, P(a), 64, P(a), P(a), s) == ld.LD_E_INVAL
    assert ld.ld_stereo(det.handle, P(a), 64, P(a), 64, 3, 1, 3, P(a), 64, None, P(a), s) == ld.LD_E_INVAL
    det.close()


def _gen(i):
    return synth.make_stereo("c2", 20 + i // 16, i % 16)[:2]


def test_benchmark_launch_sampled_frames():
    """1024 pairs of 1242x375 in one launch (64 generated, tiled): six positions, every byte."""
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=8) as ex:
        parts = list(ex.map(_gen, range(64)))
    L = np.stack([p[0] for p in parts] * 16)
    R = np.stack([p[1] for p in parts] * 16)
    got = _stereo_gpu(L, R, 128)
    for b in (0, 63, 64, 511, 700, 1023):
        want = oracle.stereo(L[b], R[b], d_max=128)
        for g, w in zip(got, want[:3]):
            assert np.array_equal(g[b], w), b


def test_lanes_from_estimated_disparity():
    """ld_stereo then ld_detect on its checked map (u8 disparity): every step as the oracle's
    path on the oracle's disparity."""
    import test_gpu_parity as par
    pairs = [synth.make_stereo("c2", 9, i) for i in range(2)]
    L = np.stack([p[0] for p in pairs])
    R = np.stack([p[1] for p in pairs])
    out, _, _ = _stereo_gpu(L, R, 128)
    res = par.run_gpu(L, out, 128)
    for b in range(2):
        want = oracle.stereo(L[b], R[b], d_max=128)[0]
        assert np.array_equal(out[b], want)
        r = par.compare_frame(res, b, L[b], want, 128)
        assert r.n_lanes >= 2
