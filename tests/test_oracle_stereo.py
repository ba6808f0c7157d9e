"""Pins of the oracle's stereo disparity (Sec. 2.1): the memorised block statistics against a
library correlation, the factorised cost (Eq. ncc_1) against the mean-subtracted definition
(Eq. ncc), exact recovery of a shifted texture (cost 1), the propagated search against an
exhaustive search on slowly varying disparity fields, and the consistency check against the
geometry of an occluding block."""
import numpy as np
import pytest
from scipy import signal

import oracle


def _texture(rng, H, W):
    return rng.integers(0, 256, (H, W)).astype(np.uint8)


def _ncc_definition(L, R, u, v, x, rho):
    """Eq. ncc with the means and standard deviations of Eq. sigma_l / sigma_r, in FP64."""
    a = L[v - rho:v + rho + 1, u - rho:u + rho + 1].astype(np.float64)
    b = R[v - rho:v + rho + 1, x - rho:x + rho + 1].astype(np.float64)
    n = a.size
    ma, mb = a.mean(), b.mean()
    sa, sb = np.sqrt(((a - ma) ** 2).sum() / n), np.sqrt(((b - mb) ** 2).sum() / n)
    return ((a - ma) * (b - mb)).sum() / (n * sa * sb)


@pytest.mark.parametrize("rho", [1, 3, 5])
def test_block_statistics_against_convolution(rho):
    img = _texture(np.random.default_rng(rho), 30, 41)
    S, Q = oracle.stereo_stats(img, rho)
    k = np.ones((2 * rho + 1, 2 * rho + 1), np.int64)
    Sv = signal.convolve2d(img.astype(np.int64), k, mode="valid")
    Qv = signal.convolve2d(img.astype(np.int64) ** 2, k, mode="valid")
    assert np.array_equal(S[rho:-rho, rho:-rho], Sv) and np.array_equal(Q[rho:-rho, rho:-rho], Qv)
    assert not S[:rho].any() and not S[:, :rho].any()


def test_shifted_texture_is_recovered_with_cost_one():
    rng = np.random.default_rng(1)
    L = _texture(rng, 40, 70)
    d0 = 9
    R = _texture(rng, 40, 70)
    R[:, :-d0] = L[:, d0:]                  # R(x) = L(x + d0): disparity d0 everywhere
    out, lf, rt, cost = oracle.stereo(L, R, d_max=24)
    rho = 3
    m = np.zeros_like(lf, bool)
    m[rho:-rho, rho + d0:-rho] = True          # left blocks whose match lies in the image
    assert np.all(lf[m] == d0) and np.all(out[m] == d0)
    assert np.max(np.abs(cost[m] - 1.0)) < 1e-12
    # the right map: right block at x matches the left block at x + d0 where that is inside
    mr = np.zeros_like(rt, bool)
    mr[rho:-rho, rho:-rho - d0] = True
    assert np.all(rt[mr] == d0)
    assert not out[:rho].any() and not out[:, :rho].any()


@pytest.mark.parametrize("rho", [1, 3, 5])
def test_factorised_cost_equals_the_definition(rho):
    rng = np.random.default_rng(2 + rho)
    L = _texture(rng, 24, 50)
    R = np.clip(np.roll(L, -5, axis=1).astype(int) + rng.integers(-30, 31, L.shape), 0, 255).astype(np.uint8)
    out, lf, rt, cost = oracle.stereo(L, R, d_max=12, rho=rho)
    for v in range(rho, 24 - rho):
        for u in range(rho + 1, 50 - rho):
            d = int(lf[v, u])
            if d:
                assert abs(cost[v, u] - _ncc_definition(L, R, u, v, u - d, rho)) < 1e-12


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_propagated_search_equals_exhaustive_search_on_smooth_fields(seed):
    """A disparity that grows by one every few rows (a road seen from above the horizon down)
    stays inside every propagated range, so wherever the exhaustive search over 1..d_max finds
    a clear match (cost > 0.6, no near tie) the propagated search must pick the same
    disparity."""
    rng = np.random.default_rng(seed)
    H, W, rho, d_max = 30, 64, 3, 16
    step = 8 + seed % 3
    D = 3 + np.arange(H) // step
    L = _texture(rng, H, W)
    R = _texture(rng, H, W)
    for v in range(H):
        R[v, :W - D[v]] = L[v, D[v]:]
    out, lf, rt, cost = oracle.stereo(L, R, d_max=d_max)
    checked = 0
    for v in range(rho, H - rho):
        for u in range(rho + D[v] + 1, W - rho):
            cs = [(_ncc_definition(L, R, u, v, u - d, rho), d) for d in range(1, d_max + 1) if u - d >= rho]
            cs.sort(key=lambda t: (-t[0], t[1]))
            if cs[0][0] < 0.6 or (len(cs) > 1 and cs[0][0] - cs[1][0] < 1e-9):
                continue
            assert lf[v, u] == cs[0][1], (v, u, lf[v, u], cs[:2])
            checked += 1
    assert checked > 0.5 * (H - 2 * rho) * (W - 2 * rho - D.max())


def test_occluding_block_is_removed_by_the_check():
    """A background at disparity 4 and a block in front of it at 20: the background pixels the
    block hides in the right view (left-view columns u0 - 16 .. u0 - 1; away from the depth
    edges by more than a block) must come out 0, the visible background 4 and the block 20."""
    rng = np.random.default_rng(6)
    H, W, rho = 40, 120, 3
    bg, fg = 4, 20
    texb = _texture(rng, H, W + 40)
    texf = _texture(rng, H, 40)
    u0, u1 = 60, 85                           # the block's columns in the left view
    L = texb[:, :W].copy()
    L[:, u0:u1 + 1] = texf[:, :u1 - u0 + 1]
    R = np.zeros_like(L)
    for x in range(W):
        R[:, x] = texb[:, x + bg] if x + bg < W + 40 else 0
    R[:, u0 - fg:u1 - fg + 1] = texf[:, :u1 - u0 + 1]
    out, lf, rt, _ = oracle.stereo(L, R, d_max=24)
    m = slice(rho, H - rho)
    hidden = list(range(u0 - fg + bg + rho + 1, u0 - rho - 1))
    assert hidden and np.all(out[m, hidden] == 0)
    visible = list(range(rho + bg + 2, u0 - fg + bg - rho - 2))
    assert np.all(out[m, visible] == bg)
    inside = list(range(u0 + rho + 1, u1 - rho))
    assert np.all(out[m, inside] == fg)


def test_flat_image_and_arguments():
    flat = np.full((20, 30), 77, np.uint8)
    out, lf, rt, _ = oracle.stereo(flat, flat)
    assert not out.any() and not lf.any() and not rt.any()
    with pytest.raises(ValueError):
        oracle.stereo(flat, flat, rho=0)
    with pytest.raises(ValueError):
        oracle.stereo(flat, flat, d_max=300)
