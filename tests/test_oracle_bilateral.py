"""Pins of the oracle's bilateral pre-filter (Sec. 2.3.1, Eq. bilateral_filter and its two
weights) against values fixed by the mathematics: a constant image, the special cases that
reduce to a box or Gaussian mean (computed by scipy's correlation), the range weight recovered
in closed form from a two-level window, the edge-preserving closed form at a step, mirror
symmetry and the convex-combination bound."""
import numpy as np
import pytest
from scipy import ndimage

import oracle

BIG = 1.0e6          # sigma so large that the weight rounds to 1.0f for every offset / difference


def _masked_mean(img, kernel):
    """Weighted mean over the in-frame part of the window (frame pixels only), in FP64."""
    num = ndimage.correlate(img.astype(np.float64), kernel, mode="constant", cval=0.0)
    den = ndimage.correlate(np.ones_like(img, dtype=np.float64), kernel, mode="constant", cval=0.0)
    return num / den


def _round_agrees(out, ref, tie=1e-3):
    """The u8 output equals the rounded reference wherever the reference is not within `tie`
    of a rounding boundary."""
    frac = ref - np.floor(ref)
    clear = np.abs(frac - 0.5) > tie
    return np.array_equal(out[clear], np.floor(ref[clear] + 0.5).astype(np.uint8)) and clear.mean() > 0.95


@pytest.mark.parametrize("c", [0, 1, 90, 254, 255])
def test_constant_image_is_unchanged(c):
    g = np.full((23, 31), c, np.uint8)
    out, val = oracle.bilateral(g)
    assert np.array_equal(out, g)
    assert np.max(np.abs(val - c)) <= 1e-4 * max(c, 1)


@pytest.mark.parametrize("rho", [1, 3, 5])
def test_large_sigmas_give_the_box_mean(rho):
    g = np.random.default_rng(rho).integers(0, 256, (19, 27)).astype(np.uint8)
    out, val = oracle.bilateral(g, rho=rho, sigma_s=BIG, sigma_r=BIG)
    ref = _masked_mean(g, np.ones((2 * rho + 1, 2 * rho + 1)))
    assert np.max(np.abs(val - ref)) <= 2e-5 * 255
    assert _round_agrees(out, ref)


@pytest.mark.parametrize("sigma_s", [1.5, 3.0, 300.0])
def test_large_range_sigma_gives_the_gaussian_mean(sigma_s):
    g = np.random.default_rng(7).integers(0, 256, (21, 25)).astype(np.uint8)
    out, val = oracle.bilateral(g, rho=5, sigma_s=sigma_s, sigma_r=BIG)
    s = np.float64(np.float32(sigma_s))
    dy, dx = np.mgrid[-5:6, -5:6]
    ref = _masked_mean(g, np.exp(-(dx * dx + dy * dy) / (s * s)))
    assert np.max(np.abs(val - ref)) <= 2e-5 * 255
    assert _round_agrees(out, ref)


@pytest.mark.parametrize("d", [20, 40, 60, 100, 155])
def test_range_weight_recovered_from_a_two_level_window(d):
    """Centre c, every other window pixel c + d, spatial weights 1: the quotient is
    (c + 120 w (c + d)) / (1 + 120 w), which fixes w = exp(-(d/255)^2 / sigma_r^2)."""
    c = 60
    g = np.full((11, 11), c + d, np.uint8)
    g[5, 5] = c
    _, val = oracle.bilateral(g, rho=5, sigma_s=BIG, sigma_r=0.3)
    q = np.float64(val[5, 5])
    wof = lambda x: (x - c) / (120.0 * (c + d - x))
    # the single-precision quotient is good to a few units in its last place: the recovered
    # weight is held to the spread that error allows
    eps = 32 * np.spacing(np.float32(c + d))
    tol = abs(wof(q + eps) - wof(q - eps)) + 1e-7
    sr = np.float64(np.float32(0.3))
    assert abs(wof(q) - np.exp(-((d / 255.0) ** 2) / (sr * sr))) <= tol, (wof(q), tol)
    assert tol < 0.05 * (1.0 - np.exp(-((d / 255.0) ** 2) / (sr * sr)))       # the pin is informative


def test_step_edge_closed_form():
    """Left half 50, right half 200, spatial weights 1: a pixel with n_s same-side and n_o
    other-side window pixels gets (n_s a + n_o w b) / (n_s + n_o w), w = w_r(150)."""
    H, W, rho = 15, 24, 5
    g = np.full((H, W), 50, np.uint8)
    g[:, W // 2:] = 200
    out, val = oracle.bilateral(g, rho=rho, sigma_s=BIG, sigma_r=0.3)
    sr = np.float64(np.float32(0.3))
    w = np.exp(-((150 / 255.0) ** 2) / (sr * sr))
    for v in (0, 3, 7, 14):
        rows = min(v + rho, H - 1) - max(v - rho, 0) + 1
        for u in range(W):
            lo_u, hi_u = max(u - rho, 0), min(u + rho, W - 1)
            left = max(0, min(hi_u, W // 2 - 1) - lo_u + 1) * rows
            right = max(0, hi_u - max(lo_u, W // 2) + 1) * rows
            a, b = (50, 200) if u < W // 2 else (200, 50)
            ns, no = (left, right) if u < W // 2 else (right, left)
            ref = (ns * a + no * w * b) / (ns + no * w)
            assert abs(val[v, u] - ref) <= 2e-5 * 255, (v, u, val[v, u], ref)
    # far from the step the image is unchanged; next to it the two sides stay apart
    assert np.all(out[:, :W // 2 - rho] == 50) and np.all(out[:, W // 2 + rho:] == 200)
    assert np.all(out[:, W // 2 - 1] < 125) and np.all(out[:, W // 2] > 125)


def test_mirror_symmetry_and_convex_bound():
    g = np.random.default_rng(3).integers(0, 256, (17, 29)).astype(np.uint8)
    g[:, 10:13] = 220
    out, val = oracle.bilateral(g)
    out_m, val_m = oracle.bilateral(np.ascontiguousarray(g[:, ::-1]))
    assert np.max(np.abs(val_m[:, ::-1] - val)) <= 2e-5 * 255
    frac = val - np.floor(val)
    clear = np.abs(frac - 0.5) > 1e-3
    assert np.array_equal(out_m[:, ::-1][clear], out[clear])
    lo = ndimage.minimum_filter(g, size=11, mode="nearest")
    hi = ndimage.maximum_filter(g, size=11, mode="nearest")
    assert np.all(val >= lo - 1e-3) and np.all(val <= hi + 1e-3)


def test_rows_from_row0_only():
    g = np.random.default_rng(4).integers(0, 256, (30, 20)).astype(np.uint8)
    full, fval = oracle.bilateral(g)
    part, pval = oracle.bilateral(g, row0=12)
    assert np.all(part[:12] == 0) and np.array_equal(part[12:], full[12:])
    assert np.array_equal(pval[12:], fval[12:])


def test_invalid_arguments():
    g = np.zeros((8, 8), np.uint8)
    for kw in (dict(rho=0), dict(rho=6), dict(sigma_s=0.0), dict(sigma_r=-1.0)):
        with pytest.raises(ValueError):
            oracle.bilateral(g, **kw)
