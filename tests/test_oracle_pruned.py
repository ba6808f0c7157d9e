"""Pins of the oracle's narrowed search (the learned part's seed, window DP, candidate-mask
tracks, band features) against exhaustive enumeration, exact rational arithmetic, the
unrestricted search and the generator's ground truth.  CPU only.

The narrowed search is a definition of this library, not of the paper; each pin below
checks a property that follows from that definition and from the plain search it narrows
(the row DP of Eq. dense_vpx_estimation and the track of Eq. lane_visualisation).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import cnn
from paper_1807_02752_amd import synth

_RANK = lambda t: 0 if t == 0 else (2 * abs(t) - 1 if t < 0 else 2 * abs(t))   # noqa: E731


# ----------------------------------------------------------------------------- window DP
def _window_bruteforce(mx, v_h, lo, hi, tau_max, lam):
    """All paths whose columns stay in lo..hi, from row v_h down to the last row, with steps
    |tau| <= tau_max; the minimum of (energy, start column, tie ranks of the steps)."""
    H, _ = mx.shape
    rows = list(range(v_h, H))
    best = None
    for c0 in range(lo, hi + 1):
        for taus in itertools.product(range(-tau_max, tau_max + 1), repeat=len(rows) - 1):
            c, path, ok = c0, [c0], True
            for t in taus:
                c += t
                if not (lo <= c <= hi):
                    ok = False
                    break
                path.append(c)
            if not ok:
                continue
            e = sum(int(mx[v, path[i]]) for i, v in enumerate(rows)) + lam * sum(abs(t) for t in taus)
            key = (e, c0, tuple(_RANK(t) for t in taus))
            if best is None or key < best[0]:
                best = (key, path)
    return best[1]


@pytest.mark.parametrize("seed", range(12))
def test_window_dp_exhaustive(seed):
    """Tiny grids: the window DP's path equals the best path confined to the window, and the
    inner-edge flag is set exactly when that path visits an inner edge column."""
    rng = np.random.default_rng(300 + seed)
    H = int(rng.integers(3, 6))
    v_h = int(rng.integers(0, 2))
    W2 = int(rng.integers(5, 9))
    tau_max = int(rng.integers(1, 3))
    lam = int(rng.integers(0, 3))
    lo = int(rng.integers(0, W2 - 2))
    hi = int(rng.integers(lo + 1, W2))
    mx = -rng.integers(0, 4, size=(H, W2)).astype(np.int64)
    path, touch = oracle.window_dp(mx, v_h, lo, hi, tau_max=tau_max, lam=lam)
    want = _window_bruteforce(mx, v_h, lo, hi, tau_max, lam)
    assert path[v_h:].tolist() == want
    assert np.all(path[:v_h] == -1)
    inner = [c for c in want if (lo > 0 and c == lo) or (hi < W2 - 1 and c == hi)]
    assert touch == bool(inner)


@pytest.mark.parametrize("seed", range(6))
def test_window_dp_full_window_is_the_row_dp(seed):
    """A window of all 2W columns has no inner edge: the path is the unrestricted row DP's."""
    rng = np.random.default_rng(400 + seed)
    H, W2 = int(rng.integers(20, 60)), int(rng.integers(30, 120))
    v_h = int(rng.integers(0, H // 2))
    tau_max, lam = int(rng.integers(1, 6)), int(rng.integers(0, 4))
    mx = -rng.integers(0, 6, size=(H, W2)).astype(np.int64)
    path, touch = oracle.window_dp(mx, v_h, 0, W2 - 1, tau_max=tau_max, lam=lam)
    assert not touch
    assert np.array_equal(path, oracle.row_dp(mx, v_h, tau_max=tau_max, lam=lam))


@pytest.mark.parametrize("seed", range(6))
def test_window_dp_around_the_optimum(seed):
    """A window that holds the unrestricted optimum strictly inside returns it unchanged: the
    window's paths are a subset of all paths that contains the optimum, and the tie order is
    the same total order on both."""
    rng = np.random.default_rng(500 + seed)
    H, W2 = 48, 200
    v_h = 6
    # a planted ridge of votes near column 90 (a lane's vanishing-point path) over weak noise
    mx = -rng.integers(0, 3, size=(H, W2)).astype(np.int64)
    ridge = 90 + np.round(8 * np.sin(np.arange(H) / 7.0)).astype(int)
    for v in range(H):
        mx[v, ridge[v] - 1:ridge[v] + 2] -= 20
    full = oracle.row_dp(mx, v_h)
    p = full[v_h:]
    for pad in (1, 3, 17):
        lo, hi = max(0, int(p.min()) - pad), min(W2 - 1, int(p.max()) + pad)
        path, touch = oracle.window_dp(mx, v_h, lo, hi)
        assert not touch and np.array_equal(path, full), pad
    # a window that cuts the optimum off must report the inner edge or find another path
    lo = int(p.min()) + 2
    path, touch = oracle.window_dp(mx, v_h, lo, min(W2 - 1, lo + 40))
    assert touch or not np.array_equal(path, full)


# ----------------------------------------------------------------------------- seed
def test_seed_by_construction():
    """Marked edges of known vote columns: per-band argmax (smallest column on ties), pooled
    argmax, vote counts, and the min_votes cut."""
    W, H, v_h = 64, 80, 20
    nb = 2
    tops = [oracle.band_top(v_h, H, nb, k) for k in range(nb)]
    assert tops == [64, 42]
    bits = np.zeros((4, 16, W), np.uint8)
    eu, ev, eb = [], [], []

    def add(v, u, b, marked=True):
        eu.append(u); ev.append(v); eb.append(b)
        if marked:
            k = [k for k in range(nb) if tops[k] <= v < tops[k] + 16][0]
            bits[k, v - tops[k], u] = 1

    for r in range(5):
        add(64 + r, 10 + r, 70)          # band 0: 5 votes at column 70
    for r in range(5):
        add(70 + r, 30 + r, 40)          # band 0: 5 votes at column 40 (tie: 40 wins)
    add(75, 50, 90, marked=False)        # unmarked: no vote
    add(76, 51, -1)                      # no vote column
    for r in range(3):
        add(42 + r, 20 + r, 90)          # band 1: 3 votes at column 90
    add(60, 5, 90, marked=False)         # between the bands: no band row holds it
    cs, est, cnt, tot = oracle.seed(eu, ev, eb, bits, W, H, v_h, n_bands=nb, min_votes=8)
    assert (cs, tot) == (40, 13)
    assert est.tolist() == [40, 90, -1, -1] and cnt.tolist() == [10, 3, 0, 0]
    cs, *_ = oracle.seed(eu, ev, eb, bits, W, H, v_h, n_bands=nb, min_votes=14)
    assert cs == -1
    cs, est, cnt, tot = oracle.seed(eu, ev, eb, np.zeros_like(bits), W, H, v_h, n_bands=nb)
    assert cs == -1 and tot == 0 and est.tolist() == [-1] * 4


def _gt_lane_bits(sc, grey_shape, v_h, nb, extra=1.0):
    """Network decisions of an ideal marker: the pixels of the scene's lane markings."""
    H, W = grey_shape
    bits = np.zeros((4, 16, W), np.uint8)
    u = np.arange(W)
    for k in range(nb):
        top = oracle.band_top(v_h, H, nb, k)
        for r in range(16):
            v = top + r
            half_w = 0.5 * synth.marking_width(sc.f(v)) + extra
            for lk in range(len(sc.lanes)):
                bits[k, r] |= (np.abs(u - sc.lane_u(lk, v)) <= half_w).astype(np.uint8)
    return bits


def _vpx_gt(sc, v):
    """V_px of the generator's scene (all lanes share it): u_c - u_c' f / f'."""
    w = v - sc.v0
    uc = sc.c + sc.p * w + sc.q * w * w
    duc = sc.p + 2 * sc.q * w
    f = sc.a * w * w + sc.b * w
    df = 2 * sc.a * w + sc.b
    return uc - duc * f / df


@pytest.mark.parametrize("seq,idx", [(5, 0), (5, 42), (6, 63), (7, 63)])
def test_seed_of_ideal_marking_is_the_vanishing_point(seq, idx):
    """Edges marked by an ideal network (the scene's markings) vote for the scene's V_px.  A
    single row's votes scatter (the Sobel angle error of a marking edge is multiplied by
    (1 + slope^2)(v - V_py)), so the seed is a coarse estimate: it must lie within 56 columns
    (less than half of the default window, 127 columns each side) of V_px at the band's rows,
    which leaves the true path inside the window."""
    greys, disps, scenes = synth.make_batch("c2", seq, 1, idx)
    sc = scenes[0]
    g, d = greys[0], disps[0]
    r = oracle.detect(g, d, 128)
    H, W = g.shape
    bits = _gt_lane_bits(sc, g.shape, r.v_h, 1, extra=0.0)
    cs, est, cnt, tot = oracle.seed(r.edge_u, r.edge_v, r.edge_bin, bits, W, H, r.v_h, n_bands=1)
    assert tot >= 8 and cs >= 0
    top = oracle.band_top(r.v_h, H, 1, 0)
    gt = [_vpx_gt(sc, v) + W // 2 for v in range(top, top + 16)]
    assert min(gt) - 56 <= cs <= max(gt) + 56, (cs, min(gt), max(gt))


# ----------------------------------------------------------------------------- tracks
def _exact_AB(vpx, vpy, v_end, H):
    """A_v, B_v of the track recursion as exact rationals of the FP64 values the oracle
    forms (numpy's IEEE divisions give the same doubles)."""
    A, B = {}, {}
    for v in range(v_end, H - 1):
        den = np.float64(v + 1) - np.float64(vpy[v + 1])
        A[v] = Fraction(float(np.float64(vpx[v + 1]) / den))
        B[v] = Fraction(float((np.float64(v) - np.float64(vpy[v + 1])) / den))
    return A, B


def _frame_tables(seed=7, idx=3):
    g, d, _ = synth.make_batch("c2", seed, 1, idx)
    r = oracle.detect(g[0], d[0], 128)
    assert r.flags & 3 == 0
    return g[0], d[0], r


def test_track_affine_against_exact_recursion():
    """u_v = fma(a_v, u_start, b_v) against the exact rational recursion u_v = B_v u_{v+1} + A_v
    from the same FP64 A_v, B_v: within 1e-9 px on every row, and the same column
    floor(u_v + 0.5) wherever the exact value is not within 1e-9 of a half-integer.  The
    sequential FP64 track of the energy step obeys the same bound."""
    g, d, r = _frame_tables()
    H, W = g.shape
    a, b = oracle.track_affine(r.vpx, r.vpy, r.v_end, r.v_h)
    A, B = _exact_AB(r.vpx, r.vpy, r.v_end, H)
    starts = [-W // 2, -300, -1, 0, 1, 137, 620, W, W + W // 2 - 1]
    _, _, curves = oracle.energy(np.zeros((H, W)), r.vpx, r.vpy, r.v_h, tracks=np.array(starts))
    assert np.all(np.isnan(a[: r.v_end]))
    checked = near = 0
    for n, us in enumerate(starts):
        u = Fraction(us)
        for v in range(H - 1, r.v_end - 1, -1):
            if v < H - 1:
                u = B[v] * u + A[v]
            x = float(Fraction(float(a[v])) * us + Fraction(float(b[v])))   # fma: one rounding
            assert abs(Fraction(x) - u) <= Fraction(1, 10 ** 9), (us, v)
            assert abs(Fraction(float(curves[n, v])) - u) <= Fraction(1, 10 ** 9), (us, v)
            frac = (u + Fraction(1, 2)) - ((u + Fraction(1, 2)).numerator // (u + Fraction(1, 2)).denominator)
            if min(frac, 1 - frac) <= Fraction(1, 10 ** 9):
                near += 1
                continue
            exact_col = (u + Fraction(1, 2)).__floor__()
            assert int(np.floor(x + 0.5)) == exact_col
            checked += 1
    assert checked > 1000 and near == 0


def test_track_affine_flat_road_meets_vanishing_point():
    """Flat road, straight lanes: V_px and V_py are constant, every track is the straight line
    through (V_px, V_py), so a_v = (v - V_py) / (v_max - V_py) and b_v = V_px (1 - a_v)."""
    H = 60
    vpy = np.full(H, 10.25)
    vpx = np.full(H, 123.5)
    a, b = oracle.track_affine(vpx, vpy, 12, 12)
    for v in range(12, H):
        aw = (v - 10.25) / (H - 1 - 10.25)
        assert abs(a[v] - aw) <= 1e-13 and abs(b[v] - 123.5 * (1 - aw)) <= 1e-10


# ----------------------------------------------------------------------------- candidate mask
def test_cand_mask_exact_columns():
    """One marked pixel per band row: the hit candidates are exactly those whose exact track
    column (rational arithmetic) is a marked pixel on a marked row, and keep is hit dilated."""
    g, d, r = _frame_tables()
    H, W = g.shape
    half = W // 2
    top = oracle.band_top(r.v_h, H, 1, 0)
    A, B = _exact_AB(r.vpx, r.vpy, r.v_end, H)
    # exact affine maps of the band rows
    ea, eb = {}, {}
    a_, b_ = Fraction(1), Fraction(0)
    for v in range(H - 1, top - 1, -1):
        if v < H - 1:
            a_, b_ = B[v] * a_, B[v] * b_ + A[v]
        ea[v], eb[v] = a_, b_
    rng = np.random.default_rng(3)
    bits = np.zeros((4, 16, W), np.uint8)
    marked = {}
    for rr in (0, 5, 11, 15):
        col = int(rng.integers(50, W - 50))
        bits[0, rr, col] = 1
        marked[top + rr] = col
    want = np.zeros(2 * W, np.uint8)
    for i in range(2 * W):
        us = i - half
        for v, col in marked.items():
            x = ea[v] * us + eb[v] + Fraction(1, 2)
            if 0 <= x < W and x.__floor__() == col:
                want[i] = 1
    assert want.sum() > 0
    for dil in (0, 3):
        hit, keep, kept = oracle.cand_mask(bits, W, r.v_h, r.v_end, r.vpx, r.vpy, n_bands=1, dilate=dil)
        assert np.array_equal(hit, want)
        wk = np.array([want[max(0, i - dil):i + dil + 1].max() for i in range(2 * W)], np.uint8)
        assert np.array_equal(keep, wk) and kept == int(wk.sum())
    hit, keep, kept = oracle.cand_mask(np.zeros_like(bits), W, r.v_h, r.v_end, r.vpx, r.vpy, dilate=4)
    assert hit.sum() == 0 and keep.sum() == 0 and kept == 0


# ----------------------------------------------------------------------------- whole narrowed search
def _plain_curve_bits(r, H, W, nb):
    """Decisions of an ideal network: within 2 + 0.139 f(v) columns of a curve of the plain
    search on the band rows (the training label of the network)."""
    bits = np.zeros((4, 16, W), np.uint8)
    u = np.arange(W, dtype=np.float64)
    for k in range(nb):
        top = oracle.band_top(r.v_h, H, nb, k)
        for rr in range(16):
            v = top + rr
            rad = 2.0 + 0.139 * r.f[v]
            for l in range(r.n_lanes):
                bits[k, rr] |= (np.abs(u - r.curves[l, v]) <= rad).astype(np.uint8)
    return bits


@pytest.mark.parametrize("seq,idx", [(8, 0), (8, 31), (9, 12), (10, 50)])
def test_ideal_decisions_return_the_plain_lanes(seq, idx):
    """Fed the plain search's own lanes as decisions, the narrowed search finds the plain
    lanes, with the V_px window and with the candidate mask, and without a fallback."""
    g, d, _ = synth.make_batch("c2", seq, 1, idx)
    g, d = g[0], d[0]
    H, W = g.shape
    plain = oracle.detect(g, d, 128, frame_idx=idx)
    assert plain.n_lanes >= 2
    for nb in (1, 2):
        bits = _plain_curve_bits(plain, H, W, nb)
        for dil in (-1, 8):
            r = oracle.detect_pruned(g, d, 128, bits, n_bands=nb, dilate=dil, frame_idx=idx)
            assert r.prune[1] == 0, (nb, dil, r.prune)
            assert np.array_equal(r.mx_path, plain.mx_path), (nb, dil)
            assert r.u_start.tolist() == plain.u_start.tolist(), (nb, dil)
            if dil >= 0:
                assert r.prune[14] < 2 * W


def test_caller_seed_in_the_narrowed_search():
    """A caller's RANSAC seed (a stream's previous fit) is hypothesis 0 of the narrowed search
    as of the full one: with ideal decisions (same DP path) the V_px fit, its trace and the lanes
    equal those of the full search with that seed; a fallback frame (no marked edge) uses it too;
    a NaN seed is no seed."""
    g, d, _ = synth.make_batch("c2", 9, 2, 20)
    H, W = g.shape[1:]
    P = oracle.default_params(n_hyp=1)                    # one hypothesis per round: the seed's, when given
    prev = oracle.detect(g[0], d[0], 128, P, frame_idx=20)
    seed = np.array(prev.gamma.raw[:5])
    plain = oracle.detect(g[1], d[1], 128, P, frame_idx=21, seed_gamma=seed)
    unseeded = oracle.detect(g[1], d[1], 128, P, frame_idx=21)
    assert plain.trace_gamma.tolist() != unseeded.trace_gamma.tolist()
    bits = _plain_curve_bits(oracle.detect(g[1], d[1], 128, frame_idx=21), H, W, 1)   # the lanes, marked
    r = oracle.detect_pruned(g[1], d[1], 128, bits, params=P, frame_idx=21, seed_gamma=seed)
    assert r.prune[1] == 0 and np.array_equal(r.mx_path, plain.mx_path)
    assert r.trace_gamma.tolist() == plain.trace_gamma.tolist() and list(r.gamma.raw) == list(plain.gamma.raw)
    assert r.u_start.tolist() == plain.u_start.tolist()
    fb = oracle.detect_pruned(g[1], d[1], 128, np.zeros((4, 16, W), np.uint8), params=P, frame_idx=21, seed_gamma=seed)
    assert fb.prune[1] & 1 and fb.trace_gamma.tolist() == plain.trace_gamma.tolist()
    none = oracle.detect_pruned(g[1], d[1], 128, bits, params=P, frame_idx=21, seed_gamma=np.full(5, np.nan))
    assert none.trace_gamma.tolist() == unseeded.trace_gamma.tolist()


def test_narrowed_search_fallbacks():
    """No marked edge: no seed, the full search, the plain lanes, flag FALLBACK.  A window of
    one column (delta 0) pinned on the seed must reach its inner edge and fall back."""
    g, d, _ = synth.make_batch("c2", 8, 1, 0)
    g, d = g[0], d[0]
    H, W = g.shape
    plain = oracle.detect(g, d, 128)
    r = oracle.detect_pruned(g, d, 128, np.zeros((4, 16, W), np.uint8))
    assert r.prune[1] & 1 and r.prune[1] & 4 and r.prune[2] == -1
    assert r.flags & 16 and r.u_start.tolist() == plain.u_start.tolist()
    bits = _plain_curve_bits(plain, H, W, 1)
    r = oracle.detect_pruned(g, d, 128, bits, delta_x=0)
    assert r.prune[3] == r.prune[4] == r.prune[2] and r.prune[1] & 8
    assert np.array_equal(r.mx_path, plain.mx_path) and r.u_start.tolist() == plain.u_start.tolist()


# ----------------------------------------------------------------------------- bands
def test_band_top_layout():
    for H in (96, 192, 375, 1080):
        for v_h in (0, H // 3, H - 40, H - 16, H - 15):
            for nb in (1, 2, 3, 4):
                tops = [oracle.band_top(v_h, H, nb, k) for k in range(nb)]
                assert tops == [cnn.band_top(v_h, H, nb, k) for k in range(nb)]
                if H - v_h < 16:
                    assert tops == [-1] * nb
                    continue
                assert tops[0] == H - 16                        # the bottom band ends on the last row
                assert all(v_h <= t <= H - 16 for t in tops)    # every band lies on road rows
                assert tops == sorted(tops, reverse=True)       # bands go up the image
                gaps = [tops[k - 1] - tops[k] for k in range(1, nb)]
                step = (H - v_h - 16) / nb                      # bands spread evenly over the road
                assert all(int(step) <= gp <= int(step) + 1 for gp in gaps), (H, v_h, nb, tops)
                assert tops[-1] - v_h <= int(step) + 1


def test_band_features_are_a_slice_of_the_frame_features():
    """The band's input tensor equals the features of the whole frame (zero outside the image)
    cut at the band's rows, for the bottom, a middle and a top band."""
    g, d, r = _frame_tables()
    H, W = g.shape
    D, ok = cnn.disparity_values(d)
    gp = np.zeros((H + 2, W), np.uint8)
    gp[1:-1] = g
    full = cnn.features(gp, D, ok, r.f)
    gx, gy = oracle.sobel(g)
    inner = (slice(1, H - 1), slice(1, W - 1))
    # the gradient channel on the frame interior is the library's Sobel
    assert np.allclose(full[..., 1][inner], np.sqrt(gx[inner] ** 2.0 + gy[inner] ** 2.0) / 1020.0, atol=0)
    for top in (H - 16, (H + r.v_h) // 2, r.v_h):
        band = cnn.band_features(g, d, r.f, top)
        assert band.shape == (16, W, 4)
        assert np.array_equal(band, full[top:top + 16]), top
