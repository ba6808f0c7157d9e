"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one oracle step against something other than the oracle itself: published
known-answer vectors, numpy/scipy library routines, exact rational arithmetic, brute-force
enumeration on tiny inputs, closed forms of the synthetic scene, or invariants.  None of
these tests needs a GPU.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from paper_1807_02752_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


# ----------------------------------------------------------------------------- Philox (O5)
def test_philox_known_answers():
    """Random123 KAT vectors of Philox4x64-10."""
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert oracle.philox(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


def _numpy_block(counter, key):
    """One Philox4x64-10 block from numpy's independent implementation.  numpy increments
    its 256-bit counter before producing a block, so start one below."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(counter)) - 1
    c &= (1 << 256) - 1
    ctr = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=ctr)
    return [int(x) for x in bg.random_raw(4)]


def test_philox_matches_numpy():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 1 << 63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 1 << 63, size=2, dtype=np.int64)]
        assert oracle.philox(ctr, key) == _numpy_block(ctr, key)
    assert oracle.philox([0, 0, 0, 0], [0, 0]) == _numpy_block([0, 0, 0, 0], [0, 0])


@pytest.mark.parametrize("n_cur,s", [(3, 3), (5, 5), (7, 3), (200, 5), (1080, 5), (129, 3)])
def test_ransac_sample_draw_from_numpy_words(n_cur, s):
    """Index draw: words of blocks 0,1,.. of counter (frame, stage<<32|round, hyp, blk) mapped
    to floor(w * n / 2^64), repeats skipped -- words taken from numpy's Philox."""
    for (seed, stream, frame, stage, rnd, hyp) in [(0, 0, 0, 0, 0, 0), (5, 9, 17, 1, 3, 63), (1 << 40, 2, 999, 0, 15, 7)]:
        got = oracle.sample(n_cur, s, seed=seed, stream_id=stream, frame_idx=frame, stage=stage, rnd=rnd, hyp=hyp)
        want = []
        for blk in range(16):
            if len(want) == s:
                break
            for w in _numpy_block([frame, (stage << 32) | rnd, hyp, blk], [seed, stream]):
                ix = (w * n_cur) >> 64
                if ix not in want and len(want) < s:
                    want.append(ix)
        assert got.tolist() == want


# ----------------------------------------------------------------------------- O1 histogram
def _hist_bruteforce(disp, d_max, fmt):
    H, W = disp.shape
    m = np.zeros((H, d_max + 1), np.int64)
    for v in range(H):
        for u in range(W):
            r = disp[v, u]
            if fmt == 1:
                x = float(r)
                if not (math.isfinite(x) and x > 0):
                    continue
                D = Fraction(x)
            elif fmt == 2:
                if r == 0:
                    continue
                D = Fraction(int(r), 16)
            else:
                if r == 0:
                    continue
                D = Fraction(int(r))
            b = math.floor(D + Fraction(1, 2))
            m[v, min(b, d_max)] += 1
    return m


def test_hist_u8_u16_f32_bruteforce():
    rng = np.random.default_rng(1)
    u8 = rng.integers(0, 256, size=(7, 23)).astype(np.uint8)
    assert (oracle.vdisp_hist(u8, 100) == _hist_bruteforce(u8, 100, 0)).all()
    u16 = rng.integers(0, 5000, size=(6, 19)).astype(np.uint16)
    u16[0, :8] = [0, 1, 7, 8, 9, 23, 24, 25]          # half-way cases of (raw + 8) >> 4
    assert (oracle.vdisp_hist(u16, 255) == _hist_bruteforce(u16, 255, 2)).all()
    f = rng.uniform(-3, 140, size=(5, 31)).astype(np.float32)
    f[0, :10] = [np.nan, np.inf, -np.inf, 0.0, -0.0, 0.5, 1.5, np.nextafter(np.float32(0.5), np.float32(0)),
                 np.float32(128.5), np.float32(1e30)]
    assert (oracle.vdisp_hist(f, 128) == _hist_bruteforce(f, 128, 1)).all()


def test_hist_row_sums_equal_valid_count():
    _, d, _ = synth.make_c2(0, 0)
    m = oracle.vdisp_hist(d, 128)
    valid = (np.isfinite(d) & (d > 0)).sum(axis=1)
    assert (m.sum(axis=1) == valid).all()
    _, d1, _ = synth.make_c1(0)
    assert (oracle.vdisp_hist(d1, 48).sum(axis=1) == (d1 != 0).sum(axis=1)).all()


def test_hist_u16q4_closed_form():
    raw = np.arange(1, 4200, dtype=np.uint16).reshape(1, -1)
    m = oracle.vdisp_hist(raw, 255)
    want = np.bincount(np.minimum((raw[0].astype(np.int64) + 8) >> 4, 255), minlength=256)
    assert (m[0] == want).all()


# ----------------------------------------------------------------------------- O2 DP
def _dp_bruteforce(m_y, tau_max, lam):
    H, D1 = m_y.shape
    best = None
    for v0 in range(H):
        for taus in itertools.product(range(tau_max + 1), repeat=D1 - 1):
            v, path, ok = v0, [v0], True
            for t in taus:
                v += t
                if v > H - 1:
                    ok = False
                    break
                path.append(v)
            if not ok:
                continue
            e = -sum(int(m_y[path[d], d]) for d in range(D1)) + lam * sum(taus)
            key = (e, v0, taus)
            if best is None or key < best[0]:
                best = (key, path)
    return best[1]


@pytest.mark.parametrize("seed", range(12))
def test_vdisp_dp_exhaustive(seed):
    rng = np.random.default_rng(seed)
    H = int(rng.integers(3, 7))
    D1 = int(rng.integers(2, 5))
    tau_max = int(rng.integers(1, 3))
    lam = int(rng.integers(0, 3))
    m_y = rng.integers(0, 3, size=(H, D1)).astype(np.int32)      # many ties on purpose
    path_v, px, py = oracle.vdisp_dp(m_y, tau_max=tau_max, lam=lam)
    want = _dp_bruteforce(m_y, tau_max, lam)
    assert path_v.tolist() == want
    keep = [(v, d) for d, v in enumerate(want) if m_y[v, d] > 0]
    assert list(zip(px.tolist(), py.tolist())) == keep


# ----------------------------------------------------------------------------- O10 row DP
_RANK = lambda t: 0 if t == 0 else (2 * abs(t) - 1 if t < 0 else 2 * abs(t))   # noqa: E731


def _rowdp_bruteforce(mx, v_h, tau_max, lam):
    H, W2 = mx.shape
    rows = list(range(v_h, H))
    best = None
    for c0 in range(W2):
        for taus in itertools.product(range(-tau_max, tau_max + 1), repeat=len(rows) - 1):
            c, path, ok = c0, [c0], True
            for t in taus:
                c += t
                if not (0 <= c < W2):
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


@pytest.mark.parametrize("seed", range(10))
def test_row_dp_exhaustive(seed):
    rng = np.random.default_rng(100 + seed)
    H = int(rng.integers(3, 6))
    v_h = int(rng.integers(0, 2))
    W2 = int(rng.integers(3, 7))
    tau_max = int(rng.integers(1, 3))
    lam = int(rng.integers(0, 3))
    mx = -rng.integers(0, 3, size=(H, W2)).astype(np.int64)
    cpath = oracle.row_dp(mx, v_h, tau_max=tau_max, lam=lam)
    assert cpath[v_h:].tolist() == _rowdp_bruteforce(mx, v_h, tau_max, lam)


# ----------------------------------------------------------------------------- O4 fit
def _exact_ls_predict(x, y, degree):
    """Exact least squares through Fractions (raw basis), predictions at x."""
    n = degree + 1
    A = [[Fraction(sum(Fraction(xi) ** (i + j) for xi in x)) for j in range(n)] for i in range(n)]
    b = [Fraction(sum(Fraction(yi) * Fraction(xi) ** i for xi, yi in zip(x, y))) for i in range(n)]
    # Gauss-Jordan in exact arithmetic
    for i in range(n):
        piv = next(r for r in range(i, n) if A[r][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        b[i], b[piv] = b[piv], b[i]
        for r in range(n):
            if r != i and A[r][i] != 0:
                f = A[r][i] / A[i][i]
                A[r] = [a - f * c for a, c in zip(A[r], A[i])]
                b[r] -= f * b[i]
    coef = [b[i] / A[i][i] for i in range(n)]
    return [sum(c * Fraction(xi) ** p for p, c in enumerate(coef)) for xi in x]


def _eval_s(coef, center, k, x):
    s = (np.asarray(x, np.float64) - center) / (2.0 ** k)
    r = np.full_like(s, coef[-1])
    for c in coef[-2::-1]:
        r = r * s + c
    return r


def _basis(x):
    c = (int(min(x)) + int(max(x))) >> 1
    wm = max(int(max(x)) - c, c - int(min(x)))
    k = 0
    while (1 << k) < wm:
        k += 1
    return c, k


@pytest.mark.parametrize("degree,seed", [(2, 0), (2, 1), (4, 2), (4, 3), (4, 4)])
def test_fit_matches_exact_rational_ls(degree, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(degree + 2, 14))
    x = np.sort(rng.choice(np.arange(150, 375), size=n, replace=False)).astype(np.int32)
    y = rng.integers(-300, 1500, size=n).astype(np.int32)
    c, k = _basis(x)
    rc, coef = oracle.fit(x, y, degree, c, k)
    assert rc == 0
    got = _eval_s(coef, c, k, x)
    want = np.array([float(p) for p in _exact_ls_predict(x.tolist(), y.tolist(), degree)])
    assert np.allclose(got, want, rtol=0, atol=1e-9 * max(1.0, np.abs(want).max()))


def test_fit_matches_polyfit_large():
    rng = np.random.default_rng(5)
    x = np.arange(480, 1080, dtype=np.int32)
    y = (3e-7 * (x - 700.0) ** 4 - 1e-4 * (x - 700.0) ** 3 + 0.01 * (x - 700.0) ** 2 + rng.normal(0, 5, x.size))
    y = np.rint(y).astype(np.int32)
    c, k = _basis(x)
    rc, coef = oracle.fit(x, y, 4, c, k)
    assert rc == 0
    ref = np.polyval(np.polyfit((x - c) / 2.0 ** k, y.astype(float), 4), (x - c) / 2.0 ** k)
    assert np.abs(_eval_s(coef, c, k, x) - ref).max() < 1e-7


def test_fit_recovers_exact_polynomial_and_flags_singular():
    x2 = np.arange(0, 40, 4, dtype=np.int32)
    y2 = (x2 * x2 - 3 * x2 + 7).astype(np.int32)
    c, k = _basis(x2)
    rc, coef = oracle.fit(x2, y2, 2, c, k)
    assert rc == 0 and np.abs(_eval_s(coef, c, k, x2) - y2).max() < 1e-9
    # fewer distinct abscissae than unknowns -> singular
    rc, _ = oracle.fit(np.array([5, 5, 5, 9], np.int32), np.array([1, 2, 3, 4], np.int32), 2, 7, 1)
    assert rc == 1


# ----------------------------------------------------------------------------- O3 RANSAC
@pytest.mark.parametrize("degree,tr", [(2, 4.0), (4, 16.0)])
def test_ransac_planted_outliers(degree, tr):
    rng = np.random.default_rng(degree)
    x = np.arange(160, 375, dtype=np.int32)
    if degree == 2:
        truth = 0.0015 * (x - 150.0) ** 2 + 0.3 * (x - 150.0)
    else:
        truth = 600 + 0.2 * (x - 260.0) + 1e-3 * (x - 260.0) ** 2 - 4e-6 * (x - 260.0) ** 3 + 2e-8 * (x - 260.0) ** 4
    y = np.rint(truth).astype(np.int32)
    out_idx = rng.choice(x.size, size=x.size // 5, replace=False)
    y[out_idx] += rng.choice([-1, 1], size=out_idx.size) * rng.integers(40, 200, size=out_idx.size)
    res, trace = oracle.ransac(x, y, degree, tr, seed=3, stream_id=1, frame_idx=2, stage=degree // 4)
    assert res.ok == 1 and res.flags == 0
    inl = np.setdiff1d(np.arange(x.size), out_idx)
    assert res.n_survivors == inl.size
    # the final model is the least-squares fit of exactly the planted inliers
    c, k = _basis(x)
    rc, coef = oracle.fit(x, y, degree, c, k, idx=inl.astype(np.int32))
    assert rc == 0 and np.array_equal(np.array(res.coef[: degree + 1]), coef)
    ref = np.polyval(np.polyfit((x[inl] - c) / 2.0 ** k, y[inl].astype(float), degree), (x - c) / 2.0 ** k)
    assert np.abs(_eval_s(coef, c, k, x) - ref).max() < 1e-6
    # the exit test of the do-while: the last round kept >= 99% of its points
    assert 100 * trace[-1, 1] >= 99 * trace[-1, 2]


def test_ransac_no_consensus_and_literal_mode():
    rng = np.random.default_rng(9)
    x = np.arange(0, 60, dtype=np.int32)
    y = rng.integers(-1000000, 1000000, size=60).astype(np.int32)   # a 6th point within 4 of a
    res, trace = oracle.ransac(x, y, 4, 16.0, seed=1)                 # random quartic: ~1e-4 chance
    assert res.flags & 1                        # no sample explains a tenth of the points
    assert trace.shape[0] == 1 and trace[0, 1] < 6
    # literal reading: one sample per round still converges on clean data
    y2 = np.rint(0.01 * (x - 30.0) ** 2).astype(np.int32)
    res2, _ = oracle.ransac(x, y2, 2, 4.0, n_hyp=1, seed=4)
    assert res2.ok == 1 and res2.n_survivors == 60
    # too few points for a quartic
    res3, _ = oracle.ransac(x[:4], y2[:4], 4, 16.0)
    assert res3.ok == 0 and res3.flags & 1


def test_ransac_seed_hypothesis():
    x = np.arange(100, 300, dtype=np.int32)
    y = np.rint(0.5 * x + 10).astype(np.int32)
    y[::7] += 500
    seed_raw = np.array([10.0, 0.5, 0, 0, 0])
    res, trace = oracle.ransac(x, y, 4, 16.0, seed_raw=seed_raw, seed=0, stage=1)
    assert res.ok and trace[0, 1] == 200 - len(range(0, 200, 7))


# ----------------------------------------------------------------------------- O6 road tables
def test_road_tables_closed_form_vpy():
    """Tables from a beta that is exactly the generator's road: V_py = v0 + a w^2/(2aw + b)."""
    for (a, b, v0, H) in [(0.0038881, 0.4, 24, 96), (0.000688, 0.35, 170, 375), (2.5e-4, 0.2, 490, 1080)]:
        beta = oracle.ldref.FitOut()
        c, k = (v0 + H - 1) >> 1, 0
        while (1 << k) < (H - 1 - c):
            k += 1
        # f(v) = a (v - v0)^2 + b (v - v0) in s = (v - c)/2^k:  w = 2^k s + (c - v0)
        sc, dc = float(2 ** k), float(c - v0)
        beta.center, beta.kshift = c, k
        beta.coef[0] = a * dc * dc + b * dc
        beta.coef[1] = (2 * a * dc + b) * sc
        beta.coef[2] = a * sc * sc
        f, fp, vpy, v_h = oracle.road_tables(beta, H)
        v = np.arange(v0 + 1, H)
        w = v - v0
        assert np.abs(vpy[v0 + 1:] - (v0 + a * w * w / (2 * a * w + b))).max() < 1e-9
        assert np.abs(f[v0 + 1:] - (a * w * w + b * w)).max() < 1e-9
        # the horizon root is v0; rounding in the s basis may leave f(v0) a hair above 0
        assert v_h in (v0, v0 + 1)
        assert (f[v_h:] > 0).all() and (fp[v_h:] > 0).all() and not (f[v_h - 1] > 0 and fp[v_h - 1] > 0)


# ----------------------------------------------------------------------------- O7 Sobel
def test_sobel_matches_scipy():
    rng = np.random.default_rng(3)
    g = rng.integers(0, 256, size=(37, 53)).astype(np.uint8)
    gx, gy = oracle.sobel(g)
    kx = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]])
    ref_x = ndi.correlate(g.astype(np.int64), kx, mode="constant")
    ref_y = ndi.correlate(g.astype(np.int64), kx.T, mode="constant")
    inner = (slice(1, -1), slice(1, -1))
    assert (gx[inner] == ref_x[inner]).all() and (gy[inner] == ref_y[inner]).all()
    assert (gx[0] == 0).all() and (gx[-1] == 0).all() and (gx[:, 0] == 0).all() and (gy[:, -1] == 0).all()
    # dark-to-light transition gives G_x > 0
    step = np.zeros((5, 6), np.uint8)
    step[:, 3:] = 200
    assert oracle.sobel(step)[0][2, 3] > 0


def test_road_edges_mask_bruteforce():
    g, d, sc = synth.make_c2(1, 3)
    f = sc.f(np.arange(375))
    v_h = 180
    eu, ev, egx, egy = oracle.road_edges(g, d, f, v_h)
    gx, gy = oracle.sobel(g)
    D = d.astype(np.float64)
    valid = np.isfinite(D) & (D > 0)
    rows = np.arange(375)[:, None] >= v_h
    road = valid & rows & (np.abs(D - f[:, None]) <= 3.0)
    edge = road & (gx.astype(np.int64) ** 2 + gy.astype(np.int64) ** 2 > 100 ** 2)
    vv, uu = np.nonzero(edge)
    assert np.array_equal(ev, vv) and np.array_equal(eu, uu)
    assert np.array_equal(egx, gx[vv, uu]) and np.array_equal(egy, gy[vv, uu])


# ----------------------------------------------------------------------------- O8 votes
def test_votes_exact_rational():
    rng = np.random.default_rng(11)
    W, H, n = 300, 90, 400
    eu = rng.integers(0, W, n).astype(np.int32)
    ev = rng.integers(30, H, n).astype(np.int32)
    egx = rng.integers(-600, 600, n).astype(np.int32)
    egy = rng.integers(-600, 600, n).astype(np.int32)
    vpy = 20.0 + rng.uniform(-5, 5, H)
    b = oracle.votes(eu, ev, egx, egy, vpy, W)
    checked = 0
    for i in range(n):
        if egx[i] == 0:
            assert b[i] == -1
            continue
        x = Fraction(int(eu[i])) + (Fraction(int(ev[i])) - Fraction(vpy[ev[i]])) * Fraction(int(egy[i]), int(egx[i]))
        t = x + Fraction(1, 2)
        if abs(t - round(t)) < Fraction(1, 10 ** 9):
            continue                                 # rounding-ambiguous: FP64 may go either way
        c = math.floor(t) + W // 2
        assert b[i] == (c if 0 <= c < 2 * W else -1)
        checked += 1
    assert checked > 300


def _flat_wedge_scene(W=200, H=80, v0=20, c=100):
    """Flat road (V_py = v0 on every row); the bright region is the wedge |u - c| <= v - v0,
    whose two boundaries are 45-degree lines through V_p = (c, v0).  Sobel is symmetric
    about such a boundary, so a pixel centred on it has |G_x| = |G_y|."""
    v = np.arange(H)[:, None]
    u = np.arange(W)[None, :]
    grey = np.where((np.abs(u - c) <= v - v0) & (v > v0), 200, 90).astype(np.uint8)
    disp = (np.where(v > v0, 0.5 * (v - v0), 0.0) * np.ones((1, W))).astype(np.float32)
    return grey, disp


def test_votes_straight_lanes_hit_vanishing_point():
    grey, disp = _flat_wedge_scene()
    H, W = grey.shape
    f = np.maximum(0.5 * (np.arange(H) - 20.0), 0)
    vpy = np.full(H, 20.0)
    eu, ev, egx, egy = oracle.road_edges(grey, disp, f, 30)
    b = oracle.votes(eu, ev, egx, egy, vpy, W)
    on_line = np.abs(eu - 100) == ev - 20
    assert on_line.sum() > 50
    assert (np.abs(egx[on_line]) == np.abs(egy[on_line])).all()
    assert (b[on_line] == 100 + W // 2).all()


# ----------------------------------------------------------------------------- O9 band
def test_band_direct_vs_sliding_prefix_sums():
    rng = np.random.default_rng(2)
    H, W2, v_h, chi = 120, 37, 20, 25
    h = rng.integers(0, 4, size=(H, W2)).astype(np.int32)
    h[:v_h] = 99                                       # above the road: must not be counted
    mx = oracle.band(h, v_h, chi)
    cs = np.vstack([np.zeros((1, W2), np.int64), np.cumsum(h[v_h:].astype(np.int64), axis=0)])
    for v in range(v_h, H):
        lo, hi = max(v - chi, v_h) - v_h, min(v + chi, H - 1) - v_h
        assert (mx[v] == -(cs[hi + 1] - cs[lo])).all()


# ----------------------------------------------------------------------------- O12 weights
def test_weights_against_angle_difference():
    rng = np.random.default_rng(4)
    n = 3000
    eu = rng.integers(0, 400, n).astype(np.int32)
    ev = rng.integers(150, 375, n).astype(np.int32)
    egx = rng.integers(-700, 700, n).astype(np.int32)
    egy = rng.integers(-700, 700, n).astype(np.int32)
    vpx = rng.uniform(100, 300, 375)
    vpy = rng.uniform(100, 140, 375)
    q = oracle.weights(eu, ev, egx, egy, vpx, vpy)
    th_e = np.arctan2(egx.astype(float), -egy.astype(float))          # edge-line orientation
    th_r = np.arctan2(vpy[ev] - ev, vpx[ev] - eu)                       # ray to V_p
    delta = np.mod(th_e - th_r, np.pi)
    delta = np.minimum(delta, np.pi - delta)                            # angle between lines
    away = np.abs(delta - np.pi / 6) > 1e-9
    w = np.where(delta <= np.pi / 6, np.exp(-(delta / (np.pi / 36)) / 3.5 ** 2), 0.0)
    assert np.allclose(q[away], (egx * w)[away], rtol=1e-12, atol=1e-9)
    assert (np.abs(delta - np.pi / 6) < 1e-6).sum() < 5


def test_weights_special_angles():
    # V_p straight above the pixel: the ray is vertical
    vpx = np.array([0.0] * 10 + [50.0])
    vpy = np.zeros(11)
    # edge tangent along the ray (vertical edge, G_y = 0) -> w = 1, q = G_x
    assert oracle.weights([50], [10], [7], [0], vpx, vpy)[0] == 7.0
    # tangent t = (-G_y, G_x) against the vertical ray: cos^2(delta) = G_x^2 / (G_x^2 + G_y^2),
    # so delta <= pi/6 iff G_x^2 >= 3 G_y^2: with G_x = 1000 the boundary lies between G_y = 577
    # (kept) and 578 (cut)
    q = oracle.weights([50, 50], [10, 10], [1000, 1000], [577, 578], vpx, vpy)
    d = math.atan(577 / 1000)
    assert abs(q[0] - 1000 * math.exp(-(d / (math.pi / 36)) / 3.5 ** 2)) < 1e-9
    assert q[1] == 0.0


def test_prior_work_vote_against_angles():
    """vote = 1: V(e) = |grad| cos(theta_e - theta_Vp), theta_e the direction of the tangent
    (-G_y, G_x), theta_Vp that of the ray from V_p(v) to the pixel, both from arctan2."""
    rng = np.random.default_rng(5)
    n = 3000
    eu = rng.integers(0, 400, n).astype(np.int32)
    ev = rng.integers(150, 375, n).astype(np.int32)
    egx = rng.integers(-700, 700, n).astype(np.int32)
    egy = rng.integers(-700, 700, n).astype(np.int32)
    vpx = rng.uniform(100, 300, 375)
    vpy = rng.uniform(100, 140, 375)
    q = oracle.weights(eu, ev, egx, egy, vpx, vpy, vote=1)
    th_e = np.arctan2(egx.astype(float), -egy.astype(float))
    th_p = np.arctan2(ev - vpy[ev], eu - vpx[ev])
    want = np.hypot(egx, egy) * np.cos(th_e - th_p)
    assert np.allclose(q, want, rtol=1e-12, atol=1e-9)


def test_prior_work_vote_special_cases():
    vpx = np.array([0.0] * 10 + [50.0])
    vpy = np.zeros(11)
    # V_p straight above: a vertical edge votes its G_x (either sign), a horizontal one 0,
    # a tangent 60 degrees off the ray half its magnitude, the pixel at V_p itself 0
    q = oracle.weights([50, 50, 50], [10, 10, 10], [7, -7, 0], [0, 0, 5], vpx, vpy, vote=1)
    assert q[0] == 7.0 and q[1] == -7.0 and q[2] == 0.0
    g = 1000.0
    q = oracle.weights([50], [10], [500], [-866], vpx, vpy, vote=1)[0]
    assert abs(q - 500.0) < 1e-9 and abs(np.hypot(500, 866) - g) < 0.5
    assert oracle.weights([0], [0], [30], [40], np.zeros(1), np.zeros(1), vote=1)[0] == 0.0


# ----------------------------------------------------------------------------- O13 M0/M1
def test_m0_m1_match_scipy():
    rng = np.random.default_rng(8)
    q = np.zeros((40, 57))
    idx = rng.integers(0, q.size, 300)
    q.flat[idx] = rng.normal(0, 300, 300)
    m0, m1 = oracle.m0m1(q)
    ref0 = ndi.correlate(q, np.ones((7, 3)), mode="constant")
    G = np.outer([1, 2, 1], [1, 0, -1]).astype(float)
    ref1 = ndi.convolve(ref0, G, mode="constant")
    assert np.allclose(m0, ref0, atol=1e-9) and np.allclose(m1, ref1, atol=1e-9)
    # negative on the centre of a bright marking (positive G_x left edge, negative right edge)
    q2 = np.zeros((20, 30))
    q2[:, 10] = 400.0
    q2[:, 14] = -400.0
    _, m1b = oracle.m0m1(q2)
    assert m1b[10, 12] < 0


# ----------------------------------------------------------------------------- O14 energy / peaks
def test_energy_tracks_are_lines_through_vp():
    H, W, v_h = 80, 100, 25
    vpx = np.full(H, 61.0)
    vpy = np.full(H, 19.5)
    m1 = np.zeros((H, W))
    starts = np.array([-30, 0, 17, 61, 99, 130], np.int32)
    _, v_end, curves = oracle.energy(m1, vpx, vpy, v_h, tracks=starts)
    assert v_end == v_h
    v = np.arange(v_h, H)
    for k, u0 in enumerate(starts):
        line = 61.0 + (u0 - 61.0) * (v - 19.5) / (H - 1 - 19.5)
        assert np.abs(curves[k, v_h:] - line).max() < 1e-9
        assert np.isnan(curves[k, :v_h]).all()


def test_energy_of_planted_track_is_minus_rows():
    H, W, v_h = 70, 90, 20
    vpx = 45.0 + 0.05 * (np.arange(H) - 40.0)
    vpy = np.full(H, 12.25)
    _, v_end, curves = oracle.energy(np.zeros((H, W)), vpx, vpy, v_h, tracks=np.array([30], np.int32))
    m1 = np.zeros((H, W))
    for v in range(v_end, H):
        m1[v, int(math.floor(curves[0, v] + 0.5))] = -1.0
    E, _, _ = oracle.energy(m1, vpx, vpy, v_h)
    assert E[30 + W // 2] == -(H - v_end)
    assert E.min() == -(H - v_end)


def _peaks_bruteforce(E, W, rho, d_nms):
    mn = E.min()
    if mn >= 0:
        return []
    cand = [i for i in range(1, len(E) - 1) if E[i] < E[i - 1] and E[i] < E[i + 1] and E[i] < rho * mn]
    cand.sort(key=lambda i: (E[i], i))
    acc = []
    for i in cand:
        if len(acc) < 16 and all(abs(i - j) > d_nms for j in acc):
            acc.append(i)
    return sorted(i - W // 2 for i in acc)


@pytest.mark.parametrize("seed", range(6))
def test_peaks_bruteforce(seed):
    rng = np.random.default_rng(seed)
    W = 150
    E = np.round(rng.normal(0, 1, 2 * W).cumsum() * 10) / 10 - 3     # ties and plateaus
    us, el = oracle.peaks(E, W, rho=0.25, d_nms=8)
    want = _peaks_bruteforce(E, W, 0.25, 8)
    assert us.tolist() == want
    assert np.array_equal(el, E[np.array(want, int) + W // 2] if want else np.zeros(0))
    assert oracle.peaks(np.abs(E), W)[0].size == 0                   # no negative energy, no lane


# ----------------------------------------------------------------------------- whole path vs GT
def _gt_tables(sc, H):
    v = np.arange(H, dtype=float)
    w = v - sc.v0
    f = sc.f(v)
    fp = 2 * sc.a * w + sc.b
    with np.errstate(all="ignore"):
        vpy = v - f / fp
        vpx = sc.u_c(v) - (sc.p + 2 * sc.q * w) * f / fp
    return vpy, vpx


def test_small_frame_against_scene_ground_truth():
    g, d, sc = synth.make_c1(0)
    r = oracle.detect(g, d, sc.d_max)
    assert r.flags == 0 and r.v_h == 25
    vpy, vpx = _gt_tables(sc, 96)
    rows = np.arange(r.v_h + 10, 96)
    assert np.abs(r.vpy[rows] - vpy[rows]).max() < 1.0
    assert np.median(np.abs(r.vpx[rows] - vpx[rows])) < 2.0
    gt = [sc.lane_u(k, 95) for k in range(2)]
    assert r.n_lanes == 2
    assert all(abs(u - g_) <= 2.0 for u, g_ in zip(sorted(r.u_start), sorted(gt)))


@pytest.mark.parametrize("seed,idx", [(0, 0), (0, 10), (3, 0)])
def test_kitti_size_frame_against_scene_ground_truth(seed, idx):
    g, d, sc = synth.make_c2(seed, idx)
    r = oracle.detect(g, d, sc.d_max)
    assert r.flags & 3 == 0
    vpy, vpx = _gt_tables(sc, 375)
    rows = np.arange(r.v_h + 10, 375)
    assert np.abs(r.vpy[rows] - vpy[rows]).max() < 1.0
    assert np.median(np.abs(r.vpx[rows] - vpx[rows])) < 4.0
    # the two inner lanes (inside the image at the bottom row) are found, within the
    # half-width of their marking (0.28 f / 2 = 14 px) plus 3 px
    for k in (1, 2):
        u = sc.lane_u(k, 374)
        assert np.min(np.abs(r.u_start - u)) <= 17.0


def test_degenerate_frames_set_flags():
    g, d = synth.degenerate("all_invalid")
    r = oracle.detect(g, d, 32)
    assert r.flags & 1 and r.n_lanes == 0 and np.isnan(r.vpx).all()
    g, d = synth.degenerate("obstacle_only")
    r = oracle.detect(g, d, 32)
    assert r.flags & 1 and r.n_lanes == 0
    g, d = synth.degenerate("flat_image")
    r = oracle.detect(g, d, 32)
    assert r.n_edges == 0 and r.n_lanes == 0


def test_nan_seed_is_no_seed():
    """A seed row whose first coefficient is NaN behaves exactly like no seed."""
    g, d, _ = synth.make_c2(0, 4)
    a = oracle.detect(g, d, 128)
    b = oracle.detect(g, d, 128, seed_gamma=np.array([np.nan, 0, 0, 0, 0.0]))
    assert np.array_equal(a.energy, b.energy) and np.array_equal(a.trace_gamma, b.trace_gamma)
    assert a.u_start.tolist() == b.u_start.tolist()
