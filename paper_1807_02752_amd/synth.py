"""Seeded synthetic stereo-road frames (stand-in for KITTI, which is not available).

This module only draws scenes and renders them: a left grey image, its disparity map
and the scene parameters that produced them.  It holds none of the lane detector's
arithmetic; ground-truth quantities that follow from the scene geometry are derived in
the tests.  The CPU reference and the GPU path consume exactly these arrays.

Scene model (Sec. 2.2 and 2.3 of the paper: a road whose projection on the v-disparity
map is a parabola, lane markings that share a per-row vanishing point):

* road profile   f(v) = a*w^2 + b*w,  w = v - v0    (disparity on road row v)
* lane centre    u_c(v) = c + p*w + q*w^2
* lane k         u_k(v) = u_c(v) + s_k * f(v)        (constant real-world offset)
* markings are brighter than the asphalt and rendered anti-aliased (area coverage);
  3 px wide in the small frame, 0.28 * f(v) px (a 0.15 m marking) in the larger ones

Randomness comes from numpy's Philox bit generator keyed by (config seed, frame index).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FMT_U8, FMT_F32, FMT_U16Q4 = 0, 1, 2


@dataclass
class Scene:
    width: int
    height: int
    fmt: int
    d_max: int
    a: float
    b: float
    v0: float
    c: float
    p: float
    q: float
    lanes: list            # list of (s_k, dashed)
    gain: float = 1.0
    obstacles: list = field(default_factory=list)   # (u0, u1, v_top, v_base, disparity)
    lane_values: list | None = None                 # per-lane marking grey (None: one value for all)
    paint: list = field(default_factory=list)       # road paint: (v_top, v_bottom, u_left, u_right, slope)

    def f(self, v):
        w = np.asarray(v, dtype=np.float64) - self.v0
        return self.a * w * w + self.b * w

    def u_c(self, v):
        w = np.asarray(v, dtype=np.float64) - self.v0
        return self.c + self.p * w + self.q * w * w

    def lane_u(self, k, v):
        return self.u_c(v) + self.lanes[k][0] * self.f(v)


def _rng(seed: int, idx: int) -> np.random.Generator:
    key = np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF), np.uint64(idx & 0xFFFFFFFFFFFFFFFF)], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def _lane_coverage(scene: Scene, k: int, width_fn, dash_k, cov: np.ndarray, sub: int = 4):
    """Max-accumulate into `cov` (H x W) the anti-aliased area coverage of lane k's marking.

    Each pixel row is split into `sub` sub-rows; on a sub-row the marking is the interval
    [u_k - hw, u_k + hw] and its overlap with the pixel [u - 0.5, u + 0.5] is exact.  Only a
    window of columns around the marking is evaluated on each row.
    """
    W, H = scene.width, scene.height
    s_k, dashed = scene.lanes[k]
    vv = np.arange(H, dtype=np.float64)[:, None] + (np.arange(sub)[None, :] + 0.5) / sub - 0.5   # H x sub
    fv = scene.f(vv)
    ok = vv >= scene.v0
    uk = scene.u_c(vv) + s_k * fv
    hw = 0.5 * width_fn(np.maximum(fv, 0.0))
    on = ok.astype(np.float64)
    if dashed and dash_k is not None:
        phase = np.floor(dash_k / np.maximum(fv, 1e-9))
        on = on * (np.mod(phase, 2) == 0)
    lo_u = np.floor(np.min(uk - hw, axis=1)) - 1                # per-row window start
    span = int(np.ceil(np.max(np.max(uk + hw, axis=1) - lo_u))) + 2
    span = max(1, min(span, W + 4))
    cols = lo_u[:, None] + np.arange(span)[None, :]             # H x span
    c = np.zeros((H, span))
    for j in range(sub):
        lo = np.maximum(cols - 0.5, (uk[:, j] - hw[:, j])[:, None])
        hi = np.minimum(cols + 0.5, (uk[:, j] + hw[:, j])[:, None])
        c += np.clip(hi - lo, 0.0, 1.0) * on[:, j][:, None]
    c /= sub
    inside = (cols >= 0) & (cols < W)
    rows = np.broadcast_to(np.arange(H)[:, None], cols.shape)
    r, cc, val = rows[inside], cols[inside].astype(np.int64), c[inside]
    np.maximum.at(cov, (r, cc), val)


def _render(scene: Scene, rng: np.random.Generator, *, disp_noise: float, dropout: float,
            dash_k: float | None, width_fn=None, lane_value: float = 200.0, road_value: float = 90.0,
            noise: float = 4.0, obstacle_value: float = 60.0):
    W, H = scene.width, scene.height
    v = np.arange(H, dtype=np.float64)[:, None]
    if width_fn is None:
        width_fn = lambda d: np.full_like(d, 3.0)   # noqa: E731  (constant 3 px markings)
    if scene.lane_values is None:
        cov = np.zeros((H, W))
        for k in range(len(scene.lanes)):
            _lane_coverage(scene, k, width_fn, dash_k, cov)
        grey = road_value + cov * (lane_value - road_value) + rng.normal(0.0, noise, size=(H, W))
    else:
        grey = np.full((H, W), road_value)
        for k in range(len(scene.lanes)):
            cov = np.zeros((H, W))
            _lane_coverage(scene, k, width_fn, dash_k, cov)
            grey += cov * (scene.lane_values[k] - road_value)
        grey += rng.normal(0.0, noise, size=(H, W))
    # road paint other than lane markings: bright parallelograms on the road surface (rows
    # v_top..v_bottom, columns u_left + slope (v_bottom - v) .. u_right + slope (v_bottom - v))
    for (vt, vb, ul, ur, sl) in scene.paint:
        for vv in range(max(0, vt), min(H - 1, vb) + 1):
            sh = sl * (vb - vv)
            c0, c1 = int(round(ul + sh)), int(round(ur + sh))
            c0, c1 = max(0, c0), min(W - 1, c1)
            if c0 <= c1:
                grey[vv, c0:c1 + 1] = lane_value + rng.normal(0.0, noise, size=c1 - c0 + 1)
    fv = scene.f(v)                                       # H x 1
    below = (v >= scene.v0)
    # disparity of the road surface, zero (invalid) above the horizon
    disp = np.where(below, np.broadcast_to(fv, (H, W)), 0.0).astype(np.float64)
    if disp_noise > 0:
        disp = np.where(below, disp + rng.normal(0.0, disp_noise, size=(H, W)), 0.0)
    # fronto-parallel obstacles standing on the road: constant disparity, darker grey
    for (u0, u1, vt, vb, d) in scene.obstacles:
        r0, r1 = max(0, vt), min(H - 1, vb)
        c0, c1 = max(0, u0), min(W - 1, u1)
        if r0 > r1 or c0 > c1:
            continue
        disp[r0:r1 + 1, c0:c1 + 1] = d
        grey[r0:r1 + 1, c0:c1 + 1] = rng.normal(obstacle_value, noise, size=(r1 - r0 + 1, c1 - c0 + 1))
    if dropout > 0:
        drop = rng.random(size=(H, W)) < dropout
        disp[drop] = 0.0
    if scene.gain != 1.0:
        grey = grey * scene.gain
    grey = np.clip(np.rint(grey), 0, 255).astype(np.uint8)
    disp = np.clip(disp, 0.0, float(scene.d_max))
    if scene.fmt == FMT_U8:
        disp = np.rint(disp).astype(np.uint8)
    elif scene.fmt == FMT_U16Q4:
        disp = np.rint(disp * 16.0).astype(np.uint16)
    else:
        disp = disp.astype(np.float32)
    return grey, disp


def marking_width(d):
    """Horizontal width in px of a 0.15 m marking seen with a 0.54 m baseline (>= 3 px)."""
    return np.maximum(3.0, (0.15 / 0.54) * d)


def _obstacles(scene: Scene, rng: np.random.Generator, frac: float):
    """Rectangles standing on the road until about `frac` of the pixels are covered."""
    W, H = scene.width, scene.height
    target = frac * W * H
    covered = 0.0
    obs = []
    # base rows range down to where the road disparity reaches d_max (partly visible)
    v_lo = scene.v0 + 0.06 * (H - scene.v0)
    aa, bb = scene.a, scene.b
    w_dmax = (-bb + math.sqrt(bb * bb + 4 * aa * scene.d_max)) / (2 * aa) if aa > 0 else (scene.d_max / bb)
    v_hi = scene.v0 + w_dmax
    tries = 0
    while covered < target and tries < 400:
        tries += 1
        vb = int(rng.uniform(v_lo, v_hi))
        d = float(scene.f(vb))
        if d <= 1.0:
            continue
        hgt = max(3, int(round(2.8 * d)))        # about 1.5 m tall over a 0.54 m baseline
        wid = max(3, int(round(rng.uniform(2.5, 4.0) * d)))
        u0 = int(rng.uniform(-0.2 * W, 1.1 * W))
        vt = vb - hgt + 1
        rect = (u0, u0 + wid - 1, vt, vb, d)
        r0, r1 = max(0, vt), min(H - 1, vb)
        c0, c1 = max(0, rect[0]), min(W - 1, rect[1])
        if r0 > r1 or c0 > c1:
            continue
        if (r1 - r0 + 1) * (c1 - c0 + 1) > 0.04 * W * H:    # keep single blocks modest
            continue
        obs.append(rect)
        covered += (r1 - r0 + 1) * (c1 - c0 + 1)
    return obs


# ----------------------------------------------------------------------------- configs
def scene_c1(seed: int = 0) -> Scene:
    """320x96 u8 frame: v0=24, b=0.4, f(95)=48, two lanes at s_k=+-1.0, q=2e-3."""
    a = (48.0 - 0.4 * 71.0) / (71.0 ** 2)
    return Scene(width=320, height=96, fmt=FMT_U8, d_max=48, a=a, b=0.4, v0=24.0,
                 c=160.0, p=0.0, q=2e-3, lanes=[(-1.0, False), (1.0, False)])


def make_c1(seed: int = 0, idx: int = 0):
    """Small single frame (320x96, u8 disparity, 5% invalid pixels)."""
    rng = _rng(seed, idx)
    sc = scene_c1(seed)
    grey, disp = _render(sc, rng, disp_noise=0.0, dropout=0.05, dash_k=None)
    return grey, disp, sc


def scaled_c1_scene(width: int, height: int, d_max: int, rng: np.random.Generator | None = None) -> Scene:
    """The small-frame scene scaled to another resolution (used for serving mixes)."""
    v0 = height / 4.0
    span = (height - 1) - v0
    b = 0.4 * (d_max / 48.0) * (96.0 / height)
    a = (d_max - b * span) / span ** 2
    s = 0.15 * width / d_max
    c = width / 2.0
    q = 2e-3 * (96.0 / height) * (width / 320.0)
    if rng is not None:
        c += rng.uniform(-0.05, 0.05) * width
        q *= rng.uniform(-1.0, 1.0)
    return Scene(width=width, height=height, fmt=FMT_U8, d_max=d_max, a=a, b=b, v0=v0,
                 c=c, p=0.0, q=q, lanes=[(-s, False), (s, False)])


def make_scaled_c1(width: int, height: int, d_max: int, seed: int, idx: int):
    rng = _rng(seed, idx)
    sc = scaled_c1_scene(width, height, d_max, rng)
    grey, disp = _render(sc, rng, disp_noise=0.0, dropout=0.05, dash_k=None)
    return grey, disp, sc


def _c2_sequence_params(seed: int):
    rng = _rng(seed, 1 << 40)
    q = rng.uniform(-1e-4, 1e-4)              # curvature 2q within +-2e-4 px^-1
    p = rng.uniform(-0.15, 0.15)
    c0 = 621.0 + rng.uniform(-60.0, 60.0)
    v00 = 170.0 + rng.uniform(-6.0, 6.0)
    # per-frame V_p drift: |delta| <= 2 px per frame (1.4 px per axis)
    steps = rng.uniform(-1.4, 1.4, size=(4096, 2))
    return q, p, c0, v00, steps


def scene_c2(seed: int, idx: int) -> Scene:
    """1242x375 f32 frame idx of sequence `seed`: 4 curved lanes, drifting V_p."""
    q, p, c0, v00, steps = _c2_sequence_params(seed)
    c, v0 = c0, v00
    for i in range(idx):
        c = float(np.clip(c + steps[i, 0], 521.0, 721.0))
        v0 = float(np.clip(v0 + steps[i, 1], 160.0, 180.0))
    span = 374.0 - v0
    b = 0.35
    a = (100.0 - b * 204.0) / (204.0 ** 2)
    del span
    return Scene(width=1242, height=375, fmt=FMT_F32, d_max=128, a=a, b=b, v0=v0,
                 c=c, p=p, q=q, lanes=[(-9.7, False), (-3.2, False), (3.2, False), (9.7, False)])


def make_c2(seed: int = 0, idx: int = 0):
    """1242x375, f32 subpixel disparity (noise sigma 0.2), ~10% obstacle pixels."""
    sc = scene_c2(seed, idx)
    rng = _rng(seed, idx)
    sc.obstacles = _obstacles(sc, rng, 0.10)
    grey, disp = _render(sc, rng, disp_noise=0.2, dropout=0.0, dash_k=None, width_fn=marking_width)
    return grey, disp, sc


def _paint(scene: Scene, rng: np.random.Generator, n: int):
    """Road paint between the two inner lanes: bars across the lane (stop lines, whose edges
    run along the rows) and strokes slanted 45 degrees (arrow heads), each about 0.4 m deep,
    on road rows in the lower two thirds of the road."""
    H = scene.height
    out = []
    v_lo = scene.v0 + (H - 1 - scene.v0) / 3.0
    for i in range(n):
        vb = int(rng.uniform(v_lo, H - 1))
        d = float(scene.f(vb))
        depth = max(2, int(round(0.05 * d)))          # rows a 0.4 m deep patch covers, roughly
        ul = float(scene.lane_u(1, vb)) + 0.25 * d
        ur = float(scene.lane_u(2, vb)) - 0.25 * d
        if ur - ul < 8:
            continue
        if i % 2 == 0:
            out.append((vb - depth + 1, vb, ul, ur, 0.0))
        else:
            w = max(3.0, 0.28 * d)
            mid = 0.5 * (ul + ur)
            ln = int(round(min(0.5 * (ur - ul), 3 * d)))
            out.append((vb - ln + 1, vb, mid - w, mid + w, 1.0 if rng.random() < 0.5 else -1.0))
    return out


def make_hard(kind: str, seed: int = 0, idx: int = 0):
    """Hard cases on the 1242x375 sequences: 'low_contrast' renders the left inner lane at
    road + 35 grey levels and the outer lanes at road + 30 (the right inner lane at 200);
    'markings' adds road paint between the inner lanes (bars across the lane and 45-degree
    strokes, six per frame).  Otherwise as make_c2."""
    sc = scene_c2(seed, idx)
    rng = _rng(seed ^ 0x5A5A, idx)
    sc.obstacles = _obstacles(sc, rng, 0.10)
    if kind == "low_contrast":
        sc.lane_values = [120.0, 125.0, 200.0, 120.0]
    elif kind == "markings":
        sc.paint = _paint(sc, rng, 6)
    else:
        raise ValueError(kind)
    grey, disp = _render(sc, rng, disp_noise=0.2, dropout=0.0, dash_k=None, width_fn=marking_width)
    return grey, disp, sc


def make_stereo(config: str = "c2", seed: int = 0, idx: int = 0):
    """A rectified stereo pair of the road scene: (left grey, right grey, true left disparity
    (float32, 0 above the horizon), scene).  The road texture (asphalt noise and lane markings)
    is drawn on a canvas wider than the frame; the left view is its first `width` columns with
    the obstacle blocks pasted in, the right view samples each road row at u = x + f(v) (linear
    interpolation; rows above the horizon unshifted) and pastes every block shifted left by its
    own, whole-pixel disparity; the right camera adds N(0, 1) sensor noise.  config "c2":
    1242x375 with ~10 % obstacle pixels; "c1": 320x96 without obstacles."""
    if config == "c2":
        sc = scene_c2(seed, idx)
        width_fn, frac = marking_width, 0.10
    elif config == "c1":
        sc = scene_c1(seed)
        width_fn, frac = None, 0.0
    else:
        raise ValueError(config)
    rng = _rng(seed ^ 0x57E5, idx)
    W, H = sc.width, sc.height
    obstacles = _obstacles(sc, rng, frac) if frac > 0 else []
    margin = sc.d_max + 8
    wide = Scene(**{**sc.__dict__, "width": W + margin, "obstacles": [], "paint": []})
    road, _ = _render(wide, rng, disp_noise=0.0, dropout=0.0, dash_k=None, width_fn=width_fn)
    road = road.astype(np.float64)
    left = road[:, :W].copy()
    right = np.empty((H, W))
    xs = np.arange(W, dtype=np.float64)
    cols = np.arange(W + margin, dtype=np.float64)
    gt = np.zeros((H, W), np.float32)
    for v in range(H):
        d = float(sc.f(v)) if v >= sc.v0 else 0.0
        right[v] = np.interp(xs + d, cols, road[v])
        gt[v] = d
    for (u0, u1, vt, vb, _) in obstacles:
        d_o = int(round(float(sc.f(vb))))
        r0, r1 = max(0, vt), min(H - 1, vb)
        if r0 > r1 or d_o < 1:
            continue
        patch = rng.normal(60.0, 4.0, size=(r1 - r0 + 1, u1 - u0 + 1))
        for x0, img in ((u0, left), (u0 - d_o, right)):
            a, b = max(0, x0), min(W - 1, x0 + u1 - u0)
            if a <= b:
                img[r0:r1 + 1, a:b + 1] = patch[:, a - x0:b - x0 + 1]
        a, b = max(0, u0), min(W - 1, u1)
        if a <= b:
            gt[r0:r1 + 1, a:b + 1] = d_o
    right = right + rng.normal(0.0, 1.0, size=right.shape)
    left = np.clip(np.rint(left), 0, 255).astype(np.uint8)
    right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    sc.obstacles = obstacles
    return left, right, gt, sc


def scene_c3(seed: int, idx: int) -> Scene:
    rng = _rng(seed, 1 << 41)
    q = rng.uniform(-6e-5, 6e-5)
    p = rng.uniform(-0.1, 0.1)
    c = 960.0 + rng.uniform(-80.0, 80.0)
    v0 = 490.0
    b = 0.2
    span = 1079.0 - v0
    a = (200.0 - b * span) / span ** 2
    gains = _rng(seed, 1 << 42).uniform(0.5, 1.5, size=4096)
    return Scene(width=1920, height=1080, fmt=FMT_U16Q4, d_max=255, a=a, b=b, v0=v0, c=c, p=p, q=q,
                 lanes=[(-16.2, False), (-9.7, True), (-3.2, True), (3.2, True), (9.7, True), (16.2, False)],
                 gain=float(gains[idx // 50]))


def make_c3(seed: int = 0, idx: int = 0):
    """1920x1080, u16 disparity in 1/16 px, 6 lanes (inner 4 dashed), 15% obstacles, gain jumps."""
    sc = scene_c3(seed, idx)
    rng = _rng(seed, idx)
    sc.obstacles = _obstacles(sc, rng, 0.15)
    grey, disp = _render(sc, rng, disp_noise=0.2, dropout=0.02, dash_k=4000.0, width_fn=marking_width)
    return grey, disp, sc


def make_frame(config: str, seed: int = 0, idx: int = 0):
    if config == "c1":
        return make_c1(seed, idx)
    if config == "c2":
        return make_c2(seed, idx)
    if config == "c3":
        return make_c3(seed, idx)
    if config in ("low_contrast", "markings"):
        return make_hard(config, seed, idx)
    raise ValueError(config)


def make_batch(config: str, seed: int, count: int, start: int = 0):
    """Stack `count` consecutive frames of one sequence: (grey[B,H,W], disp[B,H,W], scenes)."""
    greys, disps, scenes = [], [], []
    for i in range(start, start + count):
        g, d, s = make_frame(config, seed, i)
        greys.append(g)
        disps.append(d)
        scenes.append(s)
    return np.stack(greys), np.stack(disps), scenes


# ----------------------------------------------------------------------------- degenerate frames
def degenerate(kind: str, width: int = 64, height: int = 60, fmt: int = FMT_U8, d_max: int = 32, seed: int = 0):
    """Frames that exercise the method's failure branches (flags, empty sets)."""
    rng = _rng(seed, 99)
    grey = np.clip(np.rint(rng.normal(90, 4, size=(height, width))), 0, 255).astype(np.uint8)
    dt = {FMT_U8: np.uint8, FMT_F32: np.float32, FMT_U16Q4: np.uint16}[fmt]
    if kind == "all_invalid":
        disp = np.zeros((height, width), dt)
    elif kind == "flat_image":
        grey[:] = 90
        sc = scaled_c1_scene(width, height, d_max)
        _, disp = _render(sc, rng, disp_noise=0.0, dropout=0.0, dash_k=None)
        disp = disp.astype(dt) if fmt == FMT_U8 else disp
    elif kind == "obstacle_only":
        disp = np.full((height, width), 7, dt)
    elif kind == "random":
        disp = rng.integers(0, d_max + 1, size=(height, width)).astype(dt)
        grey = rng.integers(0, 256, size=(height, width)).astype(np.uint8)
    else:
        raise ValueError(kind)
    return grey, disp
