"""ctypes binding of the C++ oracle (oracle/ldref.cpp) -- TEST INFRASTRUCTURE ONLY.

Every function here runs the plain FP64 CPU reference of one step of the method, on host
numpy arrays.  See ldref.cpp for the passage of the paper each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldref.cpp")
_SO = os.environ.get("LDREF_SO") or os.path.join(_HERE, "libldref.so")   # LDREF_SO: a sanitizer build


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no contraction, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [
        ("chi", C.c_int32), ("tau_y_max", C.c_int32), ("tau_x_max", C.c_int32),
        ("lambda_y", C.c_int32), ("lambda_x", C.c_int32),
        ("tr_y", C.c_double), ("tr_x", C.c_double),
        ("eps_num", C.c_int32), ("eps_den", C.c_int32),
        ("varpi", C.c_double), ("edge_t", C.c_int32), ("sigma_g", C.c_double),
        ("nu", C.c_int32), ("varsigma", C.c_int32),
        ("n_hyp", C.c_int32), ("max_rounds", C.c_int32),
        ("rho_lpv", C.c_double), ("d_nms", C.c_int32), ("weight_squared", C.c_int32), ("vote", C.c_int32),
        ("seed", C.c_uint64),
    ]


class FitOut(C.Structure):
    _fields_ = [("ok", C.c_int32), ("flags", C.c_int32), ("center", C.c_int32), ("kshift", C.c_int32),
                ("rounds", C.c_int32), ("n_survivors", C.c_int32),
                ("coef", C.c_double * 5), ("raw", C.c_double * 5)]


_P32 = C.POINTER(C.c_int32)
_PD = C.POINTER(C.c_double)
_P64 = C.POINTER(C.c_int64)
_PF = C.POINTER(C.c_float)


class Out(C.Structure):
    _fields_ = [
        ("flags", C.c_int32), ("v_h", C.c_int32), ("v_end", C.c_int32), ("n_lanes", C.c_int32),
        ("n_my", C.c_int32), ("n_edges", C.c_int32), ("n_votes", C.c_int32), ("pad0", C.c_int32),
        ("u_start", C.c_int32 * 16), ("energy_lane", C.c_double * 16),
        ("beta", FitOut), ("gamma", FitOut),
        ("m_y", _P32), ("my_path_v", _P32), ("my_x", _P32), ("my_y", _P32),
        ("f", _PD), ("fp", _PD), ("vpy", _PD), ("vpx", _PD),
        ("edge_u", _P32), ("edge_v", _P32), ("edge_gx", _P32), ("edge_gy", _P32), ("edge_bin", _P32),
        ("edge_q", _PD), ("edge_cap", C.c_int32), ("pad1", C.c_int32),
        ("mx_path", _P32), ("energy", _PD), ("m1", _PD), ("curves", _PD),
        ("trace_beta", _P32), ("trace_gamma", _P32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        L.ldref_params_default.argtypes = [C.POINTER(Params)]
        L.ldref_philox.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.ldref_vdisp_hist.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, _P32]
        L.ldref_vdisp_dp.argtypes = [_P32, C.c_int, C.c_int, C.c_int, C.c_int, _P32, _P32, _P32, _P32]
        L.ldref_fit.argtypes = [_P32, _P32, _P32, C.c_int, C.c_int, C.c_int32, C.c_int32, _PD]
        L.ldref_ransac.argtypes = [_P32, _P32, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_uint64, C.c_uint64, C.c_int64, C.c_int, _PD, C.POINTER(FitOut), _P32]
        L.ldref_road_tables.argtypes = [C.POINTER(FitOut), C.c_int, _PD, _PD, _PD, _P32]
        L.ldref_sobel.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, _P32, _P32]
        L.ldref_track_update.argtypes = [C.POINTER(TrackState), _P32, C.c_int, C.c_int, C.c_double, C.c_double,
                                         C.c_double, C.c_int]
        L.ldref_stereo.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, _PD]
        L.ldref_stereo_stats.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, _P64, _P64]
        L.ldref_bilateral.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_float, C.c_float,
                                      C.c_int, C.c_void_p, C.c_int64, _PF]
        L.ldref_sample.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, _P32]
        L.ldref_road_edges.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, _PD,
                                       C.c_int, C.c_double, C.c_int, _P32, _P32, _P32, _P32, C.c_int]
        L.ldref_votes.argtypes = [_P32, _P32, _P32, _P32, C.c_int, _PD, C.c_int, _P32]
        L.ldref_band.argtypes = [_P32, C.c_int, C.c_int, C.c_int, C.c_int, _P64]
        L.ldref_row_dp.argtypes = [_P64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _P32]
        L.ldref_weights.argtypes = [_P32, _P32, _P32, _P32, C.c_int, _PD, _PD, C.c_double, C.c_int, _PD, C.c_int]
        L.ldref_m0m1.argtypes = [_PD, C.c_int, C.c_int, C.c_int, C.c_int, _PD, _PD]
        L.ldref_energy.argtypes = [_PD, _PD, _PD, C.c_int, C.c_int, C.c_int, _PD, _PD, _P32, C.c_int]
        L.ldref_peaks.argtypes = [_PD, C.c_int, C.c_int, C.c_double, C.c_int, _P32, _PD]
        L.ldref_band_top.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.ldref_seed.argtypes = [_P32, _P32, _P32, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 _P32, _P32, _P32]
        L.ldref_window_dp.argtypes = [_P64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _P32]
        L.ldref_track_affine.argtypes = [_PD, _PD, C.c_int, C.c_int, C.c_int, _PD, _PD]
        L.ldref_cand_mask.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _PD, _PD,
                                      C.c_void_p, C.c_void_p]
        L.ldref_detect.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.POINTER(Params), C.c_uint64, C.c_int64, _PD, C.POINTER(Out)]
        L.ldref_detect_pruned.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int,
                                          C.c_int, C.POINTER(Params), C.c_uint64, C.c_int64, _PD, C.POINTER(Learned),
                                          C.POINTER(Out)]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(_P32)


def _pd(a):
    return a.ctypes.data_as(_PD)


def default_params(**kw) -> Params:
    p = Params()
    lib().ldref_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def philox(counter, key):
    ctr = (C.c_uint64 * 4)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in counter])
    k = (C.c_uint64 * 2)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in key])
    out = (C.c_uint64 * 4)()
    lib().ldref_philox(ctr, k, out)
    return [int(x) for x in out]


def _fmt_of(disp: np.ndarray) -> int:
    return {np.dtype(np.uint8): 0, np.dtype(np.float32): 1, np.dtype(np.uint16): 2}[disp.dtype]


def vdisp_hist(disp: np.ndarray, d_max: int) -> np.ndarray:
    disp = np.ascontiguousarray(disp)
    H, W = disp.shape
    out = np.zeros((H, d_max + 1), np.int32)
    lib().ldref_vdisp_hist(disp.ctypes.data, disp.strides[0], W, H, _fmt_of(disp), d_max, _p32(out))
    return out


def vdisp_dp(m_y: np.ndarray, tau_max: int = 6, lam: int = 1):
    m_y = np.ascontiguousarray(m_y, dtype=np.int32)
    H, D1 = m_y.shape
    path_v = np.zeros(D1, np.int32)
    px = np.zeros(D1, np.int32)
    py = np.zeros(D1, np.int32)
    n = np.zeros(1, np.int32)
    lib().ldref_vdisp_dp(_p32(m_y), H, D1 - 1, tau_max, lam, _p32(path_v), _p32(px), _p32(py), _p32(n))
    k = int(n[0])
    return path_v, px[:k].copy(), py[:k].copy()


def fit(x, y, degree: int, center: int, kshift: int, idx=None):
    x = np.ascontiguousarray(x, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    coef = np.zeros(degree + 1, np.float64)
    if idx is None:
        rc = lib().ldref_fit(_p32(x), _p32(y), None, len(x), degree, center, kshift, _pd(coef))
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        rc = lib().ldref_fit(_p32(x), _p32(y), _p32(idx), len(idx), degree, center, kshift, _pd(coef))
    return rc, coef


def ransac(x, y, degree: int, tr: float, *, n_hyp=64, max_rounds=16, eps=(99, 100), seed=0, stream_id=0,
           frame_idx=0, stage=0, seed_raw=None):
    x = np.ascontiguousarray(x, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    out = FitOut()
    trace = np.full(3 * max_rounds, -9, np.int32)
    sr = None
    if seed_raw is not None:
        sr = np.ascontiguousarray(seed_raw, dtype=np.float64)
    lib().ldref_ransac(_p32(x), _p32(y), len(x), degree, tr, n_hyp, max_rounds, eps[0], eps[1], seed, stream_id,
                       frame_idx, stage, _pd(sr) if sr is not None else None, C.byref(out), _p32(trace))
    return out, trace.reshape(max_rounds, 3)[: out.rounds]


def sample(n_cur: int, s: int, *, seed=0, stream_id=0, frame_idx=0, stage=0, rnd=0, hyp=0):
    pick = np.zeros(5, np.int32)
    got = lib().ldref_sample(n_cur, s, seed, stream_id, frame_idx, stage, rnd, hyp, _p32(pick))
    return pick[:got].copy()


def road_edges(grey, disp, f, v_h: int, varpi=3.0, edge_t=100):
    grey = np.ascontiguousarray(grey, dtype=np.uint8)
    disp = np.ascontiguousarray(disp)
    H, W = grey.shape
    cap = H * W
    arrs = [np.zeros(cap, np.int32) for _ in range(4)]
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = lib().ldref_road_edges(grey.ctypes.data, grey.strides[0], disp.ctypes.data, disp.strides[0], W, H,
                               _fmt_of(disp), _pd(f), v_h, varpi, edge_t, *[_p32(a) for a in arrs], cap)
    return [a[:n].copy() for a in arrs]


def votes(eu, ev, egx, egy, vpy, W: int):
    eu, ev, egx, egy = [np.ascontiguousarray(a, dtype=np.int32) for a in (eu, ev, egx, egy)]
    vpy = np.ascontiguousarray(vpy, dtype=np.float64)
    b = np.zeros(len(eu), np.int32)
    lib().ldref_votes(_p32(eu), _p32(ev), _p32(egx), _p32(egy), len(eu), _pd(vpy), W, _p32(b))
    return b


def band(h, v_h: int, chi: int = 25):
    h = np.ascontiguousarray(h, dtype=np.int32)
    H, W2 = h.shape
    mx = np.zeros((H, W2), np.int64)
    lib().ldref_band(_p32(h), H, W2, v_h, chi, mx.ctypes.data_as(C.POINTER(C.c_int64)))
    return mx


def row_dp(mx, v_h: int, tau_max: int = 5, lam: int = 1):
    mx = np.ascontiguousarray(mx, dtype=np.int64)
    H, W2 = mx.shape
    cpath = np.full(H, -1, np.int32)
    lib().ldref_row_dp(mx.ctypes.data_as(C.POINTER(C.c_int64)), H, W2, v_h, tau_max, lam, _p32(cpath))
    return cpath


def band_top(v_h: int, H: int, n_bands: int, k: int) -> int:
    return int(lib().ldref_band_top(v_h, H, n_bands, k))


def seed(eu, ev, ebin, lane_bits, W: int, H: int, v_h: int, n_bands=1, min_votes=8):
    """Seed of the narrowed search: (c_s or -1, est[4], cnt[4], pooled votes)."""
    eu, ev, ebin = [np.ascontiguousarray(a, dtype=np.int32) for a in (eu, ev, ebin)]
    bits = np.ascontiguousarray(lane_bits, dtype=np.uint8).reshape(4, 16, W)
    est = np.zeros(4, np.int32)
    cnt = np.zeros(4, np.int32)
    tot = np.zeros(1, np.int32)
    cs = lib().ldref_seed(_p32(eu), _p32(ev), _p32(ebin), len(eu), bits.ctypes.data, W, H, v_h, n_bands, min_votes,
                          _p32(est), _p32(cnt), _p32(tot))
    return int(cs), est, cnt, int(tot[0])


def window_dp(mx, v_h: int, lo: int, hi: int, tau_max: int = 5, lam: int = 1):
    """Row DP restricted to columns lo..hi: (path columns, touched an inner window edge)."""
    mx = np.ascontiguousarray(mx, dtype=np.int64)
    H, W2 = mx.shape
    cpath = np.full(H, -1, np.int32)
    touch = lib().ldref_window_dp(mx.ctypes.data_as(C.POINTER(C.c_int64)), H, W2, v_h, tau_max, lam, lo, hi,
                                  _p32(cpath))
    return cpath, bool(touch)


def track_affine(vpx, vpy, v_end: int, v_lo: int):
    """Per-row (a_v, b_v) of the track u_v = fma(a_v, u_start, b_v); NaN outside the rows written."""
    vpx = np.ascontiguousarray(vpx, dtype=np.float64)
    vpy = np.ascontiguousarray(vpy, dtype=np.float64)
    H = len(vpx)
    a = np.full(H, np.nan)
    b = np.full(H, np.nan)
    lib().ldref_track_affine(_pd(vpx), _pd(vpy), H, v_end, v_lo, _pd(a), _pd(b))
    return a, b


def cand_mask(lane_bits, W: int, v_h: int, v_end: int, vpx, vpy, n_bands=1, dilate=0):
    """(hit, keep, kept) of the narrowed search's candidate mask."""
    bits = np.ascontiguousarray(lane_bits, dtype=np.uint8).reshape(4, 16, W)
    vpx = np.ascontiguousarray(vpx, dtype=np.float64)
    vpy = np.ascontiguousarray(vpy, dtype=np.float64)
    H = len(vpx)
    hit = np.zeros(2 * W, np.uint8)
    keep = np.zeros(2 * W, np.uint8)
    kept = lib().ldref_cand_mask(bits.ctypes.data, W, H, v_h, v_end, n_bands, dilate, _pd(vpx), _pd(vpy),
                                 hit.ctypes.data, keep.ctypes.data)
    return hit, keep, int(kept)


def weights(eu, ev, egx, egy, vpx, vpy, sigma_g=3.5, squared=0, vote=0):
    """q per edge: G_x w_g (vote 0) or the prior work's vote |grad| cos(theta_e - theta_Vp) (vote 1)."""
    eu, ev, egx, egy = [np.ascontiguousarray(a, dtype=np.int32) for a in (eu, ev, egx, egy)]
    vpx = np.ascontiguousarray(vpx, dtype=np.float64)
    vpy = np.ascontiguousarray(vpy, dtype=np.float64)
    q = np.zeros(len(eu))
    lib().ldref_weights(_p32(eu), _p32(ev), _p32(egx), _p32(egy), len(eu), _pd(vpx), _pd(vpy), sigma_g, squared,
                        _pd(q), int(vote))
    return q


def m0m1(q, nu=1, varsigma=3):
    q = np.ascontiguousarray(q, dtype=np.float64)
    H, W = q.shape
    m0 = np.zeros((H, W))
    m1 = np.zeros((H, W))
    lib().ldref_m0m1(_pd(q), W, H, nu, varsigma, _pd(m0), _pd(m1))
    return m0, m1


def energy(m1, vpx, vpy, v_h: int, tracks=None):
    m1 = np.ascontiguousarray(m1, dtype=np.float64)
    H, W = m1.shape
    vpx = np.ascontiguousarray(vpx, dtype=np.float64)
    vpy = np.ascontiguousarray(vpy, dtype=np.float64)
    E = np.zeros(2 * W)
    curves = None
    if tracks is not None:
        tracks = np.ascontiguousarray(tracks, dtype=np.int32)
        curves = np.zeros((len(tracks), H))
    v_end = lib().ldref_energy(_pd(m1), _pd(vpx), _pd(vpy), W, H, v_h, _pd(E),
                               _pd(curves) if curves is not None else None,
                               _p32(tracks) if tracks is not None else None, 0 if tracks is None else len(tracks))
    return E, v_end, curves


def peaks(E, W: int, rho=0.25, d_nms=None):
    E = np.ascontiguousarray(E, dtype=np.float64)
    if d_nms is None:
        d_nms = max(8, W // 64)
    us = np.zeros(16, np.int32)
    el = np.zeros(16)
    n = lib().ldref_peaks(_pd(E), len(E), W // 2, rho, d_nms, _p32(us), _pd(el))
    return us[:n].copy(), el[:n].copy()


def road_tables(beta: FitOut, H: int):
    f = np.zeros(H)
    fp = np.zeros(H)
    vpy = np.zeros(H)
    vh = np.zeros(1, np.int32)
    lib().ldref_road_tables(C.byref(beta), H, _pd(f), _pd(fp), _pd(vpy), _p32(vh))
    return f, fp, vpy, int(vh[0])


def sobel(grey: np.ndarray):
    grey = np.ascontiguousarray(grey, dtype=np.uint8)
    H, W = grey.shape
    gx = np.zeros((H, W), np.int32)
    gy = np.zeros((H, W), np.int32)
    lib().ldref_sobel(grey.ctypes.data, grey.strides[0], W, H, _p32(gx), _p32(gy))
    return gx, gy


def stereo(left: np.ndarray, right: np.ndarray, d_max: int = 128, rho: int = 3, tau: int = 1, tr_lrc: int = 3):
    """Disparity maps of a rectified pair (Sec. 2.1): (checked map, left map, right map, left
    costs), u8 maps with 0 for no match."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    assert left.shape == right.shape
    H, W = left.shape
    lf, rt, out = (np.zeros((H, W), np.uint8) for _ in range(3))
    cost = np.zeros((H, W))
    rc = lib().ldref_stereo(left.ctypes.data, right.ctypes.data, W, W, H, rho, d_max, tau, tr_lrc, lf.ctypes.data,
                            rt.ctypes.data, out.ctypes.data, _pd(cost))
    if rc != 0:
        raise ValueError("stereo: invalid arguments")
    return out, lf, rt, cost


def stereo_stats(img: np.ndarray, rho: int = 3):
    """Block sums S and sums of squares Q from the integral images (0 off the matchable centres)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    S = np.zeros((H, W), np.int64)
    Q = np.zeros((H, W), np.int64)
    if lib().ldref_stereo_stats(img.ctypes.data, W, W, H, rho, S.ctypes.data_as(_P64), Q.ctypes.data_as(_P64)) != 0:
        raise ValueError("stereo_stats: invalid arguments")
    return S, Q


class TrackState(C.Structure):
    """Tracker state of one stream (zero-filled: no tracks)."""
    _fields_ = [("n", C.c_int32), ("next_id", C.c_int32), ("frames", C.c_int64),
                ("id", C.c_int32 * 16), ("hits", C.c_int32 * 16), ("misses", C.c_int32 * 16),
                ("x", C.c_double * 16), ("dx", C.c_double * 16)]

    def tracks(self, confirm: int = 1):
        """[(id, x, dx, hits, misses)] of the tracks with hits >= confirm, in slot order."""
        return [(self.id[t], self.x[t], self.dx[t], self.hits[t], self.misses[t]) for t in range(self.n)
                if self.hits[t] >= confirm]


def track_update(state: TrackState, u_start, valid: bool = True, alpha: float = 0.5, beta: float = 0.1,
                 gate: float = 24.0, max_misses: int = 5) -> TrackState:
    """Fold one frame's lane start columns into a stream's tracks (in place)."""
    u = np.ascontiguousarray(np.asarray(u_start, dtype=np.int32)[:16])
    lib().ldref_track_update(C.byref(state), _p32(u) if len(u) else None, len(u), 1 if valid else 0,
                             alpha, beta, gate, max_misses)
    return state


def bilateral(grey: np.ndarray, rho: int = 5, sigma_s: float = 300.0, sigma_r: float = 0.3, row0: int = 0):
    """Bilateral pre-filter (Sec. 2.3.1, Eq. bilateral_filter): the u8 image and the float
    quotients (rows below row0: 0 in both).  sigma_s and sigma_r are taken as float32."""
    grey = np.ascontiguousarray(grey, dtype=np.uint8)
    H, W = grey.shape
    out = np.zeros((H, W), np.uint8)
    val = np.zeros((H, W), np.float32)
    rc = lib().ldref_bilateral(grey.ctypes.data, grey.strides[0], W, H, int(rho), float(np.float32(sigma_s)),
                               float(np.float32(sigma_r)), int(row0), out.ctypes.data, W,
                               val.ctypes.data_as(_PF))
    if rc != 0:
        raise ValueError("bilateral: invalid arguments")
    return out, val


class Result:
    """Plain container for everything ldref_detect reports about one frame."""


class Learned(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("delta_x", C.c_int32), ("dilate", C.c_int32), ("min_votes", C.c_int32),
                ("seed_ransac", C.c_int32), ("pad", C.c_int32),
                ("lane_bits", C.c_void_p), ("prune", C.c_int32 * 16), ("cand_mask", C.c_void_p)]


def detect_pruned(grey: np.ndarray, disp: np.ndarray, d_max: int, lane_bits: np.ndarray, *, n_bands=1, delta_x=127,
                  dilate=-1, min_votes=8, seed_ransac=0, params: Params | None = None, stream_id=0, frame_idx=0,
                  seed_gamma=None, want_m1=False):
    """The narrowed search given the network's band decisions lane_bits (4 x 16 x W u8):
    everything detect() reports plus .prune (16 int32) and .cand_mask (2W u8).  seed_gamma
    (raw-basis quartic, NaN first coefficient: none) is RANSAC hypothesis 0 of V_px whenever the
    narrowed search itself gives none (seed_ransac off, or a fallback frame)."""
    H, W = np.asarray(grey).shape
    bits = np.ascontiguousarray(lane_bits, dtype=np.uint8).reshape(4, 16, W)
    L = Learned()
    L.n_bands, L.delta_x, L.dilate, L.min_votes, L.seed_ransac = n_bands, delta_x, dilate, min_votes, seed_ransac
    L.lane_bits = bits.ctypes.data
    mask = np.zeros(2 * W, np.uint8)
    L.cand_mask = mask.ctypes.data
    r = detect(grey, disp, d_max, params, stream_id=stream_id, frame_idx=frame_idx, seed_gamma=seed_gamma,
               want_m1=want_m1, _learned=L)
    r.prune = np.array(L.prune[:], np.int32)
    r.cand_mask = mask
    return r


def detect(grey: np.ndarray, disp: np.ndarray, d_max: int, params: Params | None = None, *, stream_id=0,
           frame_idx=0, seed_gamma=None, want_m1=False, edge_cap=None, _learned=None):
    grey = np.ascontiguousarray(grey, dtype=np.uint8)
    disp = np.ascontiguousarray(disp)
    H, W = grey.shape
    if params is None:
        params = default_params()
    D1 = d_max + 1
    cap = edge_cap if edge_cap is not None else H * W
    r = Result()
    r.m_y = np.zeros((H, D1), np.int32)
    r.my_path_v = np.zeros(D1, np.int32)
    r.my_x = np.zeros(D1, np.int32)
    r.my_y = np.zeros(D1, np.int32)
    r.f = np.zeros(H)
    r.fp = np.zeros(H)
    r.vpy = np.zeros(H)
    r.vpx = np.zeros(H)
    r.edge_u = np.zeros(cap, np.int32)
    r.edge_v = np.zeros(cap, np.int32)
    r.edge_gx = np.zeros(cap, np.int32)
    r.edge_gy = np.zeros(cap, np.int32)
    r.edge_bin = np.zeros(cap, np.int32)
    r.edge_q = np.zeros(cap)
    r.mx_path = np.zeros(H, np.int32)
    r.energy = np.zeros(2 * W)
    r.m1 = np.zeros((H, W)) if want_m1 else None
    r.curves = np.zeros((16, H))
    r.trace_beta = np.full((params.max_rounds, 3), -9, np.int32)
    r.trace_gamma = np.full((params.max_rounds, 3), -9, np.int32)
    o = Out()
    o.m_y = _p32(r.m_y); o.my_path_v = _p32(r.my_path_v); o.my_x = _p32(r.my_x); o.my_y = _p32(r.my_y)
    o.f = _pd(r.f); o.fp = _pd(r.fp); o.vpy = _pd(r.vpy); o.vpx = _pd(r.vpx)
    o.edge_u = _p32(r.edge_u); o.edge_v = _p32(r.edge_v); o.edge_gx = _p32(r.edge_gx); o.edge_gy = _p32(r.edge_gy)
    o.edge_bin = _p32(r.edge_bin); o.edge_q = _pd(r.edge_q); o.edge_cap = cap
    o.mx_path = _p32(r.mx_path); o.energy = _pd(r.energy)
    o.m1 = _pd(r.m1) if want_m1 else None
    o.curves = _pd(r.curves)
    o.trace_beta = _p32(r.trace_beta); o.trace_gamma = _p32(r.trace_gamma)
    sg = None
    if seed_gamma is not None:
        sg = np.ascontiguousarray(seed_gamma, dtype=np.float64)
    fmt = _fmt_of(disp)
    if _learned is None:
        lib().ldref_detect(grey.ctypes.data, grey.strides[0], disp.ctypes.data, disp.strides[0], W, H, fmt, d_max,
                           C.byref(params), stream_id, frame_idx, _pd(sg) if sg is not None else None, C.byref(o))
    else:
        lib().ldref_detect_pruned(grey.ctypes.data, grey.strides[0], disp.ctypes.data, disp.strides[0], W, H, fmt,
                                  d_max, C.byref(params), stream_id, frame_idx, _pd(sg) if sg is not None else None,
                                  C.byref(_learned), C.byref(o))
    r.flags, r.v_h, r.v_end, r.n_lanes = o.flags, o.v_h, o.v_end, o.n_lanes
    r.n_my, r.n_edges, r.n_votes = o.n_my, o.n_edges, o.n_votes
    r.my_x = r.my_x[: o.n_my]
    r.my_y = r.my_y[: o.n_my]
    n = min(o.n_edges, cap)
    for nm in ("edge_u", "edge_v", "edge_gx", "edge_gy", "edge_bin", "edge_q"):
        setattr(r, nm, getattr(r, nm)[:n].copy())
    r.u_start = np.array(o.u_start[: o.n_lanes], np.int32)
    r.energy_lane = np.array(o.energy_lane[: o.n_lanes])
    r.curves = r.curves[: o.n_lanes]
    r.beta = o.beta
    r.gamma = o.gamma
    r.trace_beta = r.trace_beta[: o.beta.rounds]
    r.trace_gamma = r.trace_gamma[: o.gamma.rounds]
    return r
