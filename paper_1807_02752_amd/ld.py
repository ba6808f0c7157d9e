"""Python binding of libld.so (include/ld.h): argument marshalling only.

Every step of the lane-detection path runs in the library's HIP kernels.  PyTorch only
provides device memory and streams: tensors are passed by data_ptr() and the current
torch stream's handle.  If the library has not been built, importing works but every call
raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libld.so")

LD_OK, LD_E_INVAL, LD_E_NOMEM, LD_E_HIP, LD_E_STATE, LD_E_BUSY = 0, -1, -2, -3, -4, -5
LD_MAX_CLASSES = 4
LD_DISP_U8, LD_DISP_F32, LD_DISP_U16Q4 = 0, 1, 2
LD_FLAG_NOROAD, LD_FLAG_NOVP, LD_FLAG_NOCONS_Y, LD_FLAG_NOCONS_X, LD_FLAG_FALLBACK = 1, 2, 4, 8, 16
LD_MAX_LANES = 16
(LD_STATE_INFO, LD_STATE_MY_PATH, LD_STATE_BETA, LD_STATE_GAMMA, LD_STATE_TABLES, LD_STATE_ROWCOUNT,
 LD_STATE_EDGES, LD_STATE_MX_PATH, LD_STATE_ENERGY, LD_STATE_TRACE, LD_STATE_LANE_BITS, LD_STATE_PRUNE,
 LD_STATE_CAND_MASK) = range(13)
LD_CNN_PARAMS = 3057
MAX_ROUNDS_STORED = 64


class ld_params(C.Structure):
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


class ld_lanes(C.Structure):
    _fields_ = [("n", C.c_int32), ("flags", C.c_int32), ("v_h", C.c_int32), ("v_end", C.c_int32),
                ("u_start", C.c_int32 * LD_MAX_LANES), ("energy", C.c_float * LD_MAX_LANES)]


class ld_fit(C.Structure):
    _fields_ = [("ok", C.c_int32), ("flags", C.c_int32), ("center", C.c_int32), ("kshift", C.c_int32),
                ("rounds", C.c_int32), ("n_survivors", C.c_int32),
                ("coef", C.c_double * 5), ("raw", C.c_double * 5)]


class ld_cnn_config(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("theta", C.c_float), ("delta_x", C.c_int32), ("dilate", C.c_int32),
                ("min_votes", C.c_int32), ("max_batch", C.c_int32), ("max_width", C.c_int32),
                ("seed_ransac", C.c_int32)]


class ld_server_config(C.Structure):
    _fields_ = [("n_classes", C.c_int32), ("width", C.c_int32 * LD_MAX_CLASSES), ("height", C.c_int32 * LD_MAX_CLASSES),
                ("fmt", C.c_int32 * LD_MAX_CLASSES), ("d_max", C.c_int32 * LD_MAX_CLASSES),
                ("max_batch", C.c_int32 * LD_MAX_CLASSES), ("n_streams", C.c_int32), ("inflight", C.c_int32),
                ("max_queue", C.c_int32), ("use_graphs", C.c_int32), ("seed_from_state", C.c_int32),
                ("track", C.c_int32), ("hbm_budget", C.c_int64), ("cnn", C.c_void_p)]


class ld_server_result(C.Structure):
    _fields_ = [("request", C.c_int64), ("stream_id", C.c_int32), ("cls", C.c_int32), ("frame_idx", C.c_int64),
                ("t_submit", C.c_double), ("t_done", C.c_double), ("lanes", ld_lanes)]


LANES_DTYPE = np.dtype([("n", "<i4"), ("flags", "<i4"), ("v_h", "<i4"), ("v_end", "<i4"),
                        ("u_start", "<i4", (LD_MAX_LANES,)), ("energy", "<f4", (LD_MAX_LANES,))])
EDGE_DTYPE = np.dtype([("u", "<i2"), ("gx", "<i2"), ("gy", "<i2"), ("bin", "<i2")])
FIT_DTYPE = np.dtype([("ok", "<i4"), ("flags", "<i4"), ("center", "<i4"), ("kshift", "<i4"),
                      ("rounds", "<i4"), ("n_survivors", "<i4"), ("coef", "<f8", (5,)), ("raw", "<f8", (5,))])
assert LANES_DTYPE.itemsize == C.sizeof(ld_lanes)
assert FIT_DTYPE.itemsize == C.sizeof(ld_fit)

_lib = None


class LdError(RuntimeError):
    pass


def lib():
    """Load libld.so; raise if it is missing (there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LdError(f"libld.so not built ({LIB_PATH}); run paper_1807_02752_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ld_params_default.argtypes = [C.POINTER(ld_params)]
        L.ld_params_default.restype = None
        L.ld_frame_create.argtypes = [i32, i32, i32, i32, i32, C.POINTER(ld_params), C.POINTER(vp)]
        L.ld_frame_destroy.argtypes = [vp]
        L.ld_frame_set_active.argtypes = [vp, i32]
        L.ld_vdisp.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.ld_vp_ransac.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp]
        L.ld_lane_energy.argtypes = [vp, vp, vp, vp]
        L.ld_peaks.argtypes = [vp, vp, vp, vp]
        L.ld_detect.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp]
        L.ld_sync.argtypes = [vp]
        L.ld_status_string.argtypes = [i32]
        L.ld_status_string.restype = C.c_char_p
        L.ld_frame_read.argtypes = [vp, i32, i32, vp, i64, vp]
        L.ld_frame_profile.argtypes = [vp, i32]
        L.ld_server_create.argtypes = [C.POINTER(ld_server_config), C.POINTER(ld_params), C.POINTER(vp)]
        L.ld_server_destroy.argtypes = [vp]
        L.ld_server_submit.argtypes = [vp, i32, i32, vp, i64, vp, i64, C.POINTER(C.c_int64)]
        L.ld_server_poll.argtypes = [vp, C.POINTER(ld_server_result), i32, C.POINTER(C.c_int32)]
        L.ld_server_pending.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.ld_server_engines.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.ld_frame_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), i32]
        L.ld_cnn_config_default.argtypes = [C.POINTER(ld_cnn_config)]
        L.ld_cnn_config_default.restype = None
        fp = C.POINTER(C.c_float)
        L.ld_cnn_create.argtypes = [C.POINTER(ld_cnn_config), fp, C.POINTER(vp)]
        L.ld_cnn_destroy.argtypes = [vp]
        L.ld_cnn_set_params.argtypes = [vp, fp]
        L.ld_cnn_get_params.argtypes = [vp, fp]
        L.ld_cnn_forward.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
        L.ld_cnn_labels.argtypes = [vp, vp, vp, vp, C.c_float, C.c_float, vp, vp]
        L.ld_cnn_train_step.argtypes = [vp, vp, vp, i64, vp, i64, vp, C.c_float, C.c_float, C.c_float, vp, vp, vp]
        L.ld_detect_pruned.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp]
        L.ld_cnn_save.argtypes = [vp, C.c_char_p]
        L.ld_cnn_load.argtypes = [C.c_char_p, C.POINTER(ld_cnn_config), C.POINTER(vp)]
        L.ld_cnn_save.restype = i32
        L.ld_cnn_load.restype = i32
        L.ld_detect_noalloc.argtypes = [i32, i32, i32, i32, i32, C.POINTER(ld_params), vp, i64, vp, i64, vp, vp,
                                        vp, vp, vp]
        L.ld_detect_noalloc.restype = i32
        L.ld_bilateral.argtypes = [vp, vp, i64, vp, i64, i32, C.c_float, C.c_float, i32, vp]
        L.ld_bilateral.restype = i32
        L.ld_track_params_default.argtypes = [C.POINTER(ld_track_params)]
        L.ld_track_params_default.restype = None
        L.ld_track.argtypes = [vp, vp, vp, vp, C.POINTER(ld_track_params), vp]
        L.ld_track.restype = i32
        L.ld_stereo.argtypes = [vp, vp, i64, vp, i64, i32, i32, i32, vp, i64, vp, vp, vp]
        L.ld_stereo.restype = i32
        L.ld_server_tracks.argtypes = [vp, i32, vp]
        L.ld_server_tracks.restype = i32
        for name in ("ld_cnn_create", "ld_cnn_destroy", "ld_cnn_set_params", "ld_cnn_get_params", "ld_cnn_forward",
                     "ld_cnn_labels", "ld_cnn_train_step", "ld_detect_pruned"):
            getattr(L, name).restype = i32
        for name in ("ld_server_create", "ld_server_destroy", "ld_server_submit", "ld_server_poll",
                     "ld_server_pending", "ld_server_engines", "ld_frame_profile", "ld_frame_kernel_times", "ld_frame_create", "ld_frame_destroy", "ld_frame_set_active", "ld_vdisp", "ld_vp_ransac",
                     "ld_lane_energy", "ld_peaks", "ld_detect", "ld_sync", "ld_frame_read"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


EXPORTED = ["ld_params_default", "ld_frame_create", "ld_frame_destroy", "ld_frame_set_active", "ld_vdisp",
            "ld_vp_ransac", "ld_lane_energy", "ld_peaks", "ld_detect", "ld_sync", "ld_status_string",
            "ld_frame_read", "ld_frame_profile", "ld_frame_kernel_times", "ld_server_create", "ld_server_destroy",
            "ld_server_submit", "ld_server_poll", "ld_server_pending", "ld_server_engines",
            "ld_cnn_config_default", "ld_cnn_create", "ld_cnn_destroy", "ld_cnn_set_params", "ld_cnn_get_params",
            "ld_cnn_forward", "ld_cnn_labels", "ld_cnn_train_step", "ld_detect_pruned", "ld_detect_noalloc",
            "ld_cnn_save", "ld_cnn_load", "ld_bilateral", "ld_track_params_default", "ld_track",
            "ld_server_tracks", "ld_stereo"]
KERNELS = ["k_vdisp_hist", "k_vdisp_fit", "k_edges", "k_vpx_fit", "k_energy", "k_peaks", "k_cnn_fwd", "k_seed",
           "k_vpx_window", "k_cand_mask", "k_vpx_ransac"]


def check(status: int, what: str = "ld call"):
    if status != LD_OK:
        msg = lib().ld_status_string(status).decode()
        raise LdError(f"{what} failed: {msg} ({status})")


def params_default(**overrides) -> ld_params:
    p = ld_params()
    lib().ld_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------------------- raw C-ABI names
def ld_params_default(p: ld_params) -> None:
    lib().ld_params_default(C.byref(p))


def ld_frame_create(width, height, batch, fmt, d_max, params=None):
    h = C.c_void_p()
    st = lib().ld_frame_create(width, height, batch, fmt, d_max, C.byref(params) if params is not None else None,
                               C.byref(h))
    return st, h


def ld_frame_destroy(f):
    return lib().ld_frame_destroy(f)


def ld_frame_set_active(f, n):
    return lib().ld_frame_set_active(f, n)


def ld_vdisp(f, disp, disp_pitch, stream_ids, frame_idx, vdisp_out, beta_out, stream):
    return lib().ld_vdisp(f, disp, disp_pitch, stream_ids, frame_idx, vdisp_out, beta_out, stream)


def ld_vp_ransac(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, seed_gamma, vp_out, stream):
    return lib().ld_vp_ransac(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, seed_gamma, vp_out,
                              stream)


def ld_lane_energy(f, cand_mask, energy_out, stream):
    return lib().ld_lane_energy(f, cand_mask, energy_out, stream)


def ld_peaks(f, lanes_out, curves_out, stream):
    return lib().ld_peaks(f, lanes_out, curves_out, stream)


def ld_detect(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, lanes_out, curves_out, stream):
    return lib().ld_detect(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, lanes_out, curves_out,
                           stream)


def ld_detect_noalloc(width, height, batch, fmt, d_max, params, grey, grey_pitch, disp, disp_pitch, stream_ids,
                      frame_idx, lanes_out, curves_out, stream):
    return lib().ld_detect_noalloc(width, height, batch, fmt, d_max,
                                   C.byref(params) if params is not None else None, grey, grey_pitch, disp,
                                   disp_pitch, stream_ids, frame_idx, lanes_out, curves_out, stream)


LD_NOALLOC_SCRATCH_BYTES = 64 << 20


class ld_track_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("gate", C.c_double), ("confirm", C.c_int32),
                ("max_misses", C.c_int32)]


# ld_track_state as a numpy record (device arrays of it are uint8 tensors of TRACK_STATE_BYTES each)
TRACK_DTYPE = np.dtype([("n", np.int32), ("next_id", np.int32), ("frames", np.int64), ("id", np.int32, 16),
                        ("hits", np.int32, 16), ("misses", np.int32, 16), ("x", np.float64, 16),
                        ("dx", np.float64, 16)], align=True)
TRACK_STATE_BYTES = TRACK_DTYPE.itemsize


def track_params_default(**overrides) -> ld_track_params:
    tp = ld_track_params()
    lib().ld_track_params_default(C.byref(tp))
    for k, v in overrides.items():
        setattr(tp, k, v)
    return tp


def ld_track(f, lanes, states, state_index, tp, stream):
    return lib().ld_track(f, lanes, states, state_index, C.byref(tp) if tp is not None else None, stream)


def ld_stereo(f, left, left_pitch, right, right_pitch, rho, tau, tr_lrc, disp_out, disp_pitch, disp_lf, disp_rt,
              stream):
    return lib().ld_stereo(f, left, left_pitch, right, right_pitch, rho, tau, tr_lrc, disp_out, disp_pitch, disp_lf,
                           disp_rt, stream)


def ld_bilateral(f, grey, grey_pitch, out, out_pitch, rho, sigma_s, sigma_r, road_rows, stream):
    return lib().ld_bilateral(f, grey, grey_pitch, out, out_pitch, rho, sigma_s, sigma_r, road_rows, stream)


def ld_sync(f):
    return lib().ld_sync(f)


def ld_status_string(s):
    return lib().ld_status_string(s).decode()


def ld_frame_read(f, what, b, dst, nbytes, stream):
    return lib().ld_frame_read(f, what, b, dst, nbytes, stream)


def ld_frame_profile(f, enable):
    return lib().ld_frame_profile(f, enable)


def ld_frame_kernel_times(f, ms_out, calls_out, n):
    return lib().ld_frame_kernel_times(f, ms_out, calls_out, n)


def ld_server_create(cfg, params=None):
    h = C.c_void_p()
    st = lib().ld_server_create(C.byref(cfg), C.byref(params) if params is not None else None, C.byref(h))
    return st, h


def ld_server_destroy(s):
    return lib().ld_server_destroy(s)


def ld_server_submit(s, stream_id, cls, grey, grey_pitch, disp, disp_pitch):
    req = C.c_int64(-1)
    st = lib().ld_server_submit(s, stream_id, cls, grey, grey_pitch, disp, disp_pitch, C.byref(req))
    return st, req.value


def ld_server_poll(s, results, max_results):
    n = C.c_int32(0)
    st = lib().ld_server_poll(s, results, max_results, C.byref(n))
    return st, n.value


def ld_server_pending(s):
    q, f = C.c_int32(0), C.c_int32(0)
    st = lib().ld_server_pending(s, C.byref(q), C.byref(f))
    return st, q.value, f.value


def ld_server_engines(s):
    pc = (C.c_int32 * LD_MAX_CLASSES)()
    b = C.c_int64(0)
    st = lib().ld_server_engines(s, pc, C.byref(b))
    return st, list(pc), b.value


def ld_cnn_config_default(c: ld_cnn_config) -> None:
    lib().ld_cnn_config_default(C.byref(c))


def ld_cnn_create(cfg, params):
    h = C.c_void_p()
    st = lib().ld_cnn_create(C.byref(cfg) if cfg is not None else None, params, C.byref(h))
    return st, h


def ld_cnn_destroy(n):
    return lib().ld_cnn_destroy(n)


def ld_cnn_set_params(n, params):
    return lib().ld_cnn_set_params(n, params)


def ld_cnn_get_params(n, params):
    return lib().ld_cnn_get_params(n, params)


def ld_cnn_forward(n, f, grey, grey_pitch, disp, disp_pitch, prob_out, stream):
    return lib().ld_cnn_forward(n, f, grey, grey_pitch, disp, disp_pitch, prob_out, stream)


def ld_cnn_labels(n, f, lanes, curves, radius, radius_per_disp, labels_out, stream):
    return lib().ld_cnn_labels(n, f, lanes, curves, radius, radius_per_disp, labels_out, stream)


def ld_cnn_train_step(n, f, grey, grey_pitch, disp, disp_pitch, labels, pos_weight, inv_norm, lr, loss_out,
                      grad_out, stream):
    return lib().ld_cnn_train_step(n, f, grey, grey_pitch, disp, disp_pitch, labels, pos_weight, inv_norm, lr,
                                   loss_out, grad_out, stream)


def ld_detect_pruned(f, n, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, seed_gamma, lanes_out,
                     curves_out, stream):
    return lib().ld_detect_pruned(f, n, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, seed_gamma,
                                  lanes_out, curves_out, stream)


def ld_cnn_save(n, path):
    return lib().ld_cnn_save(n, os.fsencode(path))


def ld_cnn_load(path, cfg=None):
    h = C.c_void_p()
    st = lib().ld_cnn_load(os.fsencode(path), C.byref(cfg) if cfg is not None else None, C.byref(h))
    return st, h


CKPT_FIELDS = ("master", "adam_m", "adam_v")


def read_checkpoint(path):
    """(header dict, {array name: float32 array}) of a file written by ld_cnn_save."""
    import json
    with open(path, "rb") as fp:
        header = json.loads(fp.readline().decode())
        data = np.frombuffer(fp.read(), dtype="<f4")
    n = header["params"]
    if data.size != len(CKPT_FIELDS) * n:
        raise LdError(f"checkpoint {path}: {data.size} floats, expected {len(CKPT_FIELDS) * n}")
    return header, {k: data[i * n:(i + 1) * n].copy() for i, k in enumerate(CKPT_FIELDS)}


def cnn_config(**overrides) -> ld_cnn_config:
    c = ld_cnn_config()
    lib().ld_cnn_config_default(C.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def server_config(classes, *, n_streams=32, inflight=2, max_queue=256, use_graphs=True, seed_from_state=True,
                  hbm_budget=64 << 30, cnn=None, track=False):
    """classes: list of (width, height, fmt, d_max, max_batch).  cnn: a Cnn whose network runs
    the pruned path (it must stay open while the server lives)."""
    cfg = ld_server_config()
    cfg.cnn = cnn.handle if cnn is not None else None
    cfg.n_classes = len(classes)
    for k, (w, h, f, dm, mb) in enumerate(classes):
        cfg.width[k], cfg.height[k], cfg.fmt[k], cfg.d_max[k], cfg.max_batch[k] = w, h, f, dm, mb
    cfg.n_streams, cfg.inflight, cfg.max_queue = n_streams, inflight, max_queue
    cfg.use_graphs, cfg.seed_from_state, cfg.hbm_budget = int(use_graphs), int(seed_from_state), int(hbm_budget)
    cfg.track = int(track)
    return cfg


class Server:
    """Continuous-batching server (ld_server_*).  Frames are torch CUDA tensors [H, W] that
    the caller keeps alive until their result has been returned by poll()."""

    def __init__(self, cfg, params=None):
        self.cfg = cfg
        st, h = ld_server_create(cfg, params)
        check(st, "ld_server_create")
        self.handle = h
        self._buf = (ld_server_result * 256)()

    def close(self):
        if getattr(self, "handle", None):
            ld_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, stream_id, cls, grey, disp):
        st, req = ld_server_submit(self.handle, stream_id, cls, C.c_void_p(grey.data_ptr()),
                                   grey.stride(-2) * grey.element_size(), C.c_void_p(disp.data_ptr()),
                                   disp.stride(-2) * disp.element_size())
        return st, req

    def poll(self):
        st, n = ld_server_poll(self.handle, self._buf, len(self._buf))
        check(st, "ld_server_poll")
        out = []
        for i in range(n):
            r = self._buf[i]
            L = r.lanes
            out.append({"request": r.request, "stream": r.stream_id, "cls": r.cls, "frame_idx": r.frame_idx,
                        "t_submit": r.t_submit, "t_done": r.t_done, "n": L.n, "flags": L.flags, "v_h": L.v_h,
                        "v_end": L.v_end, "u_start": list(L.u_start[: L.n]), "energy": list(L.energy[: L.n])})
        return out

    def tracks(self, stream_id: int) -> np.ndarray:
        """The stream's tracker state (config track=True) as a TRACK_DTYPE record."""
        buf = np.zeros(1, dtype=TRACK_DTYPE)
        check(lib().ld_server_tracks(self.handle, int(stream_id), buf.ctypes.data_as(C.c_void_p)), "ld_server_tracks")
        return buf[0]

    def pending(self):
        st, q, f = ld_server_pending(self.handle)
        check(st, "ld_server_pending")
        return q, f

    def engines(self):
        st, pc, b = ld_server_engines(self.handle)
        check(st, "ld_server_engines")
        return pc, b


# ---------------------------------------------------------------------------- torch front end
def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_FMT_OF = {"uint8": LD_DISP_U8, "float32": LD_DISP_F32, "uint16": LD_DISP_U16Q4}


class Detector:
    """A frame object for `batch` frames of one size and disparity format.

    Inputs are torch CUDA tensors shaped [B, H, W] (rows may be padded: the row pitch is
    taken from the tensor's stride).  All calls are asynchronous on torch's current stream.
    """

    def __init__(self, width: int, height: int, batch: int, fmt: int, d_max: int, params: ld_params | None = None):
        self.width, self.height, self.batch, self.fmt, self.d_max = width, height, batch, fmt, d_max
        self.params = params if params is not None else params_default()
        st, h = ld_frame_create(width, height, batch, fmt, d_max, self.params)
        check(st, "ld_frame_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            ld_frame_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_active(self, n: int):
        check(ld_frame_set_active(self.handle, n), "ld_frame_set_active")

    @staticmethod
    def _pitch(t):
        return t.stride(-2) * t.element_size()

    def vdisp(self, disp, stream_ids=None, frame_idx=None, vdisp_out=None, beta_out=None):
        check(ld_vdisp(self.handle, _ptr(disp), self._pitch(disp), _ptr(stream_ids), _ptr(frame_idx),
                       _ptr(vdisp_out), _ptr(beta_out), _stream()), "ld_vdisp")

    def vp_ransac(self, grey, disp, stream_ids=None, frame_idx=None, seed_gamma=None, vp_out=None):
        check(ld_vp_ransac(self.handle, _ptr(grey), self._pitch(grey), _ptr(disp), self._pitch(disp),
                           _ptr(stream_ids), _ptr(frame_idx), _ptr(seed_gamma), _ptr(vp_out), _stream()),
              "ld_vp_ransac")

    def lane_energy(self, cand_mask=None, energy_out=None):
        check(ld_lane_energy(self.handle, _ptr(cand_mask), _ptr(energy_out), _stream()), "ld_lane_energy")

    def peaks(self, lanes_out, curves_out=None):
        check(ld_peaks(self.handle, _ptr(lanes_out), _ptr(curves_out), _stream()), "ld_peaks")

    def detect(self, grey, disp, lanes_out, stream_ids=None, frame_idx=None, curves_out=None):
        check(ld_detect(self.handle, _ptr(grey), self._pitch(grey), _ptr(disp), self._pitch(disp),
                        _ptr(stream_ids), _ptr(frame_idx), _ptr(lanes_out), _ptr(curves_out), _stream()),
              "ld_detect")

    def bilateral(self, grey, out, rho: int = 5, sigma_s: float = 300.0, sigma_r: float = 0.3,
                  road_rows: bool = False):
        """Bilateral pre-filter of the grey images into `out` (uint8, same shape)."""
        check(ld_bilateral(self.handle, _ptr(grey), self._pitch(grey), _ptr(out), self._pitch(out), int(rho),
                           float(sigma_s), float(sigma_r), 1 if road_rows else 0, _stream()), "ld_bilateral")

    def stereo(self, left, right, disp_out, disp_lf, disp_rt, rho: int = 3, tau: int = 1, tr_lrc: int = 3):
        """Disparity maps of rectified pairs (uint8 [n, H, W] tensors): the checked map into
        disp_out, the left and right maps into disp_lf / disp_rt (contiguous)."""
        check(ld_stereo(self.handle, _ptr(left), self._pitch(left), _ptr(right), self._pitch(right), int(rho),
                        int(tau), int(tr_lrc), _ptr(disp_out), self._pitch(disp_out), _ptr(disp_lf), _ptr(disp_rt),
                        _stream()), "ld_stereo")

    def track(self, lanes, states, state_index=None, params: ld_track_params | None = None):
        """Fold the lanes of the active frames into device tracker states (uint8 tensor of
        n x TRACK_STATE_BYTES; frame b -> state_index[b], identity when None)."""
        check(ld_track(self.handle, _ptr(lanes), _ptr(states), _ptr(state_index), params, _stream()), "ld_track")

    @staticmethod
    def track_states(n: int):
        """Zeroed device tracker states for n streams."""
        import torch
        return torch.zeros((n, TRACK_STATE_BYTES), dtype=torch.uint8, device="cuda")

    @staticmethod
    def parse_track_states(states) -> np.ndarray:
        return np.frombuffer(states.cpu().numpy().tobytes(), dtype=TRACK_DTYPE)

    def sync(self):
        check(ld_sync(self.handle), "ld_sync")

    def profile(self, enable: bool = True):
        check(ld_frame_profile(self.handle, 1 if enable else 0), "ld_frame_profile")

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since profile(True)."""
        ms = (C.c_double * len(KERNELS))()
        calls = (C.c_int64 * len(KERNELS))()
        check(ld_frame_kernel_times(self.handle, ms, calls, len(KERNELS)), "ld_frame_kernel_times")
        return {k: (ms[i], calls[i]) for i, k in enumerate(KERNELS)}

    def lanes_buffer(self, n=None):
        import torch
        return torch.empty((n or self.batch) * LANES_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    @staticmethod
    def parse_lanes(buf) -> np.ndarray:
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=LANES_DTYPE)

    def detect_pruned(self, net: "Cnn", grey, disp, lanes_out, stream_ids=None, frame_idx=None, curves_out=None,
                      seed_gamma=None):
        check(ld_detect_pruned(self.handle, net.handle, _ptr(grey), self._pitch(grey), _ptr(disp), self._pitch(disp),
                               _ptr(stream_ids), _ptr(frame_idx), _ptr(seed_gamma), _ptr(lanes_out),
                               _ptr(curves_out), _stream()),
              "ld_detect_pruned")

    def read(self, what: int, b: int = 0) -> np.ndarray:
        """Copy one piece of frame b's device state to the host (synchronous)."""
        import torch
        H, W, D1 = self.height, self.width, self.d_max + 1
        spec = {
            LD_STATE_INFO: (np.int32, 8), LD_STATE_MY_PATH: (np.int32, 2 * D1), LD_STATE_BETA: (FIT_DTYPE, 1),
            LD_STATE_GAMMA: (FIT_DTYPE, 1), LD_STATE_TABLES: (np.float64, 6 * H), LD_STATE_ROWCOUNT: (np.int32, H),
            LD_STATE_EDGES: (EDGE_DTYPE, H * W), LD_STATE_MX_PATH: (np.int32, H),
            LD_STATE_ENERGY: (np.float64, 2 * W), LD_STATE_TRACE: (np.int32, 6 * MAX_ROUNDS_STORED),
            LD_STATE_LANE_BITS: (np.uint8, 4 * 16 * W), LD_STATE_PRUNE: (np.int32, 16),
            LD_STATE_CAND_MASK: (np.uint8, 2 * W),
        }[what]
        dt = np.dtype(spec[0])
        nbytes = dt.itemsize * spec[1]
        host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        check(ld_frame_read(self.handle, what, b, C.c_void_p(host.data_ptr()), nbytes, _stream()), "ld_frame_read")
        torch.cuda.current_stream().synchronize()
        return np.frombuffer(host.numpy().tobytes(), dtype=dt)


class Cnn:
    """The candidate-pruning network (ld_cnn_*).  Parameters are host float32 arrays of
    LD_CNN_PARAMS values in the order of include/ld.h."""

    def __init__(self, params=None, **config):
        self.config = cnn_config(**config)
        p = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
            assert arr.size == LD_CNN_PARAMS
            p = arr.ctypes.data_as(C.POINTER(C.c_float))
        st, h = ld_cnn_create(self.config, p)
        check(st, "ld_cnn_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            ld_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path):
        """Checkpoint: master weights, Adam moments and step (ld_cnn_save)."""
        check(ld_cnn_save(self.handle, path), "ld_cnn_save")

    @classmethod
    def load(cls, path, **config):
        """A network restored from a checkpoint (its own configuration unless config is given)."""
        obj = cls.__new__(cls)
        obj.config = cnn_config(**config) if config else None
        st, h = ld_cnn_load(path, obj.config)
        check(st, "ld_cnn_load")
        obj.handle = h
        if obj.config is None:
            header, _ = read_checkpoint(path)
            obj.config = cnn_config(**header["config"])
        return obj

    def set_params(self, params):
        arr = np.ascontiguousarray(params, dtype=np.float32)
        assert arr.size == LD_CNN_PARAMS
        check(ld_cnn_set_params(self.handle, arr.ctypes.data_as(C.POINTER(C.c_float))), "ld_cnn_set_params")

    def get_params(self) -> np.ndarray:
        arr = np.zeros(LD_CNN_PARAMS, np.float32)
        check(ld_cnn_get_params(self.handle, arr.ctypes.data_as(C.POINTER(C.c_float))), "ld_cnn_get_params")
        return arr

    def forward(self, det: Detector, grey, disp, prob_out=None):
        check(ld_cnn_forward(self.handle, det.handle, _ptr(grey), det._pitch(grey), _ptr(disp), det._pitch(disp),
                             _ptr(prob_out), _stream()), "ld_cnn_forward")

    def labels(self, det: Detector, lanes, curves, labels_out, radius=2.0, radius_per_disp=0.139):
        check(ld_cnn_labels(self.handle, det.handle, _ptr(lanes), _ptr(curves), radius, radius_per_disp,
                            _ptr(labels_out), _stream()), "ld_cnn_labels")

    def train_step(self, det: Detector, grey, disp, labels, pos_weight, inv_norm, lr, loss_out=None, grad_out=None):
        check(ld_cnn_train_step(self.handle, det.handle, _ptr(grey), det._pitch(grey), _ptr(disp), det._pitch(disp),
                                _ptr(labels), pos_weight, inv_norm, lr, _ptr(loss_out), _ptr(grad_out), _stream()),
              "ld_cnn_train_step")
