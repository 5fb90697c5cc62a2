"""Python binding of libsgm (the C ABI in include/sgm.h).

Argument marshalling only: every function here checks tensor shapes and
dtypes, passes device pointers and the current HIP stream to the library,
and raises on a non-zero status.  All computation happens in the HIP
kernels of libsgm.so; there is no fallback of any kind, and importing this
module fails if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgm.so")

SGM_OK = 0
STATUS = {0: "SGM_OK", -1: "SGM_ERR_INVALID", -2: "SGM_ERR_UNSUPPORTED", -3: "SGM_ERR_HIP",
          -4: "SGM_ERR_WORKSPACE"}

# path index -> direction r = (du, dv); predecessor of p is p - r
PATH_DIRECTIONS = [(+1, 0), (-1, 0), (0, +1), (0, -1), (+1, +1), (-1, +1), (+1, -1), (-1, -1)]


class SgmError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__("%s: %s (%s)" % (what, STATUS.get(status, status), detail))
        self.status = status


class sgm_params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("census", ctypes.c_int32), ("ndisp", ctypes.c_int32),
                ("npaths", ctypes.c_int32), ("p1", ctypes.c_int32),
                ("p2", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class sgm_pair(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("ndisp", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("left", ctypes.c_void_p), ("right", ctypes.c_void_p),
                ("d_lo", ctypes.c_void_p), ("disp_int", ctypes.c_void_p),
                ("disp_sub", ctypes.c_void_p)]


class sgm_batch_params(ctypes.Structure):
    _fields_ = [("census", ctypes.c_int32), ("npaths", ctypes.c_int32),
                ("p1", ctypes.c_int32), ("p2", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class sgm_tuning(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("order", ctypes.c_int32), ("lanes", ctypes.c_int32)]


def _load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsgm.so is not built; run `python -m paper_2012_10802_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    D = ctypes.c_double
    sig = {
        "sgm_plan": [ctypes.POINTER(sgm_params), ctypes.POINTER(P)],
        "sgm_plan_free": [P],
        "sgm_plan_tuned": [ctypes.POINTER(sgm_params), ctypes.POINTER(sgm_tuning), ctypes.POINTER(P)],
        "sgm_plan_get_tuning": [P, ctypes.POINTER(sgm_tuning)],
        "sgm_autotune": [ctypes.POINTER(sgm_params), P, P, I, P, P, P, P, S, P, ctypes.c_char_p,
                         ctypes.POINTER(sgm_tuning)],
        "sgm_workspace_size": [P, ctypes.POINTER(S)],
        "sgm_census": [P, P, I, P, P],
        "sgm_cost": [P, P, P, I, P, P, P, S, P],
        "sgm_aggregate": [P, P, P, P, S, P],
        "sgm_aggregate_path": [P, P, I, P, P],
        "sgm_wta": [P, P, P, P, P, P],
        "sgm_aggregate_wta": [P, P, P, P, P, P, S, P],
        "sgm_match": [P, P, P, I, P, P, P, P, S, P],
        "sgm_match_noalloc": [P, P, P, I, P, P, P, P],
        "sgm_path_volumes": [P, ctypes.POINTER(I), ctypes.POINTER(S), ctypes.POINTER(S)],
        "sgm_aggregate_paths": [P, P, P, S, P],
        "sgm_wta_paths": [P, P, P, P, P, P],
        "sgm_window_from_road": [D, D, D, I, I, I, I, D, P],
        "sgm_downsample4": [P, I, I, I, P, P],
        "sgm_cost_win": [P, P, P, I, P, P, P, S, P],
        "sgm_aggregate_win_paths": [P, P, P, P, S, P],
        "sgm_wta_win_paths": [P, P, P, P, P, P],
        "sgm_match_win": [P, P, P, I, P, P, P, P, S, P],
        "sgm_debug_inject_fault": [I],
        "sgm_workspace_size_win_batch": [ctypes.c_void_p, I, ctypes.POINTER(ctypes.c_size_t)],
        "sgm_match_win_batch": [ctypes.c_void_p, P, P, I, ctypes.c_int64, P, I, P, P, P, S, P],
        "sgm_cnn_pack_weights": [P, P, P, P],
        "sgm_cnn_prepare_input": [P, P, I, I, I, P, P],
        "sgm_cnn_forward": [P, P, P, I, I, I, P, P, P],
        "sgm_cnn_infer": [P, P, P, I, I, I, P, P],
        "sgm_cnn_loss": [P, P, P, I, I, I, P, P, P],
        "sgm_cnn_backward": [P, P, P, P, I, I, I, P, P, S, P],
        "sgm_cnn_adam": [P, P, P, P, I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float, P, P, P],
        "sgm_window_map": [P, P, I, I, I, I, I, I, ctypes.c_float, I, P, P, P, P, P],
        "sgm_fallback_merge": [P, P, P, I, I, I, I, I, I, P, P, P],
        "sgm_fallback_merge_rects": [P, P, I, I, I, I, I, I, P, P, ctypes.c_int64, P, P, P],
        "sgm_window_map_batch": [P, P, I, I, I, I, I, I, ctypes.c_float, I, I, P, P, P, P, P],
        "sgm_downsample4_batch": [P, I, I, I, ctypes.c_int64, I, P, P],
        "sgm_label_downsample4": [P, I, I, P, P],
        "sgm_batch_plan": [ctypes.POINTER(sgm_batch_params), ctypes.POINTER(sgm_pair), I,
                           ctypes.POINTER(P)],
        "sgm_batch_free": [P],
        "sgm_batch_workspace_size": [P, ctypes.POINTER(S)],
        "sgm_batch_set_tuning": [P, ctypes.POINTER(sgm_tuning)],
        "sgm_batch_get_tuning": [P, ctypes.POINTER(sgm_tuning)],
        "sgm_batch_run": [P, P, S, P],
        "sgm_batch_capture": [P, P, S, P],
        "sgm_batch_launch": [P, P],
        "sgm_batch_run_timed": [P, P, S, P, ctypes.POINTER(ctypes.c_float)],
        "sgm_batch_autotune": [P, P, S, P, ctypes.c_char_p, ctypes.POINTER(sgm_tuning)],
        "sgm_road_workspace_size": [I, I, I, ctypes.POINTER(S)],
        "sgm_road_fit_batch": [P, P, I, I, I, ctypes.c_float, D, P, D, P, P, S, P],
        "sgm_road_window_batch": [P, I, I, I, I, I, D, D, P, P],
        "sgm_road_energy_batch": [P, P, I, I, I, ctypes.c_float, D, P, D, P, I, P, P, S, P],
        "sgm_disparity_transform_batch": [P, P, I, I, I, D, P, P],
        "sgm_pothole_workspace_size": [I, I, ctypes.POINTER(S)],
        "sgm_pothole_threshold_batch": [P, P, I, I, I, D, D, I, D, P, P, P, S, P],
        "sgm_pothole_label_batch": [P, P, I, I, I, P, P, P],
        "sgm_pothole_prune_batch": [P, I, I, I, P, P],
        "sgm_slic_workspace_size": [I, I, I, I, ctypes.POINTER(S)],
        "sgm_slic_batch": [P, P, I, I, I, I, D, I, D, P, P, P, P, P, S, P],
        "sgm_road_mask_batch": [P, P, I, I, I, D, D, P, P],
        "sgm_road_window_map_batch": [P, I, I, I, I, D, P, P],
        "sgm_status_str": [I],
        "sgm_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.sgm_plan_free.restype = None
    lib.sgm_cnn_num_params.argtypes = []
    lib.sgm_cnn_num_params.restype = ctypes.c_int32
    lib.sgm_cnn_scratch_bytes.argtypes = [I, I, I]
    lib.sgm_cnn_scratch_bytes.restype = ctypes.c_size_t
    lib.sgm_batch_free.restype = None
    lib.sgm_status_str.restype = ctypes.c_char_p
    lib.sgm_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load_library()


def library():
    """The loaded ctypes library (for tests of the exported symbols)."""
    return _lib


def _check(status: int, what: str):
    if status != SGM_OK:
        raise SgmError(status, what, _lib.sgm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, dtype, shape, name, device=True):
    if t is None:
        raise ValueError("%s is required" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if device and not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


# ---------------------------------------------------------------------------
# the C calls, one for one


def sgm_plan(width, height, census, ndisp, npaths, p1, p2, flags=0, lanes=None, order=None):
    """A plan (sgm_plan, or sgm_plan_tuned when `lanes` (0, 4, 8, 16) or the
    slot `order` (0, 1) is given)."""
    prm = sgm_params(width, height, census, ndisp, npaths, p1, p2, flags)
    h = ctypes.c_void_p()
    if lanes is None and order is None:
        _check(_lib.sgm_plan(ctypes.byref(prm), ctypes.byref(h)), "sgm_plan")
    else:
        t = sgm_tuning(0, int(order or 0), int(lanes or 0))
        _check(_lib.sgm_plan_tuned(ctypes.byref(prm), ctypes.byref(t), ctypes.byref(h)), "sgm_plan_tuned")
    return h


def sgm_plan_lanes(plan) -> int:
    """Lanes per scanline / pixel the plan's volume kernels use."""
    t = sgm_tuning()
    _check(_lib.sgm_plan_get_tuning(plan, ctypes.byref(t)), "sgm_plan_get_tuning")
    return int(t.lanes)


def sgm_plan_order(plan) -> int:
    """The plan's dispatch order of the aggregation's direction slots."""
    t = sgm_tuning()
    _check(_lib.sgm_plan_get_tuning(plan, ctypes.byref(t)), "sgm_plan_get_tuning")
    return int(t.order)


def sgm_plan_free(plan):
    _lib.sgm_plan_free(plan)


def sgm_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(_lib.sgm_workspace_size(plan, ctypes.byref(n)), "sgm_workspace_size")
    return int(n.value)


def sgm_window_from_road(a0, a1, phi, width, height, w, mode=0, delta=0.0):
    """Host helper: per-row window starts (int32 CPU tensor [H])."""
    out = torch.empty(height, dtype=torch.int32)
    _check(_lib.sgm_window_from_road(float(a0), float(a1), float(phi), int(width), int(height),
                                     int(w), int(mode), float(delta), _ptr(out)),
           "sgm_window_from_road")
    return out


def sgm_downsample4(image, out=None, stream=None):
    """4 x 4 box reduction of a uint8 device image [H, pitch] (width = pitch)."""
    _need(image, torch.uint8, None, "image")
    H, W = image.shape
    if out is None:
        out = torch.empty((H // 4, W // 4), dtype=torch.uint8, device=image.device)
    _need(out, torch.uint8, (H // 4, W // 4), "out")
    _check(_lib.sgm_downsample4(_ptr(image), W, H, W, _ptr(out), _stream(stream)), "sgm_downsample4")
    return out


def sgm_downsample4_batch(images, out=None, stream=None):
    """4 x 4 box reduction of every image of a uint8 device stack [n, H, pitch]."""
    _need(images, torch.uint8, None, "images")
    if images.dim() != 3:
        raise ValueError("images must be uint8 [n, H, pitch]")
    n, H, W = images.shape
    if out is None:
        out = torch.empty((n, H // 4, W // 4), dtype=torch.uint8, device=images.device)
    _need(out, torch.uint8, (n, H // 4, W // 4), "out")
    _check(_lib.sgm_downsample4_batch(_ptr(images), W, H, W, H * W, n, _ptr(out), _stream(stream)),
           "sgm_downsample4_batch")
    return out


# ---------------------------------------------------------------------------
# road model (Sec. II-A eq. (3), Sec. II-C eq. (11)-(13))

ROAD_FIT_WORDS = 8  # one sgm_road_fit = 8 float64 words (64 bytes)
ROAD_FIELDS = ("a0", "a1", "phi", "g_u", "g_v", "e0min", "count")


def road_workspace_size(width, height, nimg=1) -> int:
    n = ctypes.c_size_t()
    _check(_lib.sgm_road_workspace_size(int(width), int(height), int(nimg), ctypes.byref(n)),
           "sgm_road_workspace_size")
    return int(n.value)


def _maps(t, dtype, name):
    _need(t, dtype, None, name)
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError("%s must be [H, W] or [n, H, W]" % name)
    return t


def road_fit(disp, mask=None, min_disp=float("-inf"), margin=float("-inf"), prior=None, tol=float("inf"),
             fit=None, workspace=None, stream=None):
    """Fit of the road model to float32 device disparity maps [H, W] or
    [n, H, W] (mask: uint8 of the same shape, or None; pixels with
    d < min_disp or column - d < margin are skipped, and with a prior fit
    those farther than tol from its road line).  Returns the fits as a
    float64 device tensor [n, 8] (sgm_road_fit records; see road_fit_dicts)."""
    d = _maps(disp, torch.float32, "disp")
    n, H, W = d.shape
    if mask is not None:
        mask = _maps(mask, torch.uint8, "mask")
        if tuple(mask.shape) != (n, H, W):
            raise ValueError("mask must have the shape of disp")
    if fit is None:
        fit = torch.empty((n, ROAD_FIT_WORDS), dtype=torch.float64, device=d.device)
    _need(fit, torch.float64, (n, ROAD_FIT_WORDS), "fit")
    need = road_workspace_size(W, H, n)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=d.device)
    _need(workspace, torch.uint8, None, "workspace")
    if prior is not None:
        _need(prior, torch.float64, (n, ROAD_FIT_WORDS), "prior")
    _check(_lib.sgm_road_fit_batch(_ptr(d), _ptr(mask), W, H, n, float(min_disp), float(margin), _ptr(prior),
                                   float(tol), _ptr(fit),
                                   _ptr(workspace), workspace.numel(), _stream(stream)),
           "sgm_road_fit_batch")
    return fit


def road_energy(disp, phi, mask=None, min_disp=float("-inf"), margin=float("-inf"), prior=None, tol=float("inf"),
                energy=None, workspace=None, stream=None):
    """E0min(phi) of eq. (12) (the curve of Fig. 3) for float32 device maps
    [H, W] or [n, H, W] at the roll angles of `phi` (float64 device [m]),
    over the pixels road_fit selects with the same arguments.  Returns
    float64 [n, m] (NaN where eq. (12) is undefined)."""
    d = _maps(disp, torch.float32, "disp")
    n, H, W = d.shape
    if mask is not None:
        mask = _maps(mask, torch.uint8, "mask")
        if tuple(mask.shape) != (n, H, W):
            raise ValueError("mask must have the shape of disp")
    _need(phi, torch.float64, None, "phi")
    if phi.dim() != 1:
        raise ValueError("phi must be one-dimensional")
    m = phi.numel()
    if energy is None:
        energy = torch.empty((n, m), dtype=torch.float64, device=d.device)
    _need(energy, torch.float64, (n, m), "energy")
    if workspace is None:
        workspace = torch.empty(max(road_workspace_size(W, H, n), 1), dtype=torch.uint8, device=d.device)
    _need(workspace, torch.uint8, None, "workspace")
    if prior is not None:
        _need(prior, torch.float64, (n, ROAD_FIT_WORDS), "prior")
    _check(_lib.sgm_road_energy_batch(_ptr(d), _ptr(mask), W, H, n, float(min_disp), float(margin), _ptr(prior),
                                      float(tol), _ptr(phi), m, _ptr(energy), _ptr(workspace), workspace.numel(),
                                      _stream(stream)),
           "sgm_road_energy_batch")
    return energy


def road_fit_dicts(fit):
    """Host view of fits returned by road_fit (synchronises)."""
    h = fit.detach().cpu()
    st = h.view(torch.int32)[:, 14]
    out = []
    for i in range(h.shape[0]):
        rec = {k: float(h[i, j]) for j, k in enumerate(ROAD_FIELDS)}
        rec["status"] = int(st[i])
        out.append(rec)
    return out


def road_window(fit, width, height, w, mode=0, delta=0.0, scale=1.0, d_lo=None, stream=None):
    """Per-row window starts int32 [n, H] for W x H frames from device fits
    (of maps at 1/scale resolution)."""
    _need(fit, torch.float64, None, "fit")
    n = fit.shape[0]
    if d_lo is None:
        d_lo = torch.empty((n, height), dtype=torch.int32, device=fit.device)
    _need(d_lo, torch.int32, (n, height), "d_lo")
    _check(_lib.sgm_road_window_batch(_ptr(fit), int(width), int(height), n, int(w), int(mode), float(delta),
                                      float(scale), _ptr(d_lo), _stream(stream)), "sgm_road_window_batch")
    return d_lo


def disparity_transform(disp, fit, delta_dt, out=None, stream=None):
    """eq. (13) on float32 device maps [H, W] or [n, H, W]; out may be disp."""
    d = _maps(disp, torch.float32, "disp")
    n, H, W = d.shape
    _need(fit, torch.float64, (n, ROAD_FIT_WORDS), "fit")
    if out is None:
        out = torch.empty_like(disp)
    _need(out, torch.float32, tuple(disp.shape), "out")
    _check(_lib.sgm_disparity_transform_batch(_ptr(d), _ptr(fit), W, H, n, float(delta_dt), _ptr(out),
                                              _stream(stream)), "sgm_disparity_transform_batch")
    return out


def road_window_map(fit, width, height, w, scale=1.0, lo=None, stream=None):
    """Per-pixel window starts int32 [n, H, W] centred on the fitted road
    plane (fits of maps at 1/scale resolution)."""
    _need(fit, torch.float64, None, "fit")
    n = fit.shape[0]
    if lo is None:
        lo = torch.empty((n, height, width), dtype=torch.int32, device=fit.device)
    _need(lo, torch.int32, (n, height, width), "lo")
    _check(_lib.sgm_road_window_map_batch(_ptr(fit), int(width), int(height), n, int(w), float(scale), _ptr(lo),
                                          _stream(stream)), "sgm_road_window_map_batch")
    return lo


def road_mask(disp, fit, f_min, margin=float("-inf"), mask=None, stream=None):
    """Road region uint8 [n, H, W] from device fits: road line f >= f_min,
    column - f >= margin, finite disparity."""
    d = _maps(disp, torch.float32, "disp")
    n, H, W = d.shape
    _need(fit, torch.float64, (n, ROAD_FIT_WORDS), "fit")
    if mask is None:
        mask = torch.empty((n, H, W), dtype=torch.uint8, device=d.device)
    _need(mask, torch.uint8, (n, H, W), "mask")
    _check(_lib.sgm_road_mask_batch(_ptr(d), _ptr(fit), W, H, n, float(f_min), float(margin), _ptr(mask),
                                    _stream(stream)), "sgm_road_mask_batch")
    return mask


# ---------------------------------------------------------------------------
# pothole threshold and labelling (Sec. II-E, eq. (14), (15))

POTHOLE_WORDS = 6  # one sgm_pothole_threshold = 6 float64 words (48 bytes)


def pothole_workspace_size(nbins, nimg=1) -> int:
    n = ctypes.c_size_t()
    _check(_lib.sgm_pothole_workspace_size(int(nbins), int(nimg), ctypes.byref(n)), "sgm_pothole_workspace_size")
    return int(n.value)


def pothole_threshold(d2, lo, hi, nbins, delta_pd, mask=None, result=None, curve=False, workspace=None,
                      stream=None):
    """Threshold search on float32 device maps [H, W] or [n, H, W].  Returns
    (result float64 [n, 6] device tensor of sgm_pothole_threshold records,
    E2 curves float64 [n, nbins + 1] or None)."""
    d = _maps(d2, torch.float32, "d2")
    n, H, W = d.shape
    if mask is not None:
        mask = _maps(mask, torch.uint8, "mask")
        if tuple(mask.shape) != (n, H, W):
            raise ValueError("mask must have the shape of d2")
    if result is None:
        result = torch.empty((n, POTHOLE_WORDS), dtype=torch.float64, device=d.device)
    _need(result, torch.float64, (n, POTHOLE_WORDS), "result")
    cv = torch.empty((n, int(nbins) + 1), dtype=torch.float64, device=d.device) if curve else None
    if workspace is None:
        workspace = torch.empty(pothole_workspace_size(nbins, n), dtype=torch.uint8, device=d.device)
    _need(workspace, torch.uint8, None, "workspace")
    _check(_lib.sgm_pothole_threshold_batch(_ptr(d), _ptr(mask), W, H, n, float(lo), float(hi), int(nbins),
                                            float(delta_pd), _ptr(result), _ptr(cv), _ptr(workspace),
                                            workspace.numel(), _stream(stream)), "sgm_pothole_threshold_batch")
    return result, cv


def pothole_threshold_dicts(result):
    """Host view of pothole_threshold results (synchronises)."""
    h = result.detach().cpu()
    iv = h.view(torch.int32)
    out = []
    for i in range(h.shape[0]):
        rec = {k: float(h[i, j]) for j, k in enumerate(("t_r", "t_s", "e2", "n1", "n2"))}
        rec["k"], rec["status"] = int(iv[i, 10]), int(iv[i, 11])
        out.append(rec)
    return out


def pothole_labels(d2, result, mask=None, labels=None, stream=None):
    """8-connected pothole labels int32 [n, H, W] (1 + smallest index, 0 off)."""
    d = _maps(d2, torch.float32, "d2")
    n, H, W = d.shape
    _need(result, torch.float64, (n, POTHOLE_WORDS), "result")
    if mask is not None:
        mask = _maps(mask, torch.uint8, "mask")
    if labels is None:
        labels = torch.empty((n, H, W), dtype=torch.int32, device=d.device)
    _need(labels, torch.int32, (n, H, W), "labels")
    _check(_lib.sgm_pothole_label_batch(_ptr(d), _ptr(mask), W, H, n, _ptr(result), _ptr(labels),
                                        _stream(stream)), "sgm_pothole_label_batch")
    return labels


def pothole_prune(labels, superpixels, stream=None):
    """Removes, in place, the components of int32 device labels [H, W] or
    [n, H, W] that lie in a single superpixel (int32 superpixel labels of
    the same shape); returns `labels`."""
    lab = _maps(labels, torch.int32, "labels")
    sp = _maps(superpixels, torch.int32, "superpixels")
    if tuple(sp.shape) != tuple(lab.shape):
        raise ValueError("superpixels must have the shape of labels")
    n, H, W = lab.shape
    _check(_lib.sgm_pothole_prune_batch(_ptr(sp), W, H, n, _ptr(lab), _stream(stream)), "sgm_pothole_prune_batch")
    return labels


# ---------------------------------------------------------------------------
# superpixels (SLIC, Sec. II-D) and D3 (Sec. II-E)


def slic_workspace_size(width, height, S, nimg=1) -> int:
    n = ctypes.c_size_t()
    _check(_lib.sgm_slic_workspace_size(int(width), int(height), int(S), int(nimg), ctypes.byref(n)),
           "sgm_slic_workspace_size")
    return int(n.value)


def slic_num_centres(width, height, S) -> int:
    return ((int(width) + S - 1) // S) * ((int(height) + S - 1) // S)


def slic(d2, S, m, iters, mask=None, tol=0.0, labels=None, d3=None, centres=None, workspace=None, rounds=None,
         stream=None):
    """SLIC on float32 device maps [H, W] or [n, H, W], at most `iters`
    rounds, stopping per map after the first round whose largest centre
    change is <= tol^2.  Returns (labels int32 [n, H, W], d3 float32
    [n, H, W], centres float64 [n, K, 3]); `rounds`, an int32 [n] device
    tensor, receives the rounds each map ran."""
    d = _maps(d2, torch.float32, "d2")
    n, H, W = d.shape
    if mask is not None:
        mask = _maps(mask, torch.uint8, "mask")
        if tuple(mask.shape) != (n, H, W):
            raise ValueError("mask must have the shape of d2")
    K = slic_num_centres(W, H, S)
    if labels is None:
        labels = torch.empty((n, H, W), dtype=torch.int32, device=d.device)
    if d3 is None:
        d3 = torch.empty((n, H, W), dtype=torch.float32, device=d.device)
    if centres is None:
        centres = torch.empty((n, K, 3), dtype=torch.float64, device=d.device)
    _need(labels, torch.int32, (n, H, W), "labels")
    _need(d3, torch.float32, (n, H, W), "d3")
    _need(centres, torch.float64, (n, K, 3), "centres")
    if rounds is not None:
        _need(rounds, torch.int32, (n,), "rounds")
    if workspace is None:
        workspace = torch.empty(slic_workspace_size(W, H, S, n), dtype=torch.uint8, device=d.device)
    _need(workspace, torch.uint8, None, "workspace")
    _check(_lib.sgm_slic_batch(_ptr(d), _ptr(mask), W, H, n, int(S), float(m), int(iters), float(tol),
                               _ptr(rounds), _ptr(labels), _ptr(d3), _ptr(centres), _ptr(workspace),
                               workspace.numel(), _stream(stream)),
           "sgm_slic_batch")
    return labels, d3, centres


class Matcher:
    """A plan plus its device workspace, with one method per C call.

    Inputs and outputs are torch tensors on the current HIP device; every
    call enqueues work on the current stream (or `stream`) and returns
    without synchronising.
    """

    def __init__(self, width, height, census=7, ndisp=128, npaths=8, p1=10, p2=120,
                 device=None, workspace=None, lanes=None, order=None):
        self.W, self.H, self.n, self.w = int(width), int(height), int(census), int(ndisp)
        self.npaths, self.p1, self.p2 = int(npaths), int(p1), int(p2)
        self.plan = sgm_plan(self.W, self.H, self.n, self.w, self.npaths, self.p1, self.p2, lanes=lanes,
                             order=order)
        self.device = torch.device(device or "cuda")
        need = sgm_workspace_size(self.plan)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        _need(workspace, torch.uint8, None, "workspace")
        if workspace.numel() < need:
            raise ValueError("workspace holds %d bytes, the plan needs %d" % (workspace.numel(), need))
        self.workspace = workspace  # may be shared by matchers that run one at a time
        self.ws_bytes = workspace.numel()

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan is not None and _lib is not None:
            _lib.sgm_plan_free(plan)
            self.plan = None

    # shapes
    @property
    def image_shape(self):
        return (self.H, self.W)

    @property
    def volume_shape(self):
        return (self.H, self.W, self.w)

    def _img(self, t, name):
        _need(t, torch.uint8, None, name)
        if t.dim() != 2 or t.shape[0] != self.H or t.shape[1] < self.W:
            raise ValueError("%s must be uint8 [H, >=W]" % name)
        return t

    def _dlo(self, d_lo):
        if d_lo is None:
            return None
        return _need(d_lo, torch.int32, (self.H,), "d_lo")

    def new_volume(self, dtype=torch.uint8):
        return torch.empty(self.volume_shape, dtype=dtype, device=self.device)

    def census(self, image, codes=None, stream=None):
        self._img(image, "image")
        if codes is None:
            codes = torch.empty((self.H, self.W), dtype=torch.int64, device=self.device)
        _need(codes, torch.int64, (self.H, self.W), "codes")
        _check(_lib.sgm_census(self.plan, _ptr(image), image.shape[1], _ptr(codes),
                               _stream(stream)), "sgm_census")
        return codes

    def cost(self, left, right, d_lo=None, cost=None, stream=None):
        self._img(left, "left")
        self._img(right, "right")
        if left.shape != right.shape:
            raise ValueError("left and right must share a pitch")
        if cost is None:
            cost = self.new_volume(torch.uint8)
        _need(cost, torch.uint8, self.volume_shape, "cost")
        _check(_lib.sgm_cost(self.plan, _ptr(left), _ptr(right), left.shape[1],
                             _ptr(self._dlo(d_lo)), _ptr(cost), _ptr(self.workspace),
                             self.ws_bytes, _stream(stream)), "sgm_cost")
        return cost

    def aggregate(self, cost, out=None, stream=None):
        _need(cost, torch.uint8, self.volume_shape, "cost")
        if out is None:
            out = self.new_volume(torch.int16)
        _need(out, torch.int16, self.volume_shape, "sum")
        _check(_lib.sgm_aggregate(self.plan, _ptr(cost), _ptr(out), _ptr(self.workspace),
                                  self.ws_bytes, _stream(stream)), "sgm_aggregate")
        return out

    def aggregate_path(self, cost, path, out=None, stream=None):
        _need(cost, torch.uint8, self.volume_shape, "cost")
        if out is None:
            out = self.new_volume(torch.int16)
        _need(out, torch.int16, self.volume_shape, "L")
        _check(_lib.sgm_aggregate_path(self.plan, _ptr(cost), int(path), _ptr(out),
                                       _stream(stream)), "sgm_aggregate_path")
        return out

    def _outs(self, disp_int, disp_sub, want_sub):
        if disp_int is None:
            disp_int = torch.empty(self.image_shape, dtype=torch.int16, device=self.device)
        _need(disp_int, torch.int16, self.image_shape, "disp_int")
        if disp_sub is None and want_sub:
            disp_sub = torch.empty(self.image_shape, dtype=torch.float32, device=self.device)
        if disp_sub is not None:
            _need(disp_sub, torch.float32, self.image_shape, "disp_sub")
        return disp_int, disp_sub

    def wta(self, sum_volume, d_lo=None, disp_int=None, disp_sub=None, subpixel=True, stream=None):
        _need(sum_volume, torch.int16, self.volume_shape, "sum")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_wta(self.plan, _ptr(sum_volume), _ptr(self._dlo(d_lo)), _ptr(disp_int),
                            _ptr(disp_sub), _stream(stream)), "sgm_wta")
        return disp_int, disp_sub

    def aggregate_wta(self, cost, d_lo=None, disp_int=None, disp_sub=None, subpixel=True,
                      stream=None):
        _need(cost, torch.uint8, self.volume_shape, "cost")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_aggregate_wta(self.plan, _ptr(cost), _ptr(self._dlo(d_lo)),
                                      _ptr(disp_int), _ptr(disp_sub), _ptr(self.workspace),
                                      self.ws_bytes, _stream(stream)), "sgm_aggregate_wta")
        return disp_int, disp_sub

    def path_volumes(self):
        """(elem_bytes, volume_stride, total_bytes) of sgm_aggregate_paths' output."""
        e, vs, tot = ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.sgm_path_volumes(self.plan, ctypes.byref(e), ctypes.byref(vs), ctypes.byref(tot)),
               "sgm_path_volumes")
        return int(e.value), int(vs.value), int(tot.value)

    def new_paths(self):
        return torch.empty(self.path_volumes()[2], dtype=torch.uint8, device=self.device)

    def aggregate_paths(self, cost, paths=None, stream=None):
        _need(cost, torch.uint8, self.volume_shape, "cost")
        if paths is None:
            paths = self.new_paths()
        _need(paths, torch.uint8, None, "paths")
        _check(_lib.sgm_aggregate_paths(self.plan, _ptr(cost), _ptr(paths), paths.numel(),
                                        _stream(stream)), "sgm_aggregate_paths")
        return paths

    def path_volume(self, paths, r):
        """View of direction r's volume inside an sgm_aggregate_paths buffer."""
        e, vs, _ = self.path_volumes()
        n = self.H * self.W * self.w
        v = paths[r * vs: r * vs + n * e]
        return (v if e == 1 else v.view(torch.int16)).view(self.volume_shape)

    def wta_paths(self, paths, d_lo=None, disp_int=None, disp_sub=None, subpixel=True, stream=None):
        _need(paths, torch.uint8, None, "paths")
        if paths.numel() < self.path_volumes()[2]:
            raise ValueError("paths buffer too small")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_wta_paths(self.plan, _ptr(paths), _ptr(self._dlo(d_lo)), _ptr(disp_int),
                                  _ptr(disp_sub), _stream(stream)), "sgm_wta_paths")
        return disp_int, disp_sub

    # per-pixel windows (ndisp <= 16): lo is int32 [H, W] on the device

    def _lo(self, lo):
        return _need(lo, torch.int32, (self.H, self.W), "lo")

    def cost_win(self, left, right, lo, cost=None, stream=None):
        self._img(left, "left")
        self._img(right, "right")
        if cost is None:
            cost = self.new_volume(torch.uint8)
        _need(cost, torch.uint8, self.volume_shape, "cost")
        _check(_lib.sgm_cost_win(self.plan, _ptr(left), _ptr(right), left.shape[1], _ptr(self._lo(lo)),
                                 _ptr(cost), _ptr(self.workspace), self.ws_bytes, _stream(stream)),
               "sgm_cost_win")
        return cost

    def aggregate_win_paths(self, cost, lo, paths=None, stream=None):
        _need(cost, torch.uint8, self.volume_shape, "cost")
        if paths is None:
            paths = self.new_paths()
        _check(_lib.sgm_aggregate_win_paths(self.plan, _ptr(cost), _ptr(self._lo(lo)), _ptr(paths),
                                            paths.numel(), _stream(stream)), "sgm_aggregate_win_paths")
        return paths

    def wta_win_paths(self, paths, lo, disp_int=None, disp_sub=None, subpixel=True, stream=None):
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_wta_win_paths(self.plan, _ptr(paths), _ptr(self._lo(lo)), _ptr(disp_int),
                                      _ptr(disp_sub), _stream(stream)), "sgm_wta_win_paths")
        return disp_int, disp_sub

    def match_win(self, left, right, lo, disp_int=None, disp_sub=None, subpixel=True, stream=None):
        self._img(left, "left")
        self._img(right, "right")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_match_win(self.plan, _ptr(left), _ptr(right), left.shape[1], _ptr(self._lo(lo)),
                                  _ptr(disp_int), _ptr(disp_sub), _ptr(self.workspace), self.ws_bytes,
                                  _stream(stream)), "sgm_match_win")
        return disp_int, disp_sub

    def win_batch_workspace(self, n):
        b = ctypes.c_size_t()
        _check(_lib.sgm_workspace_size_win_batch(self.plan, int(n), ctypes.byref(b)), "sgm_workspace_size_win_batch")
        return torch.empty(int(b.value), dtype=torch.uint8, device=self.device)

    def match_win_batch(self, left, right, lo, disp_int=None, disp_sub=None, subpixel=True, workspace=None,
                        stream=None):
        """Per-pixel-window SGM of n pairs at once: left, right uint8
        [n, H, pitch]; lo int32 [n, H, W]; outputs [n, H, W].  `workspace`
        from win_batch_workspace(n) (allocated here if omitted)."""
        _need(left, torch.uint8, None, "left")
        _need(right, torch.uint8, None, "right")
        if left.dim() != 3 or left.shape != right.shape or left.shape[1] != self.H or left.shape[2] < self.W:
            raise ValueError("left and right must be uint8 [n, H, >=W] of one shape")
        n = left.shape[0]
        _need(lo, torch.int32, (n, self.H, self.W), "lo")
        if disp_int is None:
            disp_int = torch.empty((n, self.H, self.W), dtype=torch.int16, device=self.device)
        _need(disp_int, torch.int16, (n, self.H, self.W), "disp_int")
        if disp_sub is None and subpixel:
            disp_sub = torch.empty((n, self.H, self.W), dtype=torch.float32, device=self.device)
        if disp_sub is not None:
            _need(disp_sub, torch.float32, (n, self.H, self.W), "disp_sub")
        if workspace is None:
            workspace = self.win_batch_workspace(n)
        _need(workspace, torch.uint8, None, "workspace")
        pitch = left.shape[2]
        _check(_lib.sgm_match_win_batch(self.plan, _ptr(left), _ptr(right), pitch, self.H * pitch, _ptr(lo), n,
                                        _ptr(disp_int), _ptr(disp_sub), _ptr(workspace), workspace.numel(),
                                        _stream(stream)), "sgm_match_win_batch")
        return disp_int, disp_sub

    def match_at(self, left, right, y0, x0, disp_int=None, disp_sub=None, subpixel=True, stream=None):
        """Plain SGM of the H x W rectangle at row y0, column x0 of larger
        frames left, right (uint8 [Hf, pitch]); outputs are [H, W]."""
        _need(left, torch.uint8, None, "left")
        _need(right, torch.uint8, None, "right")
        if left.shape != right.shape or left.dim() != 2:
            raise ValueError("left and right must be uint8 frames of one shape")
        Hf, pitch = left.shape
        y0, x0 = int(y0), int(x0)
        if y0 < 0 or x0 < 0 or y0 + self.H > Hf or x0 + self.W > pitch:
            raise ValueError("rectangle outside the frame")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        off = y0 * pitch + x0
        _check(_lib.sgm_match(self.plan, ctypes.c_void_p(left.data_ptr() + off),
                              ctypes.c_void_p(right.data_ptr() + off), pitch, None, _ptr(disp_int),
                              _ptr(disp_sub), _ptr(self.workspace), self.ws_bytes, _stream(stream)), "sgm_match")
        return disp_int, disp_sub

    def match(self, left, right, d_lo=None, disp_int=None, disp_sub=None, subpixel=True,
              stream=None):
        self._img(left, "left")
        self._img(right, "right")
        disp_int, disp_sub = self._outs(disp_int, disp_sub, subpixel)
        _check(_lib.sgm_match(self.plan, _ptr(left), _ptr(right), left.shape[1],
                              _ptr(self._dlo(d_lo)), _ptr(disp_int), _ptr(disp_sub),
                              _ptr(self.workspace), self.ws_bytes, _stream(stream)), "sgm_match")
        return disp_int, disp_sub

    @property
    def lanes(self):
        return sgm_plan_lanes(self.plan)

    @property
    def order(self):
        return sgm_plan_order(self.plan)

    def autotune(self, left, right, d_lo=None, cache_path=None, stream=None):
        """Time every lane mapping and slot order on these inputs
        (sgm_autotune; the host waits), then rebuild the plan with the
        fastest.  Returns the lane count chosen (the order: `order`)."""
        self._img(left, "left")
        self._img(right, "right")
        di, ds = self._outs(None, None, True)
        prm = sgm_params(self.W, self.H, self.n, self.w, self.npaths, self.p1, self.p2, 0)
        t = sgm_tuning()
        path = None if cache_path is None else str(cache_path).encode()
        _check(_lib.sgm_autotune(ctypes.byref(prm), _ptr(left), _ptr(right), left.shape[1], _ptr(self._dlo(d_lo)),
                                 _ptr(di), _ptr(ds), _ptr(self.workspace), self.ws_bytes, _stream(stream), path,
                                 ctypes.byref(t)), "sgm_autotune")
        old = self.plan
        self.plan = sgm_plan(self.W, self.H, self.n, self.w, self.npaths, self.p1, self.p2, lanes=int(t.lanes),
                             order=int(t.order))
        _lib.sgm_plan_free(old)
        return int(t.lanes)


class Batch:
    """Many pairs (of several sizes) matched together by the batch calls.

    `pairs` is a list of dicts with `left`, `right` (uint8 device tensors
    [H, pitch]), `ndisp` and optionally `width` (default: the tensor width),
    `d_lo` (int32 [H] device tensor) and `subpixel` (default True).  A pair
    may also be a rectangle of its frames: `y0`, `x0`, `height`, `width`
    (the images are then read at that offset with the frames' pitch).  The
    outputs are allocated here (`disp_int[i]`, `disp_sub[i]`, [height,
    width]) unless given as `disp_int` / `disp_sub` (contiguous int16 /
    float32 device tensors of that shape), and written by every run.
    Census, paths and penalties are shared by the batch.
    """

    def __init__(self, pairs, census=7, npaths=8, p1=10, p2=120, device=None):
        self.device = torch.device(device or "cuda")
        self._keep = []
        self.disp_int, self.disp_sub = [], []
        arr = (sgm_pair * len(pairs))()
        for i, pr in enumerate(pairs):
            left, right = pr["left"], pr["right"]
            _need(left, torch.uint8, None, "left")
            _need(right, torch.uint8, None, "right")
            if left.shape != right.shape or left.dim() != 2:
                raise ValueError("pair %d: left and right must be uint8 [H, pitch] of one shape" % i)
            Hf, pitch = left.shape
            y0, x0 = int(pr.get("y0", 0)), int(pr.get("x0", 0))
            H = int(pr.get("height", Hf - y0))
            W = int(pr.get("width", pitch - x0))
            if y0 < 0 or x0 < 0 or H < 1 or W < 1 or y0 + H > Hf or x0 + W > pitch:
                raise ValueError("pair %d: rectangle outside the frames" % i)
            off = y0 * pitch + x0
            d_lo = pr.get("d_lo")
            if d_lo is not None:
                _need(d_lo, torch.int32, (H,), "d_lo")
            di = pr.get("disp_int")
            if di is None:
                di = torch.empty((H, W), dtype=torch.int16, device=self.device)
            _need(di, torch.int16, (H, W), "disp_int")
            ds = pr.get("disp_sub")
            if ds is None and pr.get("subpixel", True):
                ds = torch.empty((H, W), dtype=torch.float32, device=self.device)
            if ds is not None:
                _need(ds, torch.float32, (H, W), "disp_sub")
            self.disp_int.append(di)
            self.disp_sub.append(ds)
            self._keep += [left, right, d_lo]
            arr[i] = sgm_pair(W, H, int(pr["ndisp"]), pitch, left.data_ptr() + off, right.data_ptr() + off,
                              None if d_lo is None else d_lo.data_ptr(), di.data_ptr(),
                              None if ds is None else ds.data_ptr())
        prm = sgm_batch_params(census, npaths, p1, p2, 0)
        h = ctypes.c_void_p()
        _check(_lib.sgm_batch_plan(ctypes.byref(prm), arr, len(pairs), ctypes.byref(h)),
               "sgm_batch_plan")
        self.handle = h
        n = ctypes.c_size_t()
        _check(_lib.sgm_batch_workspace_size(self.handle, ctypes.byref(n)), "sgm_batch_workspace_size")
        self.ws_bytes = int(n.value)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.sgm_batch_free(h)
            self.handle = None

    @property
    def tuning(self):
        """(waves per CU, queue order, lanes per scanline: 0 = default)"""
        t = sgm_tuning()
        _check(_lib.sgm_batch_get_tuning(self.handle, ctypes.byref(t)), "sgm_batch_get_tuning")
        return int(t.waves_per_cu), int(t.order), int(t.lanes)

    @tuning.setter
    def tuning(self, value):
        lanes = int(value[2]) if len(value) > 2 else 0
        t = sgm_tuning(int(value[0]), int(value[1]), lanes)
        _check(_lib.sgm_batch_set_tuning(self.handle, ctypes.byref(t)), "sgm_batch_set_tuning")

    def run(self, stream=None):
        _check(_lib.sgm_batch_run(self.handle, _ptr(self.workspace), self.ws_bytes, _stream(stream)),
               "sgm_batch_run")

    def run_timed(self, stream=None):
        """One run with its stages timed by HIP events on `stream`; waits for
        it and returns the census, cost, aggregation and selection times (ms)."""
        ms = (ctypes.c_float * 4)()
        _check(_lib.sgm_batch_run_timed(self.handle, _ptr(self.workspace), self.ws_bytes, _stream(stream), ms),
               "sgm_batch_run_timed")
        return [float(x) for x in ms]

    def capture(self, stream):
        """Record one run into a graph on `stream` (a non-default torch stream)."""
        _check(_lib.sgm_batch_capture(self.handle, _ptr(self.workspace), self.ws_bytes,
                                      _stream(stream)), "sgm_batch_capture")

    def launch(self, stream=None):
        _check(_lib.sgm_batch_launch(self.handle, _stream(stream)), "sgm_batch_launch")

    def autotune(self, cache_path=None, stream=None):
        t = sgm_tuning()
        path = None if cache_path is None else str(cache_path).encode()
        _check(_lib.sgm_batch_autotune(self.handle, _ptr(self.workspace), self.ws_bytes,
                                       _stream(stream), path, ctypes.byref(t)), "sgm_batch_autotune")
        return int(t.waves_per_cu), int(t.order), int(t.lanes)


def u16(t: torch.Tensor) -> torch.Tensor:
    """Reinterpret an int16 tensor holding uint16 values as int32 values."""
    return t.to(torch.int32) & 0xFFFF
