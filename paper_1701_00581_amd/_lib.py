"""ctypes binding of libnvsm.so (argument marshalling only).

Every function here has the name of the C entry point it calls and passes
its arguments through: plain integers, device pointers (taken from torch
tensors with ``data_ptr()``) and the HIP stream.  All computation happens
in the library's HIP kernels; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnvsm.so")

NVSM_OK = 0
NVSM_ERR_INVALID_ARG = -1
NVSM_ERR_SHAPE = -2
NVSM_ERR_WORKSPACE = -3
NVSM_ERR_OOM = -4
NVSM_ERR_HIP = -5
NVSM_ERR_NOT_IMPLEMENTED = -6
NVSM_U16 = 0
NVSM_F32 = 1

EXPORTS = [
    "nvsm_create", "nvsm_destroy", "nvsm_status_string", "nvsm_last_error",
    "nvsm_default_params", "nvsm_plan", "nvsm_w_index", "nvsm_bispectrum_index",
    "nvsm_prepare", "nvsm_accumulate", "nvsm_solve", "nvsm_synthesize", "nvsm_reconstruct",
    "nvsm_reconstruct_noalloc",
    "nvsm_profile_enable", "nvsm_profile_read", "nvsm_batch_plan", "nvsm_reconstruct_batch",
    "nvsm_autotune", "nvsm_set_launch", "nvsm_tune_radius_plan", "nvsm_tune_radius", "nvsm_stream_plan", "nvsm_stream_add", "nvsm_stream_finish",
    "nvsm_model_stf_plan", "nvsm_model_stf", "nvsm_seeing_default_params", "nvsm_seeing_plan", "nvsm_seeing",
]
STAGES = ["ingest", "bispectrum", "solve", "synthesize"]


class NvsmError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)}) {detail}".strip())


class Params(ctypes.Structure):
    _fields_ = [
        ("patch", ctypes.c_int32), ("stride", ctypes.c_int32), ("u_cut", ctypes.c_int32),
        ("v_radius", ctypes.c_int32), ("window", ctypes.c_int32), ("phase_method", ctypes.c_int32),
        ("noise_bias", ctypes.c_int32), ("filter", ctypes.c_int32), ("stf_floor", ctypes.c_double),
        ("lsq_iters", ctypes.c_int32), ("reserved", ctypes.c_int32), ("photons_per_adu", ctypes.c_double),
    ]


class SeeingParams(ctypes.Structure):
    _fields_ = [
        ("screens", ctypes.c_int32), ("points", ctypes.c_int32), ("d_over_r0_min", ctypes.c_double),
        ("d_over_r0_max", ctypes.c_double), ("bins", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("patches_y", ctypes.c_int32), ("patches_x", ctypes.c_int32), ("patches", ctypes.c_int64),
        ("w_count", ctypes.c_int64), ("s_count", ctypes.c_int64), ("shells", ctypes.c_int32),
        ("frame_chunks", ctypes.c_int32), ("ws_accumulate", ctypes.c_size_t),
        ("ws_solve", ctypes.c_size_t), ("ws_synthesize", ctypes.c_size_t),
        ("ws_reconstruct", ctypes.c_size_t),
    ]


class Burst(ctypes.Structure):
    _fields_ = [
        ("frames", ctypes.c_void_p), ("F", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("row_pitch", ctypes.c_int64), ("stf", ctypes.c_void_p), ("out", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1701_00581_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        c_p, c_i32, c_i64, c_sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER(Params)
        L.nvsm_create.argtypes = [ctypes.c_int, ctypes.POINTER(c_p)]
        L.nvsm_destroy.argtypes = [c_p]
        L.nvsm_destroy.restype = None
        L.nvsm_status_string.argtypes = [ctypes.c_int]
        L.nvsm_status_string.restype = ctypes.c_char_p
        L.nvsm_last_error.argtypes = [c_p]
        L.nvsm_last_error.restype = ctypes.c_char_p
        L.nvsm_default_params.argtypes = [c_i32, P]
        L.nvsm_plan.argtypes = [P, c_i32, c_i32, c_i32, ctypes.POINTER(PlanInfo)]
        L.nvsm_w_index.argtypes = [P, c_p, c_i64]
        L.nvsm_bispectrum_index.argtypes = [P, c_p, c_i64]
        L.nvsm_prepare.argtypes = [c_p, P]
        L.nvsm_accumulate.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64,
                                      c_p, c_p, c_p, c_p, c_p, c_sz, c_p]
        L.nvsm_solve.argtypes = [c_p, P, c_i64, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]
        L.nvsm_synthesize.argtypes = [c_p, P, c_i32, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]
        L.nvsm_reconstruct.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64,
                                       c_p, c_p, c_p, c_sz, c_p]
        L.nvsm_reconstruct_noalloc.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64, c_p, c_p, c_p]
        L.nvsm_batch_plan.argtypes = [P, ctypes.POINTER(Burst), c_i32, ctypes.POINTER(c_sz),
                                      ctypes.POINTER(c_sz)]
        L.nvsm_reconstruct_batch.argtypes = [c_p, P, ctypes.c_int, ctypes.POINTER(Burst), c_i32, c_p, c_sz, c_p]
        L.nvsm_autotune.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64, c_p, c_sz, c_p,
                                    ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]
        L.nvsm_set_launch.argtypes = [c_p, P, c_i32, c_i32]
        L.nvsm_tune_radius_plan.argtypes = [P, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]
        L.nvsm_tune_radius.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64, c_p, c_i32, c_i32,
                                       ctypes.c_double, c_p, c_sz, c_p, ctypes.POINTER(c_i32), c_p]
        L.nvsm_stream_plan.argtypes = [P, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz), ctypes.POINTER(c_sz)]
        L.nvsm_stream_add.argtypes = [c_p, P, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64, c_i32, c_i32, c_p,
                                      c_sz, c_p, c_sz, c_p]
        L.nvsm_stream_finish.argtypes = [c_p, P, c_i32, c_i32, c_p, c_p, c_p, c_sz, c_p]
        L.nvsm_model_stf_plan.argtypes = [P, c_i32, ctypes.POINTER(c_sz)]
        L.nvsm_model_stf.argtypes = [c_p, P, ctypes.c_double, c_i32, ctypes.c_uint64, c_p, c_p, c_p, c_sz, c_p]
        SP = ctypes.POINTER(SeeingParams)
        L.nvsm_seeing_default_params.argtypes = [SP]
        L.nvsm_seeing_plan.argtypes = [P, SP, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz), ctypes.POINTER(c_i32)]
        L.nvsm_seeing.argtypes = [c_p, P, SP, c_p, ctypes.c_int, c_i32, c_i32, c_i32, c_i64, c_p, c_p, c_p, c_p, c_sz,
                                  c_p]
        L.nvsm_profile_enable.argtypes = [c_p, c_i32]
        L.nvsm_profile_read.argtypes = [c_p, c_p, c_p, c_i32]
        for name in EXPORTS:
            if name not in ("nvsm_destroy", "nvsm_status_string", "nvsm_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status):
    return lib().nvsm_status_string(int(status)).decode()


def _ptr(t):
    """Device (or host) address of a tensor / array / int; None -> NULL."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    if hasattr(t, "ctypes"):
        return t.ctypes.data
    raise TypeError(f"cannot take the address of {type(t)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status, where, ctx=None):
    if status != NVSM_OK:
        detail = ""
        if ctx is not None:
            detail = lib().nvsm_last_error(ctx).decode()
        raise NvsmError(status, where, detail)


def _set_fields(struct, kw):
    names = {f[0] for f in type(struct)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{type(struct).__name__} has no field {k!r}")
        setattr(struct, k, v)
    return struct


def default_params(patch, **kw):
    p = Params()
    _check(lib().nvsm_default_params(int(patch), ctypes.byref(p)), "nvsm_default_params")
    return _set_fields(p, kw)


def nvsm_create(device=0):
    h = ctypes.c_void_p()
    _check(lib().nvsm_create(int(device), ctypes.byref(h)), "nvsm_create")
    return h.value


def nvsm_destroy(ctx):
    lib().nvsm_destroy(ctx)


def nvsm_last_error(ctx):
    return lib().nvsm_last_error(ctx).decode()


def nvsm_plan(params, H, W, F):
    info = PlanInfo()
    _check(lib().nvsm_plan(ctypes.byref(params), int(H), int(W), int(F), ctypes.byref(info)), "nvsm_plan")
    return info


def nvsm_w_index(params):
    import numpy as np
    info = nvsm_plan(params, params.patch, params.patch, 1)
    out = np.zeros((info.w_count, 2), dtype=np.int32)
    _check(lib().nvsm_w_index(ctypes.byref(params), out.ctypes.data, info.w_count), "nvsm_w_index")
    return out


def nvsm_bispectrum_index(params):
    import numpy as np
    info = nvsm_plan(params, params.patch, params.patch, 1)
    out = np.zeros((info.s_count, 4), dtype=np.int32)
    _check(lib().nvsm_bispectrum_index(ctypes.byref(params), out.ctypes.data, info.s_count),
           "nvsm_bispectrum_index")
    return out


def nvsm_prepare(ctx, params):
    _check(lib().nvsm_prepare(ctx, ctypes.byref(params)), "nvsm_prepare", ctx)


def frames_dtype(frames):
    import torch
    if frames.dtype in (torch.int16, torch.uint16):
        return NVSM_U16
    if frames.dtype == torch.float32:
        return NVSM_F32
    raise TypeError("frames must be uint16 (or int16 holding uint16 bits) or float32")


def _row_pitch(frames, row_pitch=None):
    """Row pitch (elements) of a frames tensor laid out as [F][H][pitch]
    with unit stride along x.  Views of such a buffer (a crop in x or y,
    a frame range) qualify; other layouts (transposed, strided in x, every
    other frame) are rejected before any call.  An explicit row_pitch
    states the layout of the memory behind the pointer instead."""
    if row_pitch is not None:
        return int(row_pitch)
    F, H, W = frames.shape
    pitch = frames.stride(1)
    if (W > 1 and frames.stride(2) != 1) or pitch < W or (F > 1 and frames.stride(0) != H * pitch):
        raise ValueError(f"frames must be a [F][H][pitch] buffer with unit x stride; got shape "
                         f"{tuple(frames.shape)} strides {tuple(frames.stride())}")
    return pitch


def nvsm_accumulate(ctx, params, frames, power, mean_spec, mu, bispec, workspace, stream=None,
                    row_pitch=None):
    F, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    st = lib().nvsm_accumulate(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), F, H, W, pitch,
                               _ptr(power), _ptr(mean_spec), _ptr(mu), _ptr(bispec), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream))
    _check(st, "nvsm_accumulate", ctx)


def nvsm_solve(ctx, params, patches, power, mean_spec, bispec, stf, amp, phasor, workspace=None,
               stream=None):
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = lib().nvsm_solve(ctx, ctypes.byref(params), int(patches), _ptr(power), _ptr(mean_spec), _ptr(bispec),
                          _ptr(stf), _ptr(amp), _ptr(phasor), _ptr(workspace), ws_bytes, _stream(stream))
    _check(st, "nvsm_solve", ctx)


def nvsm_synthesize(ctx, params, H, W, amp, phasor, mu, patches_out, out, workspace=None, stream=None):
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = lib().nvsm_synthesize(ctx, ctypes.byref(params), int(H), int(W), _ptr(amp), _ptr(phasor), _ptr(mu),
                               _ptr(patches_out), _ptr(out), _ptr(workspace), ws_bytes, _stream(stream))
    _check(st, "nvsm_synthesize", ctx)


def nvsm_reconstruct(ctx, params, frames, stf, out, workspace, stream=None, row_pitch=None):
    F, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    st = lib().nvsm_reconstruct(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), F, H, W, pitch,
                                _ptr(stf), _ptr(out), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream))
    _check(st, "nvsm_reconstruct", ctx)


def nvsm_reconstruct_noalloc(ctx, params, frames, stf, out, stream=None, row_pitch=None):
    F, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    st = lib().nvsm_reconstruct_noalloc(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), F, H, W,
                                        pitch, _ptr(stf), _ptr(out), _stream(stream))
    _check(st, "nvsm_reconstruct_noalloc", ctx)


def _bursts(bursts):
    """ctypes array of Burst from (frames, stf, out) triples of tensors
    (frames [F][H][W] with any row pitch)."""
    arr = (Burst * len(bursts))()
    for i, (frames, stf, out) in enumerate(bursts):
        F, H, W = frames.shape
        arr[i] = Burst(_ptr(frames), F, H, W, _row_pitch(frames), _ptr(stf), _ptr(out))
    return arr


def nvsm_batch_plan(params, shapes):
    """(ws_min, ws_all) bytes for bursts of the given (F, H, W) shapes."""
    arr = (Burst * len(shapes))()
    for i, (F, H, W) in enumerate(shapes):
        arr[i] = Burst(None, F, H, W, W, None, None)
    lo, hi = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().nvsm_batch_plan(ctypes.byref(params), arr, len(shapes), ctypes.byref(lo), ctypes.byref(hi)),
           "nvsm_batch_plan")
    return lo.value, hi.value


def nvsm_reconstruct_batch(ctx, params, bursts, workspace, stream=None):
    """bursts: list of (frames, stf, out) tensors; frames share one dtype."""
    arr = _bursts(bursts)
    st = lib().nvsm_reconstruct_batch(ctx, ctypes.byref(params), frames_dtype(bursts[0][0]), arr, len(bursts),
                                      _ptr(workspace), workspace.numel() * workspace.element_size(),
                                      _stream(stream))
    _check(st, "nvsm_reconstruct_batch", ctx)


def nvsm_autotune(ctx, params, frames, workspace, stream=None, row_pitch=None):
    """(slots per wave, form) chosen for params after timing the candidates."""
    F, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    k, f = ctypes.c_int32(), ctypes.c_int32()
    st = lib().nvsm_autotune(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), F, H, W, pitch,
                             _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream),
                             ctypes.byref(k), ctypes.byref(f))
    _check(st, "nvsm_autotune", ctx)
    return k.value, f.value


def nvsm_set_launch(ctx, params, slots, form):
    _check(lib().nvsm_set_launch(ctx, ctypes.byref(params), int(slots), int(form)), "nvsm_set_launch", ctx)


def nvsm_tune_radius_plan(params, H, W, F, r_max):
    n = ctypes.c_size_t()
    _check(lib().nvsm_tune_radius_plan(ctypes.byref(params), H, W, F, r_max, ctypes.byref(n)),
           "nvsm_tune_radius_plan")
    return n.value


def nvsm_tune_radius(ctx, params, frames, stf, r_min, r_max, tol, workspace, stream=None, row_pitch=None):
    """(chosen R, {R: phase measure}) on the burst; see nvsm.h."""
    import math
    F, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    r = ctypes.c_int32()
    err = (ctypes.c_double * (r_max - r_min + 1))()
    st = lib().nvsm_tune_radius(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), F, H, W, pitch,
                                _ptr(stf), r_min, r_max, float(tol), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream), ctypes.byref(r),
                                ctypes.cast(err, ctypes.c_void_p))
    _check(st, "nvsm_tune_radius", ctx)
    return r.value, {r_min + i: err[i] for i in range(len(err)) if not math.isnan(err[i])}


def nvsm_stream_plan(params, H, W, group_frames):
    """(state bytes, workspace bytes)."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().nvsm_stream_plan(ctypes.byref(params), int(H), int(W), int(group_frames), ctypes.byref(a),
                                  ctypes.byref(b)), "nvsm_stream_plan")
    return a.value, b.value


def _nbytes(t):
    return t.numel() * t.element_size()


def nvsm_stream_add(ctx, params, frames, frames_before, total_frames, state, ws, stream=None, row_pitch=None):
    G, H, W = frames.shape
    pitch = _row_pitch(frames, row_pitch)
    _check(lib().nvsm_stream_add(ctx, ctypes.byref(params), _ptr(frames), frames_dtype(frames), G, H, W, pitch,
                                 int(frames_before), int(total_frames), _ptr(state), _nbytes(state), _ptr(ws),
                                 _nbytes(ws), _stream(stream)), "nvsm_stream_add", ctx)


def nvsm_stream_finish(ctx, params, H, W, stf, out, ws, stream=None):
    _check(lib().nvsm_stream_finish(ctx, ctypes.byref(params), int(H), int(W), _ptr(stf), _ptr(out), _ptr(ws),
                                    _nbytes(ws), _stream(stream)), "nvsm_stream_finish", ctx)


def nvsm_model_stf_plan(params, screens):
    """Workspace bytes of nvsm_model_stf."""
    n = ctypes.c_size_t()
    _check(lib().nvsm_model_stf_plan(ctypes.byref(params), int(screens), ctypes.byref(n)), "nvsm_model_stf_plan")
    return n.value


def nvsm_model_stf(ctx, params, d_over_r0, screens, seed, stf, ws, mean_otf=None, stream=None):
    """Model STF (device float64 [N][N]) by Monte Carlo at D/r0; mean_otf:
    optional device float64 [N][N][2]."""
    _check(lib().nvsm_model_stf(ctx, ctypes.byref(params), float(d_over_r0), int(screens), int(seed), _ptr(stf),
                                _ptr(mean_otf), _ptr(ws), _nbytes(ws), _stream(stream)), "nvsm_model_stf", ctx)


def seeing_default_params(**kw):
    sp = SeeingParams()
    _check(lib().nvsm_seeing_default_params(ctypes.byref(sp)), "nvsm_seeing_default_params")
    return _set_fields(sp, kw)


def nvsm_seeing_plan(params, sp, H, W, F):
    """(workspace bytes, cubes)."""
    n, c = ctypes.c_size_t(), ctypes.c_int32()
    _check(lib().nvsm_seeing_plan(ctypes.byref(params), ctypes.byref(sp), int(H), int(W), int(F), ctypes.byref(n),
                                  ctypes.byref(c)), "nvsm_seeing_plan")
    return n.value, c.value


def nvsm_seeing(ctx, params, sp, frames, d_over_r0, stf, ws, curves=None, stream=None):
    """Seeing by the spectral ratio.  frames: device [F][H][W] (view with a
    row pitch allowed) of int16 (12-bit data) or float32; d_over_r0: device
    float64 [1 + cubes]; stf: device float64 [N][N]; curves: optional device
    float64 [cubes][bins]."""
    F, H, W = frames.shape
    pitch = _row_pitch(frames)
    _check(lib().nvsm_seeing(ctx, ctypes.byref(params), ctypes.byref(sp), _ptr(frames), frames_dtype(frames), F, H, W,
                             pitch, _ptr(d_over_r0), _ptr(stf), _ptr(curves), _ptr(ws), _nbytes(ws),
                             _stream(stream)), "nvsm_seeing", ctx)


def nvsm_profile_enable(ctx, enable=True):
    _check(lib().nvsm_profile_enable(ctx, 1 if enable else 0), "nvsm_profile_enable", ctx)


def nvsm_profile_read(ctx):
    """{stage: (total ms, launches)} since the last read."""
    import numpy as np
    ms = np.zeros(len(STAGES), np.float64)
    cnt = np.zeros(len(STAGES), np.int64)
    _check(lib().nvsm_profile_read(ctx, ms.ctypes.data, cnt.ctypes.data, len(STAGES)), "nvsm_profile_read", ctx)
    return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}
