"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point the header declares, and
its host-only calls (parameters, planning, index sets, validation) must
agree with the oracle's independent enumeration and the paper's tiling.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1701_00581_amd as nv
from paper_1701_00581_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nvsm.h")).read()
    return sorted(set(re.findall(r"\b(nvsm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = nv.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(nv.EXPORTS)


def test_default_params():
    p = nv.default_params(128)
    assert (p.patch, p.stride, p.u_cut, p.v_radius, p.window) == (128, 64, 63, 10, 1)
    with pytest.raises(nv.NvsmError):
        nv.default_params(96)


@pytest.mark.parametrize("H,W,N,R,ny,nx", [
    (1024, 1024, 128, 10, 15, 15),
    (2160, 2560, 128, 12, 33, 39),
    (64, 64, 64, 8, 1, 1),
    (250, 300, 128, 10, 3, 4),
])
def test_plan_counts_match_oracle(H, W, N, R, ny, nx):
    p = nv.default_params(N, v_radius=R)
    info = nv.nvsm_plan(p, H, W, 100)
    assert (info.patches_y, info.patches_x, info.patches) == (ny, nx, ny * nx)
    ys, xs = oracle.tiling(H, W, N, N // 2)
    assert (len(ys), len(xs)) == (ny, nx)
    Wset, S, woff = oracle.bispectrum_set(N // 2 - 1, R)
    assert info.w_count == len(Wset) and info.s_count == len(S)
    assert info.shells == len(set((Wset ** 2).sum(1).tolist()))
    assert info.ws_reconstruct > info.ws_accumulate > 0


@pytest.mark.parametrize("N,R", [(64, 8), (128, 10), (128, 12), (64, 3)])
def test_index_sets_equal_oracle(N, R):
    p = nv.default_params(N, v_radius=R)
    Wset, S, woff = oracle.bispectrum_set(N // 2 - 1, R)
    np.testing.assert_array_equal(nv.nvsm_w_index(p), Wset)
    np.testing.assert_array_equal(nv.nvsm_bispectrum_index(p), S)


def test_invalid_parameters_are_rejected_before_anything_runs():
    L = nv.lib()
    info = nv.PlanInfo()
    for field, bad in [("patch", 96), ("stride", 0), ("stride", 200), ("u_cut", 64), ("v_radius", 0),
                       ("v_radius", 63), ("v_radius", 17), ("window", 2), ("noise_bias", 3), ("filter", -1),
                       ("stf_floor", float("nan"))]:
        p = nv.default_params(128)
        setattr(p, field, bad)
        assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_ERR_INVALID_ARG, field
    p = nv.default_params(128)
    p.phase_method = 2
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_ERR_NOT_IMPLEMENTED
    # frame counts: 1 .. the largest whose spectrum records one patch spans in 32-bit offsets
    for N, fmax in ((128, 26214), (64, 87381)):
        p = nv.default_params(N)
        for F, want in ((0, _lib.NVSM_ERR_SHAPE), (1, _lib.NVSM_OK), (fmax, _lib.NVSM_OK),
                        (fmax + 1, _lib.NVSM_ERR_SHAPE)):
            assert L.nvsm_plan(ctypes.byref(p), N, N, F, ctypes.byref(info)) == want, (N, F)
    p = nv.default_params(128)
    p.phase_method = 1
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_OK
    p.lsq_iters = 0
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_ERR_INVALID_ARG
    # photon-noise model: a positive finite gain; larger workspaces
    p = nv.default_params(128)
    assert p.photons_per_adu == 1.0
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_OK
    plain = (info.ws_accumulate, info.ws_reconstruct)
    p.noise_bias = 2
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_OK
    assert info.ws_accumulate > plain[0] and info.ws_reconstruct > plain[1]
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        p.photons_per_adu = bad
        assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 100, ctypes.byref(info)) == _lib.NVSM_ERR_INVALID_ARG
    # the streaming state then also holds the photon-noise sums: (sum,
    # compensation) of C over the half plane, and of q0 and T, per patch
    p.photons_per_adu = 4.0
    st2, ws2 = nv.nvsm_stream_plan(p, 1024, 1024, 10)
    p.noise_bias = 0
    st0, ws0 = nv.nvsm_stream_plan(p, 1024, 1024, 10)
    P = info.patches

    def up(n):
        return (n + 255) // 256 * 256
    assert st2 - st0 == up(P * 65 * 128 * 16) + up(P * 16)
    assert ws2 > ws0
    # model STF workspace: partial sums of min(pairs, 256) workgroups over the half plane
    p = nv.default_params(128)
    assert nv.nvsm_model_stf_plan(p, 1000) == 256 * 65 * 128 * 12
    assert nv.nvsm_model_stf_plan(p, 8) == 4 * 65 * 128 * 12
    for bad in (0, 7, -2, (1 << 24) + 2):
        n = ctypes.c_size_t()
        assert L.nvsm_model_stf_plan(ctypes.byref(p), bad, ctypes.byref(n)) == _lib.NVSM_ERR_INVALID_ARG
    assert L.nvsm_model_stf(None, ctypes.byref(p), 10.0, 8, 1, None, None, None, 0, None) == _lib.NVSM_ERR_INVALID_ARG
    # seeing: defaults, sizes and validation
    sp = nv.seeing_default_params()
    assert (sp.screens, sp.points, sp.bins) == (1000, 40, 12)
    ws, cubes = nv.nvsm_seeing_plan(p, sp, 2160, 2560, 100)
    assert cubes == 16 * 20
    box = (12 + 3) * (2 * 12 + 5)
    assert ws == (256 * 65 * 128 * 12 + 40 * 128 * 128 * 24 + 320 * 5 * box * 12)   # 5 frame groups of 20
    n, c = ctypes.c_size_t(), ctypes.c_int32()
    for field, bad in [("points", 2), ("points", 257), ("bins", 1), ("bins", 33), ("d_over_r0_min", 0.0),
                       ("d_over_r0_max", 1.0), ("screens", 3)]:
        spb = nv.seeing_default_params()
        setattr(spb, field, bad)
        assert L.nvsm_seeing_plan(ctypes.byref(p), ctypes.byref(spb), 2160, 2560, 100, ctypes.byref(n),
                                  ctypes.byref(c)) == _lib.NVSM_ERR_INVALID_ARG, field
    assert L.nvsm_seeing_plan(ctypes.byref(p), ctypes.byref(sp), 2160, 2560, 1, ctypes.byref(n),
                              ctypes.byref(c)) == _lib.NVSM_ERR_SHAPE
    assert L.nvsm_seeing_plan(ctypes.byref(p), ctypes.byref(sp), 100, 2560, 10, ctypes.byref(n),
                              ctypes.byref(c)) == _lib.NVSM_ERR_SHAPE
    p = nv.default_params(128)
    assert L.nvsm_plan(ctypes.byref(p), 100, 1024, 100, ctypes.byref(info)) == _lib.NVSM_ERR_SHAPE
    assert L.nvsm_plan(ctypes.byref(p), 1024, 1024, 0, ctypes.byref(info)) == _lib.NVSM_ERR_SHAPE
    assert L.nvsm_plan(None, 1024, 1024, 10, ctypes.byref(info)) == _lib.NVSM_ERR_INVALID_ARG
    # wrong buffer length for the index export
    buf = np.zeros(8, np.int32)
    assert L.nvsm_bispectrum_index(ctypes.byref(p), buf.ctypes.data, 2) == _lib.NVSM_ERR_SHAPE
    # compute calls reject a null context
    assert L.nvsm_reconstruct(None, ctypes.byref(p), None, 0, 1, 128, 128, 128, None, None, None, 0,
                              None) == _lib.NVSM_ERR_INVALID_ARG
    assert L.nvsm_accumulate(None, ctypes.byref(p), None, 0, 1, 128, 128, 128, None, None, None, None,
                             None, 0, None) == _lib.NVSM_ERR_INVALID_ARG


def test_parameter_helpers_reject_unknown_fields():
    with pytest.raises(TypeError):
        nv.default_params(128, phase_methd=1)
    with pytest.raises(TypeError):
        nv.seeing_default_params(screen=10)
    assert nv.default_params(128, lsq_iters=3).lsq_iters == 3


def test_frame_layouts_other_than_F_H_pitch_are_rejected_before_any_call():
    """The C ABI reads frames as [F][H][pitch]: views that keep that layout
    pass their row pitch; transposed, x-strided or frame-strided views are
    refused by the binding before the library is called."""
    import torch
    base = torch.zeros(3, 70, 90, dtype=torch.int16)
    assert _lib._row_pitch(base) == 90
    assert _lib._row_pitch(base[:, :, :81]) == 90          # crop in x: pitch 90
    assert _lib._row_pitch(base[1:, :, :]) == 90           # a frame range
    assert _lib._row_pitch(base[:, ::2, :]) == 180         # every other row: pitch 180
    for bad in (base.transpose(1, 2), base[:, :, ::2], base[::2], base[:, :40, :]):
        with pytest.raises(ValueError):
            _lib._row_pitch(bad)
    p = nv.default_params(64)
    with pytest.raises(ValueError):
        nv.nvsm_accumulate(None, p, base.transpose(1, 2), None, None, None, None, None)
    assert _lib._row_pitch(base.transpose(1, 2), row_pitch=90) == 90


def test_status_strings():
    for s in range(-6, 1):
        assert nv.status_string(s)
    assert nv.status_string(-3) == "workspace too small"


def test_workspace_sizes_scale_with_the_burst():
    p = nv.default_params(128, v_radius=12)
    a = nv.nvsm_plan(p, 2160, 2560, 100)
    b = nv.nvsm_plan(p, 2160, 2560, 50)
    assert a.ws_accumulate > b.ws_accumulate
    # spectra (P F N/2 N complex64) dominate the accumulation workspace
    assert a.ws_accumulate >= 1287 * 100 * 64 * 128 * 8
    assert a.ws_reconstruct >= a.ws_accumulate + 1287 * a.s_count * 8


def test_tune_radius_plan_is_the_crop_workspace_at_r_max():
    """The tuner's workspace is that of nvsm_reconstruct on the burst's
    central crop of at most 512 x 512 px at r_max (host call)."""
    import paper_1701_00581_amd as nv
    p = nv.default_params(128, v_radius=8)
    big = nv.nvsm_tune_radius_plan(p, 2160, 2560, 100, 12)
    q = nv.default_params(128, v_radius=12)
    assert big == nv.nvsm_plan(q, 512, 512, 100).ws_reconstruct
    small = nv.nvsm_tune_radius_plan(p, 300, 400, 30, 10)
    q.v_radius = 10
    assert small == nv.nvsm_plan(q, 300, 400, 30).ws_reconstruct
    with pytest.raises(nv.NvsmError):
        nv.nvsm_tune_radius_plan(p, 2160, 2560, 100, 64)     # r_max beyond the allowed radii
