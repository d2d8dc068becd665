"""Streaming accumulation (frames arriving in groups) through the C ABI.

One group holding the whole burst reproduces nvsm_accumulate and
nvsm_reconstruct bit for bit.  Several groups change only where the running
sums are folded, so the results stay within the parity tolerances of the
FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import (BISPEC_TOL, MOSAIC_TOL, POWER_TOL, abs_bispectrum, as_complex, bispec_errors, burst,
                         cube, oparams, say, stf, to_device)

pytestmark = pytest.mark.gpu

H, W, F = 384, 448, 30


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    return torch


@pytest.fixture(scope="module")
def setup(torch_cuda):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    fr = burst("burst1024", F=F, H=H, W=W)
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1)
    d = to_device(fr)
    st = torch.from_numpy(stf("burst1024", screens=100)).cuda()
    info = nv.nvsm_plan(p, H, W, F)
    ctx = nv.nvsm_create(0)
    # whole-burst reference: accumulate (bispectrum, power) and reconstruct
    ref = {}
    ref["power"] = torch.empty((info.patches, 128, 128), device="cuda")
    ref["mean"] = torch.empty((info.patches, 2, 2), device="cuda")
    ref["mu"] = torch.empty(info.patches, device="cuda")
    ref["bis"] = torch.empty((info.patches, info.s_count, 2), device="cuda")
    nv.nvsm_accumulate(ctx, p, d, ref["power"], ref["mean"], ref["mu"], ref["bis"],
                       torch.empty(info.ws_accumulate, dtype=torch.uint8, device="cuda"))
    ref["img"] = torch.empty((H, W), device="cuda")
    nv.nvsm_reconstruct(ctx, p, d, st, ref["img"], torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    yield dict(fr=fr, p=p, d=d, stf=st, info=info, ctx=ctx, ref=ref)
    nv.nvsm_destroy(ctx)


def _stream(nv, torch, s, groups):
    p, d, info = s["p"], s["d"], s["info"]
    state_b, ws_b = nv.nvsm_stream_plan(p, H, W, max(groups))
    state = torch.empty(state_b, dtype=torch.uint8, device="cuda")
    state.fill_(0xFF)                      # the first group must not read it
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    f0 = 0
    for i, g in enumerate(groups):
        last = i == len(groups) - 1
        nv.nvsm_stream_add(s["ctx"], p, d[f0:f0 + g], f0, F if last else 0, state, ws)
        f0 += g
    img = torch.full((H, W), float("nan"), device="cuda")
    nv.nvsm_stream_finish(s["ctx"], p, H, W, s["stf"], img, ws)
    torch.cuda.synchronize()
    bis = ws[: info.patches * info.s_count * 8].view(torch.float32).view(info.patches, info.s_count, 2)
    return img, bis


def test_stream_one_group_is_exact(torch_cuda, setup):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    img, bis = _stream(nv, torch, setup, [F])
    same_b = torch.equal(bis, setup["ref"]["bis"])
    same_i = torch.equal(img, setup["ref"]["img"])
    say(f"[stream] one group: bispectrum identical={same_b}, image identical={same_i}")
    assert same_b and same_i


def test_stream_groups_within_tolerance(torch_cuda, setup):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    groups = [7, 7, 9, 6, 1]
    assert sum(groups) == F
    img, bis = _stream(nv, torch, setup, groups)
    ref = setup["ref"]
    b = as_complex(bis)
    br = as_complex(ref["bis"])
    rel = float(np.linalg.norm(b - br) / np.linalg.norm(br))
    ri = ref["img"].cpu().numpy()
    gi = img.cpu().numpy()
    core = (slice(64, H - 64), slice(64, W - 64))
    irel = float(np.abs(gi[core] - ri[core]).max() / ri[core].std())
    say(f"[stream] groups {groups}: bispectrum vs whole-burst {rel:.2e}, image {irel:.2e}")
    assert rel < BISPEC_TOL
    assert irel < MOSAIC_TOL
    # against the FP64 oracle, two patches
    op = oparams(setup["p"])
    wv = nv.nvsm_bispectrum_index(setup["p"])
    for k in (0, setup["info"].patches - 1):
        c = cube(setup["fr"], setup["p"], k)
        I, _ = oracle.patch_spectra(c, op.window)
        bo = oracle.bispectrum(I, wv)
        A = abs_bispectrum(I, wv)
        nrm, mx = bispec_errors(b[k], bo, A)
        say(f"[stream] patch {k} vs oracle: B norm {nrm:.2e} B/A max {mx:.2e}")
        assert nrm < BISPEC_TOL and mx < BISPEC_TOL


def test_stream_least_squares_one_group_is_exact(torch_cuda, setup):
    """With least-squares phase steps (phase_method 1) the stream's finish
    runs the same solve: one group gives nvsm_reconstruct's image bit for bit."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1, phase_method=1, lsq_iters=4)
    s = dict(setup, p=p)
    img, _ = _stream(nv, torch, s, [F])
    ref = torch.empty((H, W), device="cuda")
    info = nv.nvsm_plan(p, H, W, F)
    nv.nvsm_reconstruct(setup["ctx"], p, setup["d"], setup["stf"], ref,
                        torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    same = torch.equal(img, ref)
    say(f"[stream] least squares, one group: image identical={same}")
    assert torch.isfinite(img).all() and same


def test_stream_errors(torch_cuda, setup):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = setup["p"]
    state_b, ws_b = nv.nvsm_stream_plan(p, H, W, 5)
    state = torch.empty(state_b, dtype=torch.uint8, device="cuda")
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    small = torch.empty(state_b // 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(nv.NvsmError) as e:
        nv.nvsm_stream_add(setup["ctx"], p, setup["d"][:5], 0, 0, small, ws)
    assert e.value.status == -3
    small = torch.empty(ws_b - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(nv.NvsmError) as e:
        nv.nvsm_stream_add(setup["ctx"], p, setup["d"][:5], 0, 0, state, small)
    assert e.value.status == -3
    with pytest.raises(nv.NvsmError):               # total must be frames_before + G
        nv.nvsm_stream_add(setup["ctx"], p, setup["d"][:5], 0, 3, state, ws)


def test_stream_launch_choice_may_change_mid_burst(torch_cuda, setup):
    """The streaming calls keep 16 slots per wave whatever the launch choice
    (their running sums are stored in that kernel's lane order): switching
    to 24 slots and the persistent form between two groups of a burst gives
    the same bits as keeping the default."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p, d = setup["p"], setup["d"]
    groups = [11, 19]
    ref_img, ref_bis = _stream(nv, torch, setup, groups)
    ref_bis = ref_bis.clone()
    ctx = nv.nvsm_create(0)
    try:
        state_b, ws_b = nv.nvsm_stream_plan(p, H, W, max(groups))
        state = torch.empty(state_b, dtype=torch.uint8, device="cuda")
        ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
        nv.nvsm_stream_add(ctx, p, d[:11], 0, 0, state, ws)
        nv.nvsm_set_launch(ctx, p, 24, 1)
        nv.nvsm_stream_add(ctx, p, d[11:], 11, F, state, ws)
        img = torch.full((H, W), float("nan"), device="cuda")
        nv.nvsm_stream_finish(ctx, p, H, W, setup["stf"], img, ws)
        torch.cuda.synchronize()
        info = setup["info"]
        bis = ws[: info.patches * info.s_count * 8].view(torch.float32).view(info.patches, info.s_count, 2)
        same_b, same_i = torch.equal(bis, ref_bis), torch.equal(img, ref_img)
        say(f"[stream] launch choice changed mid-burst: bispectrum identical={same_b}, image identical={same_i}")
        assert same_b and same_i
    finally:
        nv.nvsm_destroy(ctx)


def test_persistent_form_on_two_streams(torch_cuda, setup):
    """The persistent bispectrum form on two streams at once, one context,
    two workspaces: each call's work-queue counters live in its own
    workspace, so both equal the per-item form's result bit for bit."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p, d, info = setup["p"], setup["d"], setup["info"]
    ctx = nv.nvsm_create(0)
    try:
        nv.nvsm_set_launch(ctx, p, 16, 1)
        outs = []
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        bufs = []
        for _ in streams:
            bufs.append(dict(power=torch.empty((info.patches, 128, 128), device="cuda"),
                             mean=torch.empty((info.patches, 2, 2), device="cuda"),
                             mu=torch.empty(info.patches, device="cuda"),
                             bis=torch.full((info.patches, info.s_count, 2), float("nan"), device="cuda"),
                             ws=torch.empty(info.ws_accumulate, dtype=torch.uint8, device="cuda")))
        torch.cuda.synchronize()
        for rep in range(3):
            for st, b in zip(streams, bufs):
                with torch.cuda.stream(st):
                    nv.nvsm_accumulate(ctx, p, d, b["power"], b["mean"], b["mu"], b["bis"], b["ws"],
                                       stream=st)
            torch.cuda.synchronize()
            for i, b in enumerate(bufs):
                same = torch.equal(b["bis"], setup["ref"]["bis"])
                say(f"[queue] repeat {rep} stream {i}: identical to the per-item form={same}")
                assert same
                b["bis"].fill_(float("nan"))
            torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)


def test_stream_photon_noise(torch_cuda, setup):
    """noise_bias 2 in the streaming calls (a low photon level, so the terms
    are large): one group gives nvsm_accumulate's corrected bispectrum and
    nvsm_reconstruct's image bit for bit; five uneven groups stay within the
    tolerances of the whole burst and of the oracle's corrected bispectrum."""
    import dataclasses
    import paper_1701_00581_amd as nv
    import synth
    torch = torch_cuda
    photons = 40.0
    say(f"case stream photon noise: burst1024 scene at {photons:.0f} photons/px, {H}x{W} F={F}, N=128, R=10")
    cfg = dataclasses.replace(synth.CONFIGS["burst1024"], photons=photons, index=91)
    fr = np.ascontiguousarray(synth.make_burst(cfg, frames=F)[:, :H, :W])
    gain = photons / 2048.0
    p = nv.default_params(128, v_radius=10, noise_bias=2, photons_per_adu=gain, filter=1)
    d = to_device(fr)
    info = nv.nvsm_plan(p, H, W, F)
    ctx = setup["ctx"]
    bis_ref = torch.empty((info.patches, info.s_count, 2), device="cuda")
    nv.nvsm_accumulate(ctx, p, d, torch.empty((info.patches, 128, 128), device="cuda"),
                       torch.empty((info.patches, 2, 2), device="cuda"), torch.empty(info.patches, device="cuda"),
                       bis_ref, torch.empty(info.ws_accumulate, dtype=torch.uint8, device="cuda"))
    img_ref = torch.empty((H, W), device="cuda")
    nv.nvsm_reconstruct(ctx, p, d, setup["stf"], img_ref,
                        torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    s = dict(setup, p=p, d=d, fr=fr)
    img, bis = _stream(nv, torch, s, [F])
    same_b = torch.equal(bis, bis_ref)
    same_i = torch.equal(img, img_ref)
    say(f"[stream photon] one group: bispectrum identical={same_b}, image identical={same_i}")
    assert same_b and same_i
    groups = [7, 7, 9, 6, 1]
    img, bis = _stream(nv, torch, s, groups)
    b = as_complex(bis)
    br = as_complex(bis_ref)
    rel = float(np.linalg.norm(b - br) / np.linalg.norm(br))
    say(f"[stream photon] groups {groups}: bispectrum vs whole-burst {rel:.2e}")
    assert rel < BISPEC_TOL and torch.isfinite(img).all()
    op = oparams(p)
    op0 = oparams(nv.default_params(128, v_radius=10, filter=1))
    S = nv.nvsm_bispectrum_index(p)
    for k in (0, info.patches - 1):
        c = cube(fr, p, k)
        acc = oracle.accumulate_patch(c, op, S)
        raw = oracle.accumulate_patch(c, op0, S)
        I, _ = oracle.patch_spectra(c, op.window)
        A = abs_bispectrum(I, S)
        nrm, mx = bispec_errors(b[k], acc["B"], A)
        moved = float(np.max(np.abs(acc["B"] - raw["B"]) / A))
        say(f"[stream photon] patch {k} vs oracle: B norm {nrm:.2e} B/A max {mx:.2e} (correction B/A up to {moved:.2e})")
        assert nrm < BISPEC_TOL and mx < BISPEC_TOL
        assert moved > 100 * BISPEC_TOL
