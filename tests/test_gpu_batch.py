"""Batched reconstruction of uneven bursts, its graph replay and the launch
tuning, through the C ABI.

Every value of the batched path is computed by the same arithmetic in the
same order as for the burst alone, so the checks here are bit-for-bit
against nvsm_reconstruct (which the oracle parity tests pin).
"""
import dataclasses

import numpy as np
import pytest

import synth
from gpu_helpers import say, to_device

pytestmark = pytest.mark.gpu

# (H, W, F, row padding): uneven shapes and frame counts, one with a row
# pitch wider than the frame (no vector loads for the whole batch)
SHAPES = [(256, 320, 23, 0), (300, 256, 37, 0), (260, 270, 12, 6), (256, 256, 41, 0)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    return torch


def _params():
    import paper_1701_00581_amd as nv
    return nv.default_params(64, v_radius=8, noise_bias=1, filter=1)


@pytest.fixture(scope="module")
def bursts(torch_cuda):
    torch = torch_cuda
    out = []
    for i, (H, W, F, pad) in enumerate(SHAPES):
        cfg = dataclasses.replace(synth.CONFIGS["burst1024"], name=f"batch{i}", index=40 + i, H=H, W=W, F=F,
                                  patch=64, v_radius=8)
        fr = synth.make_burst(cfg)
        d = to_device(fr)
        if pad:
            wide = torch.zeros((F, H, W + pad), dtype=d.dtype, device=d.device)
            wide[:, :, :W] = d
            d = wide[:, :, :W]
        stf = torch.from_numpy(synth.stf_table(cfg, screens=40, patch=64)).cuda()
        out.append((d, stf))
    return out


def _alone(torch, p, bursts):
    import paper_1701_00581_amd as nv
    ctx = nv.nvsm_create(0)
    imgs = []
    for d, stf in bursts:
        F, H, W = d.shape
        info = nv.nvsm_plan(p, H, W, F)
        ws = torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda")
        img = torch.empty((H, W), dtype=torch.float32, device="cuda")
        nv.nvsm_reconstruct(ctx, p, d, stf, img, ws)
        imgs.append(img)
    torch.cuda.synchronize()
    nv.nvsm_destroy(ctx)
    return imgs


def _batch(torch, p, bursts, ws_bytes, ctx=None):
    import paper_1701_00581_amd as nv
    own = ctx is None
    if own:
        ctx = nv.nvsm_create(0)
    outs = [torch.full((d.shape[1], d.shape[2]), float("nan"), device="cuda") for d, _ in bursts]
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    nv.nvsm_reconstruct_batch(ctx, p, [(d, stf, o) for (d, stf), o in zip(bursts, outs)], ws)
    torch.cuda.synchronize()
    if own:
        nv.nvsm_destroy(ctx)
    return outs


def test_batch_equals_alone(torch_cuda, bursts):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = _params()
    ref = _alone(torch, p, bursts)
    shapes = [tuple(d.shape) for d, _ in bursts]
    ws_min, ws_all = nv.nvsm_batch_plan(p, shapes)
    say(f"[batch] workspace one-per-group {ws_min} B, all-in-one {ws_all} B")
    assert ws_all >= ws_min > 0
    for label, wsb in (("one group", ws_all), ("one burst per group", ws_min)):
        got = _batch(torch, p, bursts, wsb)
        for i, (g, r) in enumerate(zip(got, ref)):
            same = torch.equal(g, r)
            say(f"[batch] {label}: burst {i} {tuple(g.shape)} identical={same}")
            assert torch.isfinite(g).all()
            assert same


def test_batch_photon_noise_equals_alone(torch_cuda, bursts):
    """With the photon-noise terms (noise_bias 2) as well."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = _params()
    p.noise_bias = 2
    p.photons_per_adu = synth.CONFIGS["burst1024"].photons / 2048.0
    ref = _alone(torch, p, bursts)
    _, ws_all = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _ in bursts])
    got = _batch(torch, p, bursts, ws_all)
    for i, (g, r) in enumerate(zip(got, ref)):
        same = torch.equal(g, r)
        say(f"[batch photon] burst {i} identical={same}")
        assert torch.isfinite(g).all()
        assert same


def test_batch_least_squares_equals_alone(torch_cuda, bursts):
    """With least-squares phase steps (phase_method 1): their fixed-point
    sums make the batched result bit-identical as well."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = _params()
    p.phase_method = 1
    p.lsq_iters = 5
    ref = _alone(torch, p, bursts)
    _, ws_all = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _ in bursts])
    got = _batch(torch, p, bursts, ws_all)
    for i, (g, r) in enumerate(zip(got, ref)):
        same = torch.equal(g, r)
        say(f"[batch lsq] burst {i} identical={same}")
        assert torch.isfinite(g).all()
        assert same


def test_batch_workspace_errors(torch_cuda, bursts):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = _params()
    ws_min, _ = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _ in bursts])
    with pytest.raises(nv.NvsmError) as e:
        _batch(torch, p, bursts, ws_min - 256)
    assert e.value.status == -3
    with pytest.raises(nv.NvsmError):
        nv.nvsm_batch_plan(p, [(0, 256, 256)])


def test_batch_graph_replay(torch_cuda, bursts):
    """The batched call captured in a HIP graph and replayed three times,
    with eager work between the replays: every replay equals the eager
    result bit for bit."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = _params()
    ctx = nv.nvsm_create(0)
    nv.nvsm_prepare(ctx, p)
    _, ws_all = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _ in bursts])
    eager = _batch(torch, p, bursts, ws_all, ctx)
    outs = [torch.zeros_like(e) for e in eager]
    ws = torch.empty(ws_all, dtype=torch.uint8, device="cuda")
    args = [(d, stf, o) for (d, stf), o in zip(bursts, outs)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):            # warm-up on the capture stream
        nv.nvsm_reconstruct_batch(ctx, p, args, ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        nv.nvsm_reconstruct_batch(ctx, p, args, ws)
    for r in range(3):
        for o in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")          # eager work between replays
        (junk * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        same = all(torch.equal(o, e) for o, e in zip(outs, eager))
        say(f"[graph] replay {r}: identical={same}")
        assert same
    del g
    nv.nvsm_destroy(ctx)


def test_launch_choices_identical_and_autotune(torch_cuda):
    """Every bispectrum launch candidate (16 or 24 slots, per-item grid or
    persistent work queue) gives the same bits; the tuner picks one."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    cfg = synth.CONFIGS["burst1024"]
    fr = synth.make_burst(cfg, frames=20)[:, :384, :448].copy()
    d = to_device(fr)
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1)
    F, H, W = d.shape
    info = nv.nvsm_plan(p, H, W, F)
    results = {}
    for slots in (16, 24):
        for form in (0, 1):
            ctx = nv.nvsm_create(0)
            nv.nvsm_set_launch(ctx, p, slots, form)
            s_pow = torch.empty((info.patches, 128, 128), device="cuda")
            s_mean = torch.empty((info.patches, 2, 2), device="cuda")
            s_mu = torch.empty(info.patches, device="cuda")
            bis = torch.full((info.patches, info.s_count, 2), float("nan"), device="cuda")
            ws = torch.empty(info.ws_accumulate, dtype=torch.uint8, device="cuda")
            nv.nvsm_accumulate(ctx, p, d, s_pow, s_mean, s_mu, bis, ws)
            torch.cuda.synchronize()
            assert torch.isfinite(bis).all()
            results[(slots, form)] = bis
            nv.nvsm_destroy(ctx)
    base = results[(16, 0)]
    for k, v in results.items():
        same = torch.equal(v, base)
        say(f"[tune] slots {k[0]} form {k[1]}: identical={same}")
        assert same
    ctx = nv.nvsm_create(0)
    ws = torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda")
    choice = nv.nvsm_autotune(ctx, p, d, ws)
    say(f"[tune] autotune chose slots {choice[0]} form {choice[1]}")
    assert choice in results
    bis = torch.full_like(base, float("nan"))
    nv.nvsm_accumulate(ctx, p, d, torch.empty((info.patches, 128, 128), device="cuda"),
                       torch.empty((info.patches, 2, 2), device="cuda"), torch.empty(info.patches, device="cuda"),
                       bis, torch.empty(info.ws_accumulate, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(bis, base)
    nv.nvsm_destroy(ctx)


# Two (N, R) classes of uneven bursts for the batch-versus-oracle test: the
# four N = 64 bursts above (R = 8) and two N = 128 bursts (R = 12), one of
# them with 100 frames.
CLASS128 = [(256, 256, 100, 0), (300, 260, 57, 0)]


def _np_burst(i, H, W, F, patch, v_radius, screens):
    cfg = dataclasses.replace(synth.CONFIGS["burst1024"], name=f"batch{i}", index=40 + i, H=H, W=W, F=F,
                              patch=patch, v_radius=v_radius)
    return synth.make_burst(cfg), synth.stf_table(cfg, screens=screens, patch=patch)


@pytest.mark.timeout(900)
def test_batch_against_the_oracle(torch_cuda):
    """nvsm_reconstruct_batch on six uneven bursts in two (N, R) classes, one
    call per class with every burst in one launch group, against the FP64
    oracle: the whole mosaic of every burst, and the bispectrum, modulus and
    phases of the first and last patch of every burst (read from the
    workspace, whose layout the header documents)."""
    import oracle
    import oracle_pool
    import paper_1701_00581_amd as nv
    from gpu_helpers import (BISPEC_TOL, MOSAIC_TOL, PHASE_RMS_TOL, abs_bispectrum, as_complex, bispec_errors,
                             oparams, phase_rms, reconstruct_views)
    torch = torch_cuda
    classes = [(64, 8, [(i, *s) for i, s in enumerate(SHAPES)], 40),
               (128, 12, [(10 + i, *s) for i, s in enumerate(CLASS128)], 100)]
    for N, R, members, screens in classes:
        p = nv.default_params(N, v_radius=R, noise_bias=1, filter=1)
        say(f"case batch vs oracle: N {N} R {R}, bursts {[m[1:4] for m in members]}")
        host, dev, outs = [], [], []
        for i, H, W, F, pad in members:
            fr, st = _np_burst(i, H, W, F, N, R, screens)
            host.append((fr, st))
            d = to_device(fr)
            if pad:
                wide = torch.zeros((F, H, W + pad), dtype=d.dtype, device=d.device)
                wide[:, :, :W] = d
                d = wide[:, :, :W]
            outs.append(torch.full((H, W), float("nan"), device="cuda"))
            dev.append((d, torch.from_numpy(st).cuda(), outs[-1]))
        _, ws_all = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _, _ in dev])
        ws = torch.empty(ws_all, dtype=torch.uint8, device="cuda")
        ctx = nv.nvsm_create(0)
        try:
            nv.nvsm_reconstruct_batch(ctx, p, dev, ws)
            torch.cuda.synchronize()
        finally:
            nv.nvsm_destroy(ctx)
        infos = [nv.nvsm_plan(p, H, W, F) for _, H, W, F, _ in members]
        P = sum(int(x.patches) for x in infos)
        v = reconstruct_views(ws, P, N, infos[0].w_count, infos[0].s_count)
        B = as_complex(v["bispec"])
        ph = as_complex(v["phasor"])
        amp = v["amp"].cpu().numpy()
        imgs = [o.cpu().numpy() for o in outs]
        Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
        op = oparams(p)
        patch0 = 0
        for (i, H, W, F, pad), info, (fr, st), g in zip(members, infos, host, imgs):
            last = int(info.patches) - 1
            keep = [(0, 0), divmod(last, int(info.patches_x))]
            ref = oracle_pool.reconstruct(fr, op, st, keep=keep, say=say)
            for k, t in zip((0, last), keep):
                o = ref["tiles"][t]
                ys, xs = ref["ys"], ref["xs"]
                c = fr[:, ys[t[0]]:ys[t[0]] + N, xs[t[1]]:xs[t[1]] + N].astype(np.float64)
                I, _ = oracle.patch_spectra(c, op.window)
                nerr, aerr = bispec_errors(B[patch0 + k], o["B"], abs_bispectrum(I, S))
                rms, mx = phase_rms(ph[patch0 + k], o["phasor"])
                a_err = np.max(np.abs(amp[patch0 + k] - o["amp"])) / np.max(o["amp"])
                say(f"[batch vs oracle] N {N} burst {H}x{W}x{F} patch {k}: B norm {nerr:.2e} B/A max {aerr:.2e} "
                    f"amp {a_err:.2e} phase rms {rms:.2e}")
                assert nerr <= BISPEC_TOL and aerr <= BISPEC_TOL
                assert a_err <= 1e-4 and rms <= PHASE_RMS_TOL
            o = ref["image"]
            sl = np.s_[1:, 1:]
            merr = np.linalg.norm(g[sl] - o[sl]) / np.linalg.norm(o[sl] - o[sl].mean())
            say(f"[batch vs oracle] N {N} burst {H}x{W}x{F}: mosaic {merr:.2e}")
            assert np.isfinite(g).all() and merr <= MOSAIC_TOL
            patch0 += int(info.patches)
