"""The whole 1024x1024 x 100-frame burst (15 x 15 patches of 128, R = 10)
through nvsm_reconstruct against the FP64 oracle run on every patch: the
whole mosaic interior, and the bispectrum and phases of patches on every
side of the grid, the clamped last row and column included."""
import numpy as np
import pytest

import oracle
from gpu_helpers import (BISPEC_TOL, MOSAIC_TOL, PHASE_RMS_TOL, abs_bispectrum, as_complex, bispec_errors, burst,
                         cube, oparams, phase_rms, reconstruct_views, say, stf, to_device)
import oracle_pool

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_burst1024_full_mosaic_against_the_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    say("case burst1024 full: nvsm_reconstruct vs the oracle on all 225 patches")
    fr = burst("burst1024")
    F, H, W = fr.shape
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1)
    st = stf("burst1024", screens=100)
    ctx = nv.nvsm_create(0)
    try:
        info = nv.nvsm_plan(p, H, W, F)
        assert (info.patches_y, info.patches_x) == (15, 15)
        ws = torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda")
        img = torch.full((H, W), float("nan"), device="cuda")
        nv.nvsm_reconstruct(ctx, p, to_device(fr), torch.from_numpy(st).cuda(), img, ws)
        torch.cuda.synchronize()
        v = reconstruct_views(ws, info.patches, 128, info.w_count, info.s_count)
        g_img = img.cpu().numpy()
        B = as_complex(v["bispec"])
        ph = as_complex(v["phasor"])
        amp = v["amp"].cpu().numpy()
    finally:
        nv.nvsm_destroy(ctx)
    assert np.isfinite(g_img).all()
    # corners, edge middles (the last row and column clamped flush) and the centre
    ks = [0, 7, 14, 105, 112, 119, 210, 217, 224]
    keep = [divmod(k, 15) for k in ks]
    op = oparams(p)
    ref = oracle_pool.reconstruct(fr, op, st, keep=keep, say=say)
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    for k, t in zip(ks, keep):
        o = ref["tiles"][t]
        I, _ = oracle.patch_spectra(cube(fr, p, k), op.window)
        nerr, aerr = bispec_errors(B[k], o["B"], abs_bispectrum(I, S))
        rms, mx = phase_rms(ph[k], o["phasor"])
        a_err = np.max(np.abs(amp[k] - o["amp"])) / np.max(o["amp"])
        say(f"[burst1024] patch {k} {t}: B norm {nerr:.2e} B/A max {aerr:.2e} amp {a_err:.2e} "
            f"phase rms {rms:.2e} max {mx:.2e}")
        assert nerr <= BISPEC_TOL and aerr <= BISPEC_TOL
        assert a_err <= 1e-4
        assert rms <= PHASE_RMS_TOL
    o = ref["image"]
    sl = np.s_[64:H - 64, 64:W - 64]
    merr = np.linalg.norm(g_img[sl] - o[sl]) / np.linalg.norm(o[sl] - o[sl].mean())
    full = np.linalg.norm(g_img[1:, 1:] - o[1:, 1:]) / np.linalg.norm(o[1:, 1:] - o[1:, 1:].mean())
    say(f"[burst1024] mosaic interior {merr:.2e}, whole frame but row/col 0 {full:.2e}")
    assert merr <= MOSAIC_TOL and full <= MOSAIC_TOL
    assert np.all(g_img[0, :] == 0) and np.all(g_img[:, 0] == 0)
