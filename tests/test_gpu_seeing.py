"""Seeing by the spectral ratio on the GPU: against the FP64 oracle on the
same frames and random numbers, and the estimate for bursts made by the
test generator at a known D/r0."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    return torch


def _gpu_seeing(torch, fr, N, sp, window=1):
    import paper_1701_00581_amd as nv
    p = nv.default_params(N, window=window)
    F, H, W = fr.shape
    ws_b, cubes = nv.nvsm_seeing_plan(p, sp, H, W, F)
    ctx = nv.nvsm_create(0)
    try:
        x = torch.full((1 + cubes,), float("nan"), dtype=torch.float64, device="cuda")
        stf = torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda")
        curves = torch.full((cubes, sp.bins), float("nan"), dtype=torch.float64, device="cuda")
        ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
        nv.nvsm_seeing(ctx, p, sp, to_device(fr), x, stf, ws, curves=curves)
        torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)
    return x.cpu().numpy(), stf.cpu().numpy(), curves.cpu().numpy()


@pytest.mark.parametrize("window", [1, 0])
def test_seeing_matches_oracle(torch_cuda, window):
    """256 x 384 crop (6 cubes), 21 frames (odd: a ragged frame group), 8
    model points of 16 screens, 8 annuli."""
    import paper_1701_00581_amd as nv
    say(f"case seeing parity: 256x384 F=21 N=128 J=8 K=16 Q=8 window={window}")
    cfg = dataclasses.replace(synth.CONFIGS["burst1024"], index=310, H=256, W=384)
    fr = synth.make_burst(cfg, frames=21)
    sp = nv.seeing_default_params(screens=16, points=8, d_over_r0_min=5.0, d_over_r0_max=40.0, bins=8, seed=77)
    x, S, curves = _gpu_seeing(torch_cuda, fr, 128, sp, window)
    o = oracle.seeing(fr.astype(np.float64), 128, window, 16, 77, 5.0, 40.0, 8, 8)
    cerr = np.max(np.abs(curves - o["curves"]))
    xerr = np.max(np.abs(x[1:] / o["d_over_r0_cubes"] - 1.0))
    say(f"[seeing] curves max |diff| {cerr:.2e}; D/r0 per cube rel {xerr:.2e}; burst GPU {x[0]:.4f} oracle "
        f"{o['d_over_r0']:.4f}")
    assert cerr < 1e-4
    assert xerr < 2e-3 and abs(x[0] / o["d_over_r0"] - 1.0) < 2e-3
    # the model STF at the GPU's estimate, against the oracle's Monte Carlo there (model point J)
    _, So = oracle.model(128, float(x[0]), 16, 77, 8)
    nrm = np.linalg.norm(S - So) / np.linalg.norm(So)
    say(f"[seeing] STF at the estimate: normwise {nrm:.2e}")
    assert S[0, 0] == pytest.approx(1.0, abs=1e-12) and nrm < 1e-4


@pytest.mark.parametrize("name", ["burst1024", "burst2560"])
def test_seeing_of_generated_bursts(torch_cuda, name):
    """512 x 512 bursts of 100 frames from the test generator (D/r0 15 and
    20), default settings (40 model points of 1000 screens): the estimate
    lies within 15 % of the generator's D/r0 (measured 2-12 % low on the
    same kind of bursts with the oracle's procedure)."""
    import paper_1701_00581_amd as nv
    cfg = dataclasses.replace(synth.CONFIGS[name], index=320, H=512, W=512)
    fr = synth.make_burst(cfg, frames=100)
    x, S, _ = _gpu_seeing(torch_cuda, fr, 128, nv.seeing_default_params())
    say(f"[seeing] {name}: generator D/r0 {cfg.d_over_r0}, estimate {x[0]:.2f} (cubes {np.round(x[1:], 1)})")
    assert np.isfinite(x).all() and np.isfinite(S).all()
    assert abs(x[0] / cfg.d_over_r0 - 1.0) < 0.15
