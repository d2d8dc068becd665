"""Serving loop: bursts of three channels arriving frame by frame, mixed on
the device, give the same image as each burst served alone."""
import dataclasses

import numpy as np
import pytest

import synth
from gpu_helpers import MOSAIC_TOL, say

pytestmark = pytest.mark.gpu

CHANNELS = {"A": (256, 320), "B": (300, 256), "C": (260, 270)}
GROUP = 5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    return torch


@pytest.fixture(scope="module")
def world(torch_cuda):
    import paper_1701_00581_amd as nv
    from paper_1701_00581_amd import serve
    torch = torch_cuda
    p = nv.default_params(64, v_radius=8, noise_bias=1, filter=1)
    specs, frames = [], {}
    for ci, (name, (H, W)) in enumerate(CHANNELS.items()):
        cfg = dataclasses.replace(synth.CONFIGS["burst1024"], name=name, index=60 + ci, H=H, W=W, F=1, patch=64,
                                  v_radius=8)
        stf = torch.from_numpy(synth.stf_table(cfg, screens=40, patch=64)).cuda()
        specs.append(serve.ChannelSpec(name, H, W, p, stf))
        for k in range(3):
            c2 = dataclasses.replace(cfg, index=70 + 10 * ci + k, F=31)
            frames[(name, k)] = synth.make_burst(c2)
    events = serve.schedule(list(CHANNELS), seconds=4.0, fps=10.0, fmin=12, fmax=31, gap_s=0.5, seed=5)
    events = [e for e in events if e[2] < 3]           # at most 3 bursts per channel
    return dict(p=p, specs=specs, frames=frames, events=events)


def _serve(world, policy, events, channels=None):
    from paper_1701_00581_amd import serve
    specs = [s for s in world["specs"] if channels is None or s.name in channels]
    srv = serve.Server(specs, policy=policy, group=GROUP, budget=1 << 30, max_frames=31)
    done, wall = serve.run(srv, events, lambda c, k, f: world["frames"][(c, k)][f], pace=False)
    srv.close()
    return {(d.channel, d.burst): d for d in done}, wall


def test_serve_mixed_equals_alone(torch_cuda, world):
    torch = torch_cuda
    events = world["events"]
    mixed, wall = _serve(world, "stream", events)
    bursts = sorted({(e[1], e[2]) for e in events})
    assert set(mixed) == set(bursts)
    say(f"[serve] {len(bursts)} bursts mixed in {wall:.2f} s, latency ms "
        + ", ".join(f"{k[0]}{k[1]}={mixed[k].latency_ms:.1f}" for k in bursts))
    for key in bursts:
        ev = [e for e in events if (e[1], e[2]) == key]
        alone, _ = _serve(world, "stream", ev, channels={key[0]})
        a = alone[key].image
        m = mixed[key].image
        same = torch.equal(a, m)
        say(f"[serve] {key}: F={mixed[key].frames} alone == mixed: {same}")
        assert torch.isfinite(m).all()
        assert same


def test_serve_policies_agree(torch_cuda, world):
    """The plain policy (one nvsm_reconstruct per burst) and the streaming
    policy differ only in where the running sums are folded."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    events = [e for e in world["events"] if e[2] < 2]
    st, _ = _serve(world, "stream", events)
    pl, _ = _serve(world, "plain", events)
    assert set(st) == set(pl)
    for key in sorted(st):
        a = st[key].image.cpu().numpy()
        b = pl[key].image.cpu().numpy()
        core = (slice(64, a.shape[0] - 64), slice(64, a.shape[1] - 64))
        rel = float(np.abs(a[core] - b[core]).max() / b[core].std())
        say(f"[serve] {key}: stream vs plain {rel:.2e}")
        assert rel < MOSAIC_TOL
        # plain equals the library call on the same frames
        F = st[key].frames
        fr = torch.from_numpy(world["frames"][key][:F].view(np.int16)).cuda()
        spec = [s for s in world["specs"] if s.name == key[0]][0]
        info = nv.nvsm_plan(world["p"], spec.H, spec.W, F)
        ref = torch.empty((spec.H, spec.W), device="cuda")
        ctx = nv.nvsm_create(0)
        nv.nvsm_reconstruct(ctx, world["p"], fr, spec.stf, ref,
                            torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
        torch.cuda.synchronize()
        nv.nvsm_destroy(ctx)
        assert torch.equal(ref, pl[key].image)
