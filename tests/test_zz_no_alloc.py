"""nvsm_reconstruct_noalloc (workspace in the library's fixed device scratch
array) against nvsm_reconstruct (caller's workspace), through the C ABI."""
import numpy as np
import pytest

from gpu_helpers import burst, say, stf, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()
    return torch


def _reference(nv, torch, ctx, p, d, st):
    F, H, W = d.shape
    info = nv.nvsm_plan(p, H, W, F)
    out = torch.full((H, W), float("nan"), device="cuda")
    nv.nvsm_reconstruct(ctx, p, d, st, out, torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    return out, info


def test_noalloc_equals_reconstruct_twice(torch_cuda):
    """Two calls in a row, the second on a smaller burst: each equals
    nvsm_reconstruct on the same input bit for bit."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = nv.default_params(128, v_radius=12, noise_bias=1, filter=1)
    st = torch.from_numpy(stf("burst1024", screens=100)).cuda()
    ctx = nv.nvsm_create(0)
    try:
        nv.nvsm_prepare(ctx, p)
        for F, H, W in ((40, 256, 300), (12, 160, 192)):
            say(f"case noalloc: {F}x{H}x{W}, N 128, R 12")
            d = to_device(burst("burst1024", F=F, H=H, W=W))
            ref, info = _reference(nv, torch, ctx, p, d, st)
            out = torch.full((H, W), float("nan"), device="cuda")
            nv.nvsm_reconstruct_noalloc(ctx, p, d, st, out)
            torch.cuda.synchronize()
            same = torch.equal(out, ref)
            say(f"[noalloc] {F}x{H}x{W}: {info.patches} patches, workspace {info.ws_reconstruct / 2**20:.0f} MiB, "
                f"identical to nvsm_reconstruct={same}")
            assert torch.isfinite(out).all() and same
    finally:
        nv.nvsm_destroy(ctx)


def test_noalloc_refusals(torch_cuda):
    """A burst beyond the 256 MiB array, and parameters whose tables do not
    exist yet, are refused before anything is launched."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    p = nv.default_params(128, v_radius=12, noise_bias=1, filter=1)
    st = torch.from_numpy(stf("burst1024", screens=100)).cuda()
    ctx = nv.nvsm_create(0)
    try:
        d = to_device(burst("burst1024", F=12, H=160, W=192))
        out = torch.zeros((160, 192), device="cuda")
        with pytest.raises(nv.NvsmError) as e:               # no tables yet
            nv.nvsm_reconstruct_noalloc(ctx, p, d, st, out)
        assert e.value.status == -1
        nv.nvsm_prepare(ctx, p)
        big = to_device(burst("burst1024", F=100, H=512, W=512))
        info = nv.nvsm_plan(p, 512, 512, 100)
        assert info.ws_reconstruct > 256 << 20
        out = torch.zeros((512, 512), device="cuda")
        with pytest.raises(nv.NvsmError) as e:
            nv.nvsm_reconstruct_noalloc(ctx, p, big, st, out)
        assert e.value.status == -3
        assert "scratch" in nv.nvsm_last_error(ctx)
        torch.cuda.synchronize()
        assert torch.count_nonzero(out).item() == 0
    finally:
        nv.nvsm_destroy(ctx)
