"""The v-radius tuner through the C ABI: the chosen R is the smallest whose
phases agree with those at r_max within the stated tolerance, and the choice
is repeatable."""
import math

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


def test_tune_radius_picks_the_smallest_converged_radius(torch_cuda):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    F, H, W = 60, 640, 700
    say(f"case tune radius: burst1024 crop {F}x{H}x{W}, N 128, R 6..12")
    d = to_device(burst("burst1024", F=F, H=H, W=W))
    st = torch.from_numpy(stf("burst1024", screens=100)).cuda()
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1)
    ws = torch.empty(nv.nvsm_tune_radius_plan(p, H, W, F, 12), dtype=torch.uint8, device="cuda")
    ctx = nv.nvsm_create(0)
    try:
        # tol 0: nothing but r_max itself agrees exactly, so every R is run
        r0, err0 = nv.nvsm_tune_radius(ctx, p, d, st, 6, 12, 0.0, ws)
        say(f"[tune] tol 0: R {r0}, measures " + ", ".join(f"{r}: {e:.3g}" for r, e in sorted(err0.items())))
        assert r0 == 12 and sorted(err0) == list(range(6, 13)) and err0[12] == 0.0
        assert all(err0[r] > 0.0 for r in range(6, 12))
        # the measure falls as R approaches r_max
        assert err0[11] < err0[6]
        tol = 0.5 * (err0[6] + err0[11])
        r1, err1 = nv.nvsm_tune_radius(ctx, p, d, st, 6, 12, tol, ws)
        say(f"[tune] tol {tol:.3g}: R {r1}")
        assert err1[r1] <= tol and all(err0[r] > tol for r in range(6, r1))
        assert all(err1[r] == err0[r] for r in err1)          # repeatable, bit for bit
        assert all(r <= r1 for r in err1)                     # stopped at the first R within tol
    finally:
        nv.nvsm_destroy(ctx)
