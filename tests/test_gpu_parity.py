"""GPU path versus the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_helpers import (BISPEC_TOL, MEAN_SPEC_TOL, MOSAIC_TOL, PHASE_RMS_TOL, POWER_TOL, abs_bispectrum, as_complex,
                         bispec_errors, burst, cube, oparams, phase_rms, say, stf, to_device)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1701_00581_amd as nv
    nv.lib()  # the HIP library must be there: no fallback
    return torch


def _session(p, H, W, F):
    import paper_1701_00581_amd as nv
    return nv.Session(p, H, W, F)


def _check_accumulate(s, frames, p, patches, Sset, label):
    """Power, mean spectrum, mean level and bispectrum of chosen patches."""
    op = oparams(p)
    P = s.power.cpu().numpy()
    M = s.mean_spec.cpu().numpy()
    mu = s.mu.cpu().numpy()
    B = as_complex(s.bispec)
    for k in patches:
        c = cube(frames, p, k)
        I, muf = oracle.patch_spectra(c, op.window)
        Po = np.mean(np.abs(I) ** 2, axis=0)
        Mo = np.mean(I, axis=0)
        perr = np.linalg.norm(P[k] - Po) / np.linalg.norm(Po)
        m10 = abs(complex(M[k, 0, 0], M[k, 0, 1]) - Mo[0, 1]) / abs(Mo[0, 1])
        m01 = abs(complex(M[k, 1, 0], M[k, 1, 1]) - Mo[1, 0]) / abs(Mo[1, 0])
        muerr = abs(mu[k] - muf.mean()) / abs(muf.mean())
        Bo = oracle.bispectrum(I, Sset)
        A = abs_bispectrum(I, Sset)
        nerr, aerr = bispec_errors(B[k], Bo, A)
        say(f"[{label}] patch {k}: P {perr:.2e} M10 {m10:.2e} M01 {m01:.2e} mu {muerr:.2e} "
            f"B norm {nerr:.2e} B/A max {aerr:.2e}")
        assert perr <= POWER_TOL
        # the mean spectrum's only use is the phase of the two seeds, which a
        # relative error d moves by at most d rad: kept 10x under the phase
        # tolerance
        assert m10 <= MEAN_SPEC_TOL and m01 <= MEAN_SPEC_TOL and muerr <= 1e-6
        assert nerr <= BISPEC_TOL and aerr <= BISPEC_TOL


def test_single64_whole_path(torch_cuda):
    """64x64 subimage, 100 float32 frames, no taper, R = 8."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case single64: accumulate/solve/synthesize, F=100, N=64, R=8")
    fr = burst("single64")
    p = nv.default_params(64, v_radius=8, window=0)
    s = _session(p, 64, 64, 100)
    d = to_device(fr)
    s.accumulate(d)
    torch.cuda.synchronize()
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    _check_accumulate(s, fr, p, [0], S, "single64")
    # modulus and phase from the GPU accumulation vs the oracle end to end
    st = stf("single64")
    st_d = torch.from_numpy(st).cuda()
    s.solve(st_d)
    s.synthesize()
    torch.cuda.synchronize()
    ref = oracle.reconstruct(fr, oparams(p), st)
    t = ref["tiles"][(0, 0)]
    amp = s.amp.cpu().numpy()[0]
    ph = as_complex(s.phasor)[0]
    aerr = np.max(np.abs(amp - t["amp"]) / np.maximum(t["amp"], 1e-30 + np.max(t["amp"]) * 1e-12))
    rms, mx = phase_rms(ph, t["phasor"])
    say(f"[single64] amp rel max {aerr:.2e} phase rms {rms:.2e} max {mx:.2e}")
    assert aerr <= 1e-4
    assert rms <= PHASE_RMS_TOL
    img = s.image.cpu().numpy()
    o = ref["image"]
    merr = np.linalg.norm(img - o) / np.linalg.norm(o - o.mean())
    say(f"[single64] mosaic {merr:.2e}")
    assert merr <= MOSAIC_TOL


def test_ragged_crop_accumulate(torch_cuda):
    """250x300 crop (clamped last row and column), 37 frames (odd, two frame
    groups with a ragged tail), N = 128, R = 10, Hann taper."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case crop250x300 F=37: accumulate")
    fr = burst("burst1024", F=37, H=250, W=300)
    p = nv.default_params(128, v_radius=10)
    s = _session(p, 250, 300, 37)
    assert s.info.patches == 12
    s.accumulate(to_device(fr))
    torch.cuda.synchronize()
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    _check_accumulate(s, fr, p, list(range(12)), S, "crop")


@pytest.mark.parametrize("F,dtype,pad", [(1, "u16", 0), (2, "f32", 8), (3, "u16", 5)])
def test_few_frames_strided_rows_clamped_patch(torch_cuda, F, dtype, pad):
    """Degenerate frame counts (one frame: the bispectrum is a single
    triple product and every closure is exact; two and three frames: one
    transform pair with and without a partner), rows with a pitch wider
    than the image (a strided view), scalar pixel loads (odd width), and a
    second patch clamped to x0 = 3 that overlaps the first almost whole.
    N = 128, R = 12, Hann taper."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    H, W = 128, 131
    say(f"case few frames F={F} {dtype} pitch W+{pad}: accumulate")
    fr = burst("burst1024", F=3, H=H, W=W)[:F]
    if dtype == "f32":
        fr = fr.astype(np.float32)
    p = nv.default_params(128, v_radius=12)
    s = _session(p, H, W, F)
    assert s.info.patches == 2
    big = np.zeros((F, H, W + pad), fr.dtype)
    big[:, :, :W] = fr
    d = to_device(big)[:, :, :W]
    assert d.stride(1) == W + pad
    s.accumulate(d)
    torch.cuda.synchronize()
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    _check_accumulate(s, fr, p, [0, 1], S, f"F={F}")
    if F != 1:
        return
    # one frame: the whole path against the oracle
    st = stf("burst1024", screens=100)
    s.solve(torch.from_numpy(st).cuda())
    s.synthesize()
    torch.cuda.synchronize()
    ref = oracle.reconstruct(fr, oparams(p), st)
    ph = as_complex(s.phasor)
    for k, key in enumerate([(0, 0), (0, 1)]):
        rms, mx = phase_rms(ph[k], ref["tiles"][key]["phasor"])
        say(f"[F=1] patch {k}: phase rms {rms:.2e} max {mx:.2e}")
        assert rms <= PHASE_RMS_TOL
    img = s.image.cpu().numpy()
    o = ref["image"]
    inner = (slice(16, H - 16), slice(16, W - 16))
    merr = np.linalg.norm(img[inner] - o[inner]) / np.linalg.norm(o[inner] - o[inner].mean())
    say(f"[F=1] mosaic {merr:.2e}")
    assert merr <= MOSAIC_TOL


def test_solve_on_identical_inputs(torch_cuda):
    """The FP64 solve alone: both sides get the same FP32-rounded power,
    mean spectrum and bispectrum (computed by the oracle)."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case solve-only: oracle inputs rounded to FP32, N=128, R=10, noise bias on")
    fr = burst("burst1024", F=37, H=250, W=300)
    p = nv.default_params(128, v_radius=10, noise_bias=1)
    op = oparams(p)
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    ks = [0, 5, 11]
    Ps, Ms, Bs = [], [], []
    for k in ks:
        acc = oracle.accumulate_patch(cube(fr, p, k), op, S)
        Ps.append(acc["P"].astype(np.float32))
        Ms.append(np.array([[acc["M10"].real, acc["M10"].imag], [acc["M01"].real, acc["M01"].imag]], np.float32))
        Bs.append(np.stack([acc["B"].real, acc["B"].imag], -1).astype(np.float32))
    st = stf("burst1024", screens=100)
    ctx = nv.nvsm_create(0)
    try:
        n = len(ks)
        amp = torch.empty(n, len(Wset), dtype=torch.float64, device="cuda")
        ph = torch.empty(n, len(Wset), 2, dtype=torch.float64, device="cuda")
        nv.nvsm_solve(ctx, p, n, torch.from_numpy(np.stack(Ps)).cuda(), torch.from_numpy(np.stack(Ms)).cuda(),
                      torch.from_numpy(np.stack(Bs)).cuda(), torch.from_numpy(st).cuda(), amp, ph)
        torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)
    amp = amp.cpu().numpy()
    ph = as_complex(ph)
    for i in range(len(ks)):
        P64 = Ps[i].astype(np.float64)
        nb = oracle.noise_bias(P64)
        ao = oracle.amplitude(P64, st, Wset, nb, p.stf_floor)
        B64 = Bs[i][..., 0].astype(np.float64) + 1j * Bs[i][..., 1].astype(np.float64)
        eo = oracle.phase_recursion(B64, complex(*Ms[i][0].astype(np.float64)),
                                    complex(*Ms[i][1].astype(np.float64)), Wset, S, woff, p.patch)
        aerr = np.max(np.abs(amp[i] - ao)) / np.max(ao)
        rms, mx = phase_rms(ph[i], eo)
        say(f"[solve] patch {ks[i]}: amp {aerr:.2e} phase rms {rms:.2e} max {mx:.2e}")
        assert aerr <= 1e-12
        assert rms <= 1e-9


@pytest.mark.parametrize("N,u_cut,R,stride,window,H,W,F", [
    (128, 40, 16, 40, 1, 200, 200, 8),     # the largest R, a low cut-off, 3x3 patches at a short stride
    (128, 63, 16, 32, 1, 128, 160, 3),     # the phase kernel's large window (2768 ring entries), 8 samples a lane
    (64, 20, 5, 24, 0, 100, 90, 9),        # no taper, odd F, clamped last row and column
    (64, 31, 3, 32, 1, 96, 130, 6),        # the smallest usual R
    (64, 3, 2, 32, 1, 96, 96, 5),          # |S| = 44, fewer samples than one padded code block
])
def test_other_geometries_accumulate_and_solve(torch_cuda, N, u_cut, R, stride, window, H, W, F):
    """Parameter sets away from the benchmark's: the bispectrum work plan
    (groups, regions, items) and the solve's phasor window differ.  The
    accumulation against the oracle, then the solve on the GPU's own
    accumulations against the oracle's solve of the same FP32 values."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say(f"case geometry N={N} u_cut={u_cut} R={R} stride={stride} window={window} {H}x{W} F={F}")
    fr = burst("burst1024", F=F, H=H, W=W)
    p = nv.default_params(N, u_cut=u_cut, v_radius=R, stride=stride, window=window)
    s = _session(p, H, W, F)
    s.accumulate(to_device(fr))
    torch.cuda.synchronize()
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    P = s.info.patches
    _check_accumulate(s, fr, p, [0, P - 1], S, f"geom N={N} R={R}")
    st = np.ones((N, N))
    s.solve(torch.from_numpy(st).cuda())
    torch.cuda.synchronize()
    amp = s.amp.cpu().numpy()
    ph = as_complex(s.phasor)
    Pg = s.power.cpu().numpy().astype(np.float64)
    Mg = s.mean_spec.cpu().numpy().astype(np.float64)
    Bg = as_complex(s.bispec)
    # three least-squares steps on the same inputs (the accumulator ring of
    # the steps is largest at R = 16)
    p2 = nv.default_params(N, u_cut=u_cut, v_radius=R, stride=stride, window=window, phase_method=1, lsq_iters=3)
    amp2 = torch.empty_like(s.amp)
    ph2 = torch.empty_like(s.phasor)
    nv.nvsm_solve(s.ctx, p2, P, s.power, s.mean_spec, s.bispec, torch.from_numpy(st).cuda(), amp2, ph2)
    torch.cuda.synchronize()
    ph2 = as_complex(ph2)
    for k in (0, P - 1):
        ao = oracle.amplitude(Pg[k], st, Wset, 0.0, p.stf_floor)
        eo = oracle.phase_recursion(Bg[k].astype(np.complex128), complex(*Mg[k][0]), complex(*Mg[k][1]),
                                    Wset, S, woff, N)
        aerr = np.max(np.abs(amp[k] - ao)) / np.max(ao)
        rms, mx = phase_rms(ph[k], eo)
        el = oracle.phase_least_squares(Bg[k].astype(np.complex128), eo, Wset, S, woff, 3)
        lrms, lmx = phase_rms(ph2[k], el)
        moved, _ = phase_rms(el, eo)
        say(f"[geom N={N} R={R}] patch {k}: solve amp {aerr:.2e} phase rms {rms:.2e} max {mx:.2e}; "
            f"3 least-squares steps rms {lrms:.2e} max {lmx:.2e} (moved {moved:.2e})")
        assert aerr <= 1e-12
        assert rms <= 1e-9
        assert moved > 1e-6 and lrms <= 1e-9


def test_synthesize_on_identical_inputs(torch_cuda):
    """Inverse transforms and mosaic from the same FP64 modulus and phase."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case synthesize-only: crop 250x300, N=128, filter on")
    H, W = 250, 300
    p = nv.default_params(128, v_radius=10, filter=1)
    op = oparams(p)
    ys, xs = oracle.tiling(H, W, 128, 64)
    Wset = oracle.frequency_half_disk(p.u_cut)
    rng = np.random.default_rng(7)
    n = len(ys) * len(xs)
    amp = rng.random((n, len(Wset))) * 1e4 / (1.0 + np.hypot(Wset[:, 0], Wset[:, 1]))[None]
    phase = rng.uniform(-np.pi, np.pi, (n, len(Wset)))
    ph = np.exp(1j * phase)
    mu = rng.uniform(1500, 2500, n).astype(np.float32)
    filt = oracle.diffraction_filter(Wset, 128)
    pats = np.stack([oracle.synthesize_patch(amp[k], ph[k], Wset, 128, float(mu[k]), 1, filt) for k in range(n)])
    ref = oracle.mosaic(pats.reshape(len(ys), len(xs), 128, 128), ys, xs, H, W, 1)
    s = _session(p, H, W, 1)
    s.synthesize(torch.from_numpy(amp).cuda(), torch.from_numpy(np.stack([ph.real, ph.imag], -1)).cuda(),
                 torch.from_numpy(mu).cuda())
    torch.cuda.synchronize()
    pg = s.patches.cpu().numpy()
    perr = np.linalg.norm(pg - pats) / np.linalg.norm(pats - pats.mean())
    img = s.image.cpu().numpy()
    inner = (slice(64, H - 64), slice(64, W - 64))
    merr = np.linalg.norm(img[inner] - ref[inner]) / np.linalg.norm(ref[inner] - ref[inner].mean())
    full = np.max(np.abs(img - ref)) / np.max(np.abs(ref))
    say(f"[synth] patches {perr:.2e} mosaic interior {merr:.2e} full max {full:.2e}")
    assert perr <= 1e-5 and merr <= 1e-5 and full <= 1e-5
    assert np.all(img[0, :] == 0) and np.all(img[:, 0] == 0)


def test_reconstruct_crop_end_to_end_and_deterministic(torch_cuda):
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case reconstruct crop 250x300 F=37, N=128, R=10, noise bias + filter")
    fr = burst("burst1024", F=37, H=250, W=300)
    p = nv.default_params(128, v_radius=10, noise_bias=1, filter=1)
    st = stf("burst1024", screens=100)
    s = _session(p, 250, 300, 37)
    d = to_device(fr)
    std = torch.from_numpy(st).cuda()
    a = s.reconstruct(d, std).clone()
    b = s.reconstruct(d, std).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b), "two runs differ"
    ref = oracle.reconstruct(fr, oparams(p), st)["image"]
    img = a.cpu().numpy()
    inner = (slice(64, 250 - 64), slice(64, 300 - 64))
    merr = np.linalg.norm(img[inner] - ref[inner]) / np.linalg.norm(ref[inner] - ref[inner].mean())
    say(f"[reconstruct] mosaic interior {merr:.2e}")
    assert merr <= MOSAIC_TOL


def test_error_paths(torch_cuda):
    import ctypes
    import paper_1701_00581_amd as nv
    from paper_1701_00581_amd import _lib
    torch = torch_cuda
    say("case error paths")
    p = nv.default_params(128)
    ctx = nv.nvsm_create(0)
    L = nv.lib()
    try:
        fr = torch.zeros(3, 256, 256, dtype=torch.int16, device="cuda")
        info = nv.nvsm_plan(p, 256, 256, 3)
        out = torch.zeros(256, 256, device="cuda")
        st = torch.ones(128, 128, dtype=torch.float64, device="cuda")
        ws = torch.empty(info.ws_reconstruct - 1, dtype=torch.uint8, device="cuda")
        args = lambda w, n: (ctx, ctypes.byref(p), fr.data_ptr(), 0, 3, 256, 256, 256, st.data_ptr(),  # noqa: E731
                             out.data_ptr(), w, n, None)
        assert L.nvsm_reconstruct(*args(ws.data_ptr(), ws.numel())) == _lib.NVSM_ERR_WORKSPACE
        assert "workspace" in nv.nvsm_last_error(ctx)
        assert L.nvsm_reconstruct(*args(None, 0)) == _lib.NVSM_ERR_WORKSPACE
        a = list(args(ws.data_ptr(), ws.numel()))
        a[8] = None
        assert L.nvsm_reconstruct(*a) == _lib.NVSM_ERR_INVALID_ARG
        a = list(args(ws.data_ptr(), ws.numel()))
        a[7] = 100   # pitch < W
        assert L.nvsm_reconstruct(*a) == _lib.NVSM_ERR_SHAPE
        a = list(args(ws.data_ptr(), ws.numel()))
        a[3] = 7     # bad dtype
        assert L.nvsm_reconstruct(*a) == _lib.NVSM_ERR_INVALID_ARG
        a = list(args(ws.data_ptr(), ws.numel()))
        a[7] = (1 << 30) // 128 + 1   # pitch beyond 32-bit pixel offsets
        assert L.nvsm_reconstruct(*a) == _lib.NVSM_ERR_SHAPE
        assert "row_pitch" in nv.nvsm_last_error(ctx)
        a = list(args(ws.data_ptr(), ws.numel()))
        a[4] = 26215  # frame count beyond 32-bit spectrum offsets
        assert L.nvsm_reconstruct(*a) == _lib.NVSM_ERR_SHAPE
        assert torch.count_nonzero(out).item() == 0
        torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)


def test_full_burst2560_sampled(torch_cuda):
    """The benchmark workload at full size (2560x2160 x 100 frames, 39x33
    patches, R = 12, noise bias and filter on) through nvsm_reconstruct and
    the stage calls: sampled patches against the oracle (power, mean
    spectrum, 20000 bispectrum samples, modulus, all phases of two patches)
    and a mosaic window covered by four patches."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case burst2560 full size: reconstruct + sampled stages")
    fr = burst("burst2560")
    F, H, W = fr.shape
    p = nv.default_params(128, v_radius=12, noise_bias=1, filter=1)
    st = stf("burst2560", screens=100)
    s = _session(p, H, W, F)
    assert s.info.patches == 1287
    d = to_device(fr)
    std = torch.from_numpy(st).cuda()
    img = s.reconstruct(d, std).clone()
    s.accumulate(d)
    s.solve(std)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
    op = oparams(p)
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    rng = np.random.default_rng(2560)
    pick = rng.choice(len(S), 20000, replace=False)
    P = s.power.cpu().numpy()
    B = as_complex(s.bispec)
    amp = s.amp.cpu().numpy()
    ph = as_complex(s.phasor)
    for k in [0, 643, 1286, int(rng.integers(0, 1287))]:
        c = cube(fr, p, k)
        I, muf = oracle.patch_spectra(c, op.window)
        Po = np.mean(np.abs(I) ** 2, axis=0)
        perr = np.linalg.norm(P[k] - Po) / np.linalg.norm(Po)
        Bo = oracle.bispectrum(I, S[pick])
        A = abs_bispectrum(I, S[pick])
        nerr, aerr = bispec_errors(B[k][pick], Bo, A)
        nb = oracle.noise_bias(Po)
        ao = oracle.amplitude(Po, st, Wset, nb, p.stf_floor)
        aerr2 = np.max(np.abs(amp[k] - ao)) / np.max(ao)
        say(f"[burst2560] patch {k}: P {perr:.2e} B norm {nerr:.2e} B/A max {aerr:.2e} amp {aerr2:.2e}")
        assert perr <= POWER_TOL and nerr <= BISPEC_TOL and aerr <= BISPEC_TOL and aerr2 <= 1e-4
    for k in [0, 1286]:
        acc = oracle.accumulate_patch(cube(fr, p, k), op, S)
        eo = oracle.phase_recursion(acc["B"], acc["M10"], acc["M01"], Wset, S, woff, p.patch)
        rms, mx = phase_rms(ph[k], eo)
        say(f"[burst2560] patch {k}: phase rms {rms:.2e} max {mx:.2e}")
        assert rms <= PHASE_RMS_TOL
    # mosaic window [64, 128) x [64, 128): covered by tiles (0..1, 0..1) only
    ref = oracle.reconstruct(fr, op, st, patch_list=[(0, 0), (0, 1), (1, 0), (1, 1)])
    win = np.zeros((64, 64))
    den = np.zeros((64, 64))
    w2 = oracle.window2d(128, 1)
    for (i, j), t in ref["tiles"].items():
        oy, ox = ref["ys"][i], ref["xs"][j]
        win += t["patch"][64 - oy:128 - oy, 64 - ox:128 - ox]
        den += w2[64 - oy:128 - oy, 64 - ox:128 - ox]
    win /= den
    g = img.cpu().numpy()[64:128, 64:128]
    merr = np.linalg.norm(g - win) / np.linalg.norm(win - win.mean())
    say(f"[burst2560] mosaic window {merr:.2e}")
    assert merr <= MOSAIC_TOL


def _lsq_case(torch, nv, name, F, H, W, v_radius, ks, iters, screens):
    """Least-squares refinement on identical FP32-rounded inputs: the GPU
    solve with phase_method 1 against the oracle's recursion followed by
    its least-squares steps, patch by patch."""
    fr = burst(name, F=F, H=H, W=W)
    p = nv.default_params(128, v_radius=v_radius, noise_bias=1)
    p.phase_method = 1
    p.lsq_iters = iters
    op = oparams(p)
    Wset, S, woff = oracle.bispectrum_set(p.u_cut, p.v_radius)
    Ps, Ms, Bs = [], [], []
    for k in ks:
        acc = oracle.accumulate_patch(cube(fr, p, k), op, S)
        Ps.append(acc["P"].astype(np.float32))
        Ms.append(np.array([[acc["M10"].real, acc["M10"].imag], [acc["M01"].real, acc["M01"].imag]], np.float32))
        Bs.append(np.stack([acc["B"].real, acc["B"].imag], -1).astype(np.float32))
    st = stf(name, screens=screens)
    ctx = nv.nvsm_create(0)
    try:
        n = len(ks)
        amp = torch.empty(n, len(Wset), dtype=torch.float64, device="cuda")
        ph = torch.empty(n, len(Wset), 2, dtype=torch.float64, device="cuda")
        nv.nvsm_solve(ctx, p, n, torch.from_numpy(np.stack(Ps)).cuda(), torch.from_numpy(np.stack(Ms)).cuda(),
                      torch.from_numpy(np.stack(Bs)).cuda(), torch.from_numpy(st).cuda(), amp, ph)
        torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)
    ph = as_complex(ph)
    for i in range(len(ks)):
        B64 = Bs[i][..., 0].astype(np.float64) + 1j * Bs[i][..., 1].astype(np.float64)
        e0 = oracle.phase_recursion(B64, complex(*Ms[i][0].astype(np.float64)),
                                    complex(*Ms[i][1].astype(np.float64)), Wset, S, woff, p.patch)
        eo = oracle.phase_least_squares(B64, e0, Wset, S, woff, iters)
        rms, mx = phase_rms(ph[i], eo)
        moved, _ = phase_rms(eo, e0)
        say(f"[lsq {name} R={v_radius} it={iters}] patch {ks[i]}: vs oracle rms {rms:.2e} max {mx:.2e} "
            f"(refinement moved the phases by rms {moved:.2e})")
        assert moved > 1e-6               # the steps did something
        assert rms <= 1e-9
        assert np.max(np.abs(ph[i][:2] - e0[:2])) < 1e-12     # the seeds stay


def test_lsq_on_identical_inputs(torch_cuda):
    """Crop of the 1024 burst, N = 128, R = 10, three patches (corner, inner,
    edge), 10 steps; then one step, where a wrong side entry shows alone."""
    import paper_1701_00581_amd as nv
    say("case lsq: burst1024 crop 250x300 F=37 N=128 R=10, iters 10 and 1")
    _lsq_case(torch_cuda, nv, "burst1024", 37, 250, 300, 10, [0, 5, 11], 10, 100)
    _lsq_case(torch_cuda, nv, "burst1024", 37, 250, 300, 10, [5], 1, 100)


def test_lsq_full_size_patch(torch_cuda):
    """The 2160x2560 burst's configuration (N = 128, R = 12, all of W): one
    patch, 8 frames, 10 steps."""
    import paper_1701_00581_amd as nv
    say("case lsq: burst2560 patch 0 F=8 N=128 R=12, iters 10")
    _lsq_case(torch_cuda, nv, "burst2560", 8, 128, 128, 12, [0], 10, 60)


def test_single64_lsq_whole_path(torch_cuda):
    """The whole path with the least-squares phase (phase_method 1) against
    the oracle's reconstruction with the same method."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case single64 lsq: accumulate/solve/synthesize, F=100, N=64, R=8, 10 steps")
    fr = burst("single64")
    p = nv.default_params(64, v_radius=8, window=0)
    p.phase_method = 1
    p.lsq_iters = 10
    s = _session(p, 64, 64, 100)
    s.accumulate(to_device(fr))
    st = stf("single64")
    s.solve(torch.from_numpy(st).cuda())
    s.synthesize()
    torch.cuda.synchronize()
    ref = oracle.reconstruct(fr, oparams(p), st)
    t = ref["tiles"][(0, 0)]
    rms, mx = phase_rms(as_complex(s.phasor)[0], t["phasor"])
    img = s.image.cpu().numpy()
    o = ref["image"]
    merr = np.linalg.norm(img - o) / np.linalg.norm(o - o.mean())
    say(f"[single64 lsq] phase rms {rms:.2e} max {mx:.2e} mosaic {merr:.2e}")
    assert rms <= PHASE_RMS_TOL
    assert merr <= MOSAIC_TOL


def _photon_burst(photons, F, H, W):
    """The 1024 burst's scene at a low photon level (12-bit frames, gain
    photons / 2048 photons per unit), so the noise terms are large."""
    import dataclasses
    import synth
    cfg = dataclasses.replace(synth.CONFIGS["burst1024"], photons=float(photons), index=91)
    return np.ascontiguousarray(synth.make_burst(cfg, frames=F)[:, :H, :W]), photons / 2048.0


def test_photon_noise_accumulate(torch_cuda):
    """noise_bias 2 on a 250x300 crop, 37 frames, 40 photons per pixel:
    corrected power spectrum and bispectrum against the oracle's, and the
    correction itself far above the tolerance."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case photon noise: burst1024 scene at 40 photons/px, crop 250x300 F=37, N=128, R=10")
    fr, gain = _photon_burst(40, 37, 250, 300)
    p = nv.default_params(128, v_radius=10, noise_bias=2, photons_per_adu=gain)
    s = _session(p, 250, 300, 37)
    s.accumulate(to_device(fr))
    torch.cuda.synchronize()
    op = oparams(p)
    op0 = oparams(nv.default_params(128, v_radius=10))
    S = oracle.bispectrum_set(p.u_cut, p.v_radius)[1]
    P = s.power.cpu().numpy()
    B = as_complex(s.bispec)
    for k in (0, 6, 11):
        c = cube(fr, p, k)
        acc = oracle.accumulate_patch(c, op, S)
        raw = oracle.accumulate_patch(c, op0, S)
        I, _ = oracle.patch_spectra(c, op.window)
        A = abs_bispectrum(I, S)
        perr = np.linalg.norm(P[k] - acc["P"]) / np.linalg.norm(acc["P"])
        nerr, aerr = bispec_errors(B[k], acc["B"], A)
        moved = np.max(np.abs(acc["B"] - raw["B"]) / A)
        pmoved = np.linalg.norm(acc["P"] - raw["P"]) / np.linalg.norm(raw["P"])
        say(f"[photon] patch {k}: P {perr:.2e} B norm {nerr:.2e} B/A max {aerr:.2e} "
            f"(correction: B/A up to {moved:.2e}, P by {pmoved:.2e})")
        assert perr <= POWER_TOL
        assert nerr <= BISPEC_TOL and aerr <= BISPEC_TOL
        assert moved > 100 * BISPEC_TOL and pmoved > 100 * POWER_TOL


def test_photon_noise_whole_path(torch_cuda):
    """noise_bias 2 through nvsm_reconstruct on a 160x192 crop (N = 64,
    R = 8, 20 patches, 24 frames at 1000 photons per pixel) against the
    oracle's reconstruction with the same model.  (Far fewer photons make
    the corrected power of most high frequencies a small difference of
    large numbers, which the division by the transfer function then
    magnifies: the mosaic is no longer a stable function of the inputs.)"""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case photon noise whole path: 160x192 F=24, N=64, R=8, 1000 photons/px")
    fr, gain = _photon_burst(1000, 24, 160, 192)
    p = nv.default_params(64, v_radius=8, noise_bias=2, photons_per_adu=gain, filter=1)
    import synth
    st = synth.stf_table(synth.CONFIGS["burst1024"], screens=60, patch=64)
    info = nv.nvsm_plan(p, 160, 192, 24)
    ctx = nv.nvsm_create(0)
    try:
        img = torch.empty((160, 192), device="cuda")
        nv.nvsm_reconstruct(ctx, p, to_device(fr), torch.from_numpy(st).cuda(), img,
                            torch.empty(info.ws_reconstruct, dtype=torch.uint8, device="cuda"))
        torch.cuda.synchronize()
    finally:
        nv.nvsm_destroy(ctx)
    ref = oracle.reconstruct(fr, oparams(p), st)["image"]
    ref0 = oracle.reconstruct(fr, oparams(nv.default_params(64, v_radius=8, filter=1)), st)["image"]
    g = img.cpu().numpy()
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref - ref.mean())
    moved = np.linalg.norm(ref0 - ref) / np.linalg.norm(ref - ref.mean())
    say(f"[photon path] mosaic vs oracle {err:.2e} (the correction moved the image by {moved:.2e})")
    assert err <= MOSAIC_TOL
    assert moved > 10 * MOSAIC_TOL


def test_single64_photon_noise_no_taper(torch_cuda):
    """noise_bias 2 without a taper (single 64x64 subimage, float32 photon
    counts, one photon per unit): whole path against the oracle."""
    import paper_1701_00581_amd as nv
    torch = torch_cuda
    say("case single64 photon noise: no taper, F=100, N=64, R=8, gain 1")
    fr = burst("single64")
    p = nv.default_params(64, v_radius=8, window=0, noise_bias=2, photons_per_adu=1.0)
    s = _session(p, 64, 64, 100)
    s.accumulate(to_device(fr))
    st = stf("single64")
    s.solve(torch.from_numpy(st).cuda())
    s.synthesize()
    torch.cuda.synchronize()
    op = oparams(p)
    S = oracle.bispectrum_set(p.u_cut, p.v_radius)[1]
    acc = oracle.accumulate_patch(fr.astype(np.float64), op, S)
    I, _ = oracle.patch_spectra(fr.astype(np.float64), 0)
    nerr, aerr = bispec_errors(as_complex(s.bispec)[0], acc["B"], abs_bispectrum(I, S))
    perr = np.linalg.norm(s.power.cpu().numpy()[0] - acc["P"]) / np.linalg.norm(acc["P"])
    ref = oracle.reconstruct(fr, op, st)
    rms, mx = phase_rms(as_complex(s.phasor)[0], ref["tiles"][(0, 0)]["phasor"])
    img = s.image.cpu().numpy()
    merr = np.linalg.norm(img - ref["image"]) / np.linalg.norm(ref["image"] - ref["image"].mean())
    say(f"[single64 photon] P {perr:.2e} B norm {nerr:.2e} B/A max {aerr:.2e} phase rms {rms:.2e} mosaic {merr:.2e}")
    assert perr <= POWER_TOL
    assert nerr <= BISPEC_TOL and aerr <= BISPEC_TOL
    assert rms <= PHASE_RMS_TOL
    assert merr <= MOSAIC_TOL
