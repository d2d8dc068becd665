"""Pins of the FP64 oracle against facts fixed by the paper and mathematics.

None of these compares the oracle with itself: each checks it against a
brute-force computation, an invariant, a closed form or the paper's own
arithmetic, chosen so that a dropped term, a wrong sign or index, or a
transposed operand fails at least one test.
"""
import math

import numpy as np
import pytest

import oracle


def _rng(k):
    return np.random.default_rng(12345 + k)


# ---------------------------------------------------------------------------
# Bispectrum definition (Sections 2 and 3.2, speckle masking).
# ---------------------------------------------------------------------------
def test_bispectrum_equals_bruteforce_triple_correlation_8x8():
    """B(u1,u2) = I(u1) I(u2) conj I(u1+u2) is the 4-D DFT of the circular
    triple correlation T(x1,x2) = sum_x i(x) i(x+x1) i(x+x2), computed here
    with explicit exponentials (no FFT) on an 8x8 non-symmetric image."""
    N = 8
    img = _rng(0).random((N, N))
    q = img - img.mean()
    # triple correlation, brute force
    T = np.zeros((N, N, N, N))
    for y1 in range(N):
        for x1 in range(N):
            s1 = np.roll(q, (-y1, -x1), axis=(0, 1))
            for y2 in range(N):
                for x2 in range(N):
                    s2 = np.roll(q, (-y2, -x2), axis=(0, 1))
                    T[y1, x1, y2, x2] = np.sum(q * s1 * s2)
    # all (w, v) with components in [-3, 3]
    rng = range(-3, 4)
    wv = np.array([(wx, wy, vx, vy) for wx in rng for wy in rng for vx in rng for vy in rng])
    I, mu = oracle.patch_spectra(img[None], window=0)
    assert abs(mu[0] - img.mean()) < 1e-15
    B = oracle.bispectrum(I, wv)
    n = np.arange(N)
    for k in _rng(1).choice(len(wv), 200, replace=False):
        wx, wy, vx, vy = wv[k]
        u1 = (wx - vx, wy - vy)
        u2 = (vx, vy)
        e1 = np.exp(-2j * np.pi * (u1[0] * n[None, :] + u1[1] * n[:, None]) / N)  # [y1][x1]
        e2 = np.exp(-2j * np.pi * (u2[0] * n[None, :] + u2[1] * n[:, None]) / N)  # [y2][x2]
        ref = np.einsum("abcd,ab,cd->", T, e1, e2)
        assert abs(B[k] - ref) <= 1e-12 * max(1.0, abs(ref)), (wv[k], B[k], ref)


def test_bispectrum_invariant_under_integer_frame_shifts():
    N, F = 16, 4
    Wset, S, woff = oracle.bispectrum_set(7, 4)
    frames = _rng(2).random((F, N, N))
    shifted = np.stack([np.roll(frames[f], tuple(_rng(10 + f).integers(0, N, 2)), axis=(0, 1))
                        for f in range(F)])
    B0 = oracle.accumulate_patch(frames, oracle.Params(patch=N, v_radius=4, window=0), S)["B"]
    B1 = oracle.accumulate_patch(shifted, oracle.Params(patch=N, v_radius=4, window=0), S)["B"]
    scale = np.max(np.abs(B0))
    assert np.max(np.abs(B0 - B1)) <= 1e-12 * scale
    # a non-shift change (transpose of one frame) must change it
    frames[0] = frames[0].T
    B2 = oracle.accumulate_patch(frames, oracle.Params(patch=N, v_radius=4, window=0), S)["B"]
    assert np.max(np.abs(B0 - B2)) > 1e-3 * scale


def test_bispectrum_symmetries():
    N = 16
    I, _ = oracle.patch_spectra(_rng(3).random((3, N, N)), window=1)
    Wset, S, woff = oracle.bispectrum_set(7, 5)
    B = oracle.bispectrum(I, S)
    wx, wy, vx, vy = (S[:, i] for i in range(4))
    # Hermitian: B(-w, -v) = conj B(w, v)
    Bneg = oracle.bispectrum(I, np.stack([-wx, -wy, -vx, -vy], 1))
    np.testing.assert_allclose(Bneg, np.conj(B), rtol=0, atol=1e-12 * np.abs(B).max())
    # exchange of the two short sides: B(w, v) = B(w, w - v)
    Bsw = oracle.bispectrum(I, np.stack([wx, wy, wx - vx, wy - vy], 1))
    np.testing.assert_allclose(Bsw, B, rtol=0, atol=1e-12 * np.abs(B).max())
    # B(u1, u2) = B(-u1-u2, u2):  (w, v) -> (v - w, v)
    Bp = oracle.bispectrum(I, np.stack([vx - wx, vy - wy, vx, vy], 1))
    np.testing.assert_allclose(Bp, B, rtol=0, atol=1e-12 * np.abs(B).max())


# ---------------------------------------------------------------------------
# The index sets.
# ---------------------------------------------------------------------------
def _gauss_circle(r):
    """Lattice points with x^2 + y^2 <= r^2 (column sums of the disk)."""
    return sum(2 * math.isqrt(r * r - x * x) + 1 for x in range(-r, r + 1))


@pytest.mark.parametrize("uc,R", [(7, 3), (31, 8), (63, 12)])
def test_bispectrum_set_definition(uc, R):
    Wset, S, woff = oracle.bispectrum_set(uc, R)
    # |W| is half the punctured disk (Gauss circle count)
    assert len(Wset) == (_gauss_circle(uc) - 1) // 2
    n2 = (Wset ** 2).sum(1)
    assert np.all(np.diff(n2) >= 0)
    assert np.all((Wset[:, 1] > 0) | ((Wset[:, 1] == 0) & (Wset[:, 0] > 0)))
    assert woff[-1] == len(S)
    # every sample is a triangle with two strictly shorter nonzero sides
    w2 = S[:, 0] ** 2 + S[:, 1] ** 2
    v2 = S[:, 2] ** 2 + S[:, 3] ** 2
    d2 = (S[:, 0] - S[:, 2]) ** 2 + (S[:, 1] - S[:, 3]) ** 2
    assert np.all((v2 > 0) & (v2 < w2) & (v2 <= R * R) & (d2 > 0) & (d2 < w2))
    # completeness against a direct set-builder for a sample of w
    for i in _rng(4).choice(len(Wset), 30, replace=False):
        wx, wy = Wset[i]
        ref = {(vx, vy) for vx in range(-R, R + 1) for vy in range(-R, R + 1)
               if 0 < vx * vx + vy * vy <= R * R and vx * vx + vy * vy < wx * wx + wy * wy
               and 0 < (wx - vx) ** 2 + (wy - vy) ** 2 < wx * wx + wy * wy}
        got = {(int(a), int(b)) for a, b in S[woff[i]:woff[i + 1], 2:4]}
        assert got == ref
        assert np.all(S[woff[i]:woff[i + 1], 0] == wx)
    # only (1,0) and (0,1) have no samples
    empty = [tuple(Wset[i]) for i in range(len(Wset)) if woff[i + 1] == woff[i]]
    assert sorted(empty) == [(0, 1), (1, 0)]


# ---------------------------------------------------------------------------
# Phase recursion: exact recovery up to translation.
# ---------------------------------------------------------------------------
def _recovery_case(transfer):
    N, F, uc, R = 16, 6, 7, 3
    rng = _rng(5)
    obj = rng.random((N, N))
    O = np.fft.fft2(obj)
    frames = []
    for f in range(F):
        sh = tuple(rng.integers(0, N, 2))
        img = np.roll(obj, sh, axis=(0, 1))
        if transfer:
            # real, positive per-frame transfer function (Gaussian blur)
            k = np.fft.fftfreq(N)
            g = np.exp(-(k[None, :] ** 2 + k[:, None] ** 2) * (1.0 + 3.0 * rng.random()))
            img = np.real(np.fft.ifft2(np.fft.fft2(img) * g))
        frames.append(img)
    frames = np.stack(frames)
    p = oracle.Params(patch=N, u_cut=uc, v_radius=R, window=0)
    Wset, S, woff = oracle.bispectrum_set(uc, R)
    acc = oracle.accumulate_patch(frames, p, S)
    e = oracle.phase_recursion(acc["B"], 1.0, 1.0, Wset, S, woff, N)
    phi = np.angle(O)
    ref = phi[Wset[:, 1] % N, Wset[:, 0] % N] - Wset[:, 0] * phi[0, 1] - Wset[:, 1] * phi[1, 0]
    d = np.angle(e * np.exp(-1j * ref))
    return np.max(np.abs(d))


def test_phase_recursion_recovers_object_up_to_translation():
    assert _recovery_case(False) < 1e-10


def test_phase_recursion_recovers_object_through_real_positive_transfer():
    assert _recovery_case(True) < 1e-10


def test_phase_recursion_weights_by_bispectrum_modulus():
    """w = (1,1) has two samples, v = (1,0) and v = (0,1).  With the seeds at
    phase 0 and B = 1 and 3i, the |B|-weighted phasor sum is 1 - 3i, so
    arg e(1,1) = -atan(3) (an unweighted average would give -pi/4)."""
    N = 8
    Wset, S, woff = oracle.bispectrum_set(2, 1)
    i11 = [k for k, w in enumerate(Wset) if tuple(w) == (1, 1)][0]
    B = np.zeros(len(S), dtype=complex)
    seg = S[woff[i11]:woff[i11 + 1]]
    assert sorted(map(tuple, seg[:, 2:4])) == [(0, 1), (1, 0)]
    B[woff[i11]:woff[i11 + 1]] = [1.0 if tuple(v) == (1, 0) else 3j for v in seg[:, 2:4]]
    e = oracle.phase_recursion(B, 1.0, 1.0, Wset, S, woff, N)
    assert abs(np.angle(e[i11]) + math.atan(3.0)) < 1e-14
    # the seeds come from the mean spectrum phase
    e = oracle.phase_recursion(B, 2.0 * np.exp(0.3j), -1.0, Wset, S, woff, N)
    i10 = [k for k, w in enumerate(Wset) if tuple(w) == (1, 0)][0]
    i01 = [k for k, w in enumerate(Wset) if tuple(w) == (0, 1)][0]
    assert abs(e[i10] - np.exp(0.3j)) < 1e-15 and abs(e[i01] + 1.0) < 1e-15


# ---------------------------------------------------------------------------
# Fourier modulus, Eq. 1.
# ---------------------------------------------------------------------------
def test_amplitude_eq1_closed_form():
    """Noiseless periodic frames o (*) h_f, no taper: <|I|^2> / <|H|^2> =
    |O|^2 exactly when the STF is the sample mean of |H_f|^2."""
    N, F = 32, 8
    rng = _rng(6)
    obj = 1.0 + 0.1 * rng.standard_normal((N, N))
    O = np.fft.fft2(obj)
    H = []
    frames = []
    for f in range(F):
        h = rng.random((N, N)) ** 8
        h /= h.sum()
        Hf = np.fft.fft2(h)
        H.append(Hf)
        frames.append(np.real(np.fft.ifft2(O * Hf)))
    stf = np.mean(np.abs(np.stack(H)) ** 2, axis=0)
    p = oracle.Params(patch=N, window=0, v_radius=4)
    acc = oracle.accumulate_patch(np.stack(frames), p)
    Wset = oracle.frequency_half_disk(p.u_cut)
    amp = oracle.amplitude(acc["P"], stf, Wset, 0.0, 1e-12)
    ref = np.abs(O[Wset[:, 1] % N, Wset[:, 0] % N])
    np.testing.assert_allclose(amp, ref, rtol=1e-10)
    # the floor zeroes the modulus and the bias is subtracted before the root
    stf2 = stf.copy()
    stf2[Wset[0, 1] % N, Wset[0, 0] % N] = 1e-9
    amp2 = oracle.amplitude(acc["P"], stf2, Wset, 0.0, 1e-6)
    assert amp2[0] == 0.0
    big = float(acc["P"].max()) * 2
    assert np.all(oracle.amplitude(acc["P"], stf, Wset, big, 1e-12) == 0.0)


def test_noise_bias_reads_the_corners_only():
    N = 64
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    P = 7.5 + np.where(r <= N / 2, 1e6 * np.exp(-r / 5.0), 0.0)
    assert abs(oracle.noise_bias(P) - 7.5) < 1e-12


# ---------------------------------------------------------------------------
# Synthesis and mosaic (Section 3.2).
# ---------------------------------------------------------------------------
def test_diffraction_filter_is_the_disk_overlap():
    N = 64
    Wset = np.array([[0, 1], [5, 3], [12, 10], [20, 21], [31, 1], [40, 0]])
    T = oracle.diffraction_filter(Wset, N)
    # overlap area of two unit disks at distance 2 rho, grid integration
    g = np.linspace(-1, 1, 1601)
    X, Y = np.meshgrid(g, g)
    inside = X ** 2 + Y ** 2 <= 1.0
    for (wx, wy), t in zip(Wset, T):
        rho = math.hypot(wx, wy) / (N / 2)
        if rho >= 1:
            assert t == 0.0
            continue
        ov = inside & ((X - 2 * rho) ** 2 + Y ** 2 <= 1.0)
        assert abs(ov.sum() / inside.sum() - t) < 5e-3


def test_hann_taper_is_cola_at_half_overlap():
    h = oracle.hann(32)
    s = h[:16] + h[16:]
    np.testing.assert_allclose(s, 1.0, atol=1e-15)


def _sinusoid_image(H, W, N):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = 3.0 + 0.0 * x
    for (kx, ky, a, th) in [(1, 0, 0.5, 0.3), (2, 3, 0.2, 1.0), (-3, 2, 0.1, -0.7), (0, 4, 0.3, 2.0)]:
        img += a * np.cos(2 * np.pi * (kx * x + ky * y) / N + th)
    return img


@pytest.mark.parametrize("clampcase", [False, True])
def test_synthesis_and_mosaic_reproduce_a_band_limited_image(clampcase):
    """Feeding the true tapered patch spectra through synthesis and the
    mosaic returns the image wherever the summed taper is nonzero.  The
    image holds sinusoids periodic in the patch, so each tapered patch's
    spectrum lies inside |u| <= u_cut."""
    N, s = 16, 8
    H, W = (48, 52) if clampcase else (48, 48)
    img = _sinusoid_image(H, W, N)
    ys, xs = oracle.tiling(H, W, N, s)
    Wset = oracle.frequency_half_disk(N // 2 - 1)
    pat = np.zeros((len(ys), len(xs), N, N))
    for i, y0 in enumerate(ys):
        for j, x0 in enumerate(xs):
            I, mu = oracle.patch_spectra(img[None, y0:y0 + N, x0:x0 + N], window=1)
            vals = I[0][Wset[:, 1] % N, Wset[:, 0] % N]
            amp = np.abs(vals)
            ph = np.where(amp > 0, vals / np.where(amp > 0, amp, 1), 1.0)
            pat[i, j] = oracle.synthesize_patch(amp, ph, Wset, N, mu[0], 1)
    out = oracle.mosaic(pat, ys, xs, H, W, 1)
    np.testing.assert_allclose(out[1:, 1:], img[1:, 1:], atol=1e-10)
    assert np.all(out[0, :] == 0) and np.all(out[:, 0] == 0)


def test_constant_image_stays_constant():
    N = 16
    img = np.full((40, 40), 5.25)
    ys, xs = oracle.tiling(40, 40, N, 8)
    Wset = oracle.frequency_half_disk(N // 2 - 1)
    pat = np.zeros((len(ys), len(xs), N, N))
    for i, y0 in enumerate(ys):
        for j, x0 in enumerate(xs):
            I, mu = oracle.patch_spectra(img[None, y0:y0 + N, x0:x0 + N], window=1)
            assert np.max(np.abs(I)) < 1e-12
            pat[i, j] = oracle.synthesize_patch(np.zeros(len(Wset)), np.ones(len(Wset)), Wset, N, mu[0], 1)
    out = oracle.mosaic(pat, ys, xs, 40, 40, 1)
    np.testing.assert_allclose(out[1:, 1:], 5.25, atol=1e-12)


# ---------------------------------------------------------------------------
# Tiling: the paper's own arithmetic (Sections 3.2 and 4).
# ---------------------------------------------------------------------------
def test_tiling_matches_the_papers_cube_counts():
    # 1110 overlapping 256x256 cubes from 2560x2160 (Sections 3.2, 4)
    ys, xs = oracle.tiling(2160, 2560, 256, 64, clamp=False)
    assert len(ys) * len(xs) == 1110 and (len(xs), len(ys)) == (37, 30)
    # the 2368x1920 mosaic is the central 64x64 of every cube (Section 4)
    assert (len(xs) * 64, len(ys) * 64) == (2368, 1920)
    # 80 non-overlapping 256x256 seeing cubes (Section 3.2)
    ys, xs = oracle.tiling(2160, 2560, 256, 256, clamp=False)
    assert len(ys) * len(xs) == 80
    # the reconstruction grids used here: 128 px patches at 50 % overlap
    ys, xs = oracle.tiling(1024, 1024, 128, 64)
    assert (len(ys), len(xs)) == (15, 15)
    ys, xs = oracle.tiling(2160, 2560, 128, 64)
    assert (len(ys), len(xs)) == (33, 39) and ys[-1] == 2160 - 128 and xs[-1] == 2560 - 128
    # "around 55 GB" of cubes holds for 8-byte pixels (Section 4)
    assert abs(1110 * 100 * 256 * 256 * 8 / 1e9 - 58.2) < 0.1


# ---------------------------------------------------------------------------
# Least-squares phase refinement (an alternative to the recursion).
# ---------------------------------------------------------------------------
def _consistent_case(N=32, uc=12, R=5, seed=7):
    """Bispectrum samples of a single real object: every closure is exact."""
    Wset, S, woff = oracle.bispectrum_set(uc, R)
    S = np.asarray(S)
    O = np.fft.fft2(_rng(seed).random((N, N)))
    wx, wy, vx, vy = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    B = O[(wy - vy) % N, (wx - vx) % N] * O[vy % N, vx % N] * np.conj(O[wy % N, wx % N])
    truth = np.array([O[y % N, x % N] / abs(O[y % N, x % N]) for x, y in Wset])
    return Wset, S, woff, B, O, truth


def _closure_gain(e, Wset, S, B):
    """J(e) = sum Re[e(w-v) e(v) conj e(w) conj B], from a full N x N table."""
    N = 64
    E = np.zeros((N, N), dtype=np.complex128)
    for i, (x, y) in enumerate(Wset):
        E[y % N, x % N] = e[i]
        E[(-y) % N, (-x) % N] = np.conj(e[i])
    wx, wy, vx, vy = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    return float(np.real(np.sum(E[(wy - vy) % N, (wx - vx) % N] * E[vy % N, vx % N] *
                                np.conj(E[wy % N, wx % N]) * np.conj(B))))


def test_least_squares_keeps_exact_phases():
    """With exact closures the true phasors (which the recursion finds) are
    a fixed point of the refinement."""
    Wset, S, woff, B, O, truth = _consistent_case()
    e = oracle.phase_least_squares(B, truth, Wset, S, woff, 5)
    assert np.abs(np.angle(e * np.conj(truth))).max() < 1e-12


def test_least_squares_pulls_perturbed_phases_back():
    """From the truth disturbed by up to 0.5 rad (seeds kept) the refinement
    returns towards the truth: RMS error from ~0.29 rad to < 0.02 rad in 10
    steps."""
    Wset, S, woff, B, O, truth = _consistent_case()
    d = _rng(9).uniform(-0.5, 0.5, len(truth))
    for i, (x, y) in enumerate(Wset):
        if (x, y) in ((1, 0), (0, 1)):
            d[i] = 0.0
    e0 = truth * np.exp(1j * d)
    e = oracle.phase_least_squares(B, e0, Wset, S, woff, 10)
    r0 = np.sqrt(np.mean(np.angle(e0 * np.conj(truth)) ** 2))
    r = np.sqrt(np.mean(np.angle(e * np.conj(truth)) ** 2))
    assert r0 > 0.25 and r < 0.02


def test_least_squares_raises_the_closure_agreement_on_noisy_data():
    """With noisy samples the refined phasors agree better with the samples
    than the recursion's, J(refined) > J(recursion), and the seeds stay."""
    Wset, S, woff, B, O, truth = _consistent_case()
    rng = _rng(11)
    Bn = B + (rng.normal(size=B.shape) + 1j * rng.normal(size=B.shape)) * 0.3 * np.abs(B).mean()
    N = 32
    er = oracle.phase_recursion(Bn, O[0, 1], O[1, 0], Wset, S, woff, N)
    el = oracle.phase_least_squares(Bn, er, Wset, S, woff, 20)
    assert _closure_gain(el, Wset, S, Bn) > _closure_gain(er, Wset, S, Bn)
    seeds = [i for i, (x, y) in enumerate(Wset) if (x, y) in ((1, 0), (0, 1))]
    assert np.array_equal(el[seeds], er[seeds])


def test_least_squares_step_matches_the_gradient_sample_by_sample():
    """One step, recomputed with an explicit loop over the samples that
    finds each role of u by comparing coordinates: the target of every
    phasor is the unit of the partial derivative of J by conj(e(u))."""
    Wset, S, woff, B, O, truth = _consistent_case(N=16, uc=5, R=3, seed=3)
    rng = _rng(13)
    e0 = np.exp(1j * rng.uniform(-np.pi, np.pi, len(Wset)))
    Bn = B * np.exp(1j * rng.uniform(-0.3, 0.3, len(B)))
    e1 = oracle.phase_least_squares(Bn, e0, Wset, S, woff, 1)
    Wl = [tuple(map(int, w)) for w in Wset]

    def phasor(x, y):
        if (x, y) in Wl:
            return e0[Wl.index((x, y))]
        return np.conj(e0[Wl.index((-x, -y))])

    g = np.zeros(len(Wl), dtype=np.complex128)
    for (wx, wy, vx, vy), b in zip(S.tolist(), Bn):
        a, bb, c = phasor(wx - vx, wy - vy), phasor(vx, vy), phasor(wx, wy)
        # J term Re[a bb conj(c) conj(b)]: dJ/d conj(x) for x = each factor
        for (x, y), part in (((wx, wy), a * bb * np.conj(b)),
                             ((wx - vx, wy - vy), np.conj(bb) * c * b),
                             ((vx, vy), np.conj(a) * c * b)):
            if (x, y) in Wl:
                g[Wl.index((x, y))] += part
            else:
                g[Wl.index((-x, -y))] += np.conj(part)
    for i, u in enumerate(Wl):
        if u in ((1, 0), (0, 1)):
            assert e1[i] == e0[i]
            continue
        t = g[i] / abs(g[i]) + e0[i]
        assert abs(e1[i] - t / abs(t)) < 1e-12


# ---------------------------------------------------------------------------
# Photon-noise terms (noise_bias 2).  The paper gives no noise model; the
# pins hold the estimates to the two facts that define them: with no taper
# they are the classical photon-counting corrections of the power spectrum
# and the bispectrum, and their means over Poisson frames are the spectra of
# the noise-free frame.
# ---------------------------------------------------------------------------
def _photon_frames(rng, lam, F, gain):
    return rng.poisson(np.broadcast_to(lam, (F,) + lam.shape)) / gain


def _smooth_scene(N):
    y, x = np.mgrid[0:N, 0:N]
    return (3.0 + 2.5 * np.exp(-((x - 6.3) ** 2 + (y - 8.1) ** 2) / 6.0)
            + 1.5 * np.exp(-((x - 10.5) ** 2 + (y - 5.2) ** 2) / 3.0))


def test_photon_terms_reduce_to_the_classical_correction_without_taper():
    """No taper, one photon per unit: P - K and
    B - P(w) - P(v) - P(w - v) + 2K with K the mean photon count per frame
    (the photon-counting corrections of speckle interferometry and speckle
    masking), on every sample."""
    rng = np.random.default_rng(11)
    N, R = 16, 4
    cube = _photon_frames(rng, _smooth_scene(N), 30, 1.0)
    S = oracle.bispectrum_set(N // 2 - 1, R)[1]
    raw = oracle.accumulate_patch(cube, oracle.Params(patch=N, v_radius=R, window=0), S)
    cor = oracle.accumulate_patch(cube, oracle.Params(patch=N, v_radius=R, window=0, noise_bias=2,
                                                      photons_per_adu=1.0), S)
    K = cube.sum(axis=(1, 2)).mean()
    P = raw["P"]
    assert np.allclose(cor["P"], P - K, rtol=0, atol=1e-9 * P.max())
    wx, wy, vx, vy = S.T
    ref = raw["B"] - (P[wy % N, wx % N] + P[vy % N, vx % N] + P[(wy - vy) % N, (wx - vx) % N]) + 2 * K
    assert np.max(np.abs(cor["B"] - ref)) <= 1e-9 * np.max(np.abs(raw["B"]))


def _mc(window, gain, nb=40, per=1000, N=16, R=3, seed=3):
    rng = np.random.default_rng(seed)
    lam = _smooth_scene(N)
    op = oracle.Params(patch=N, v_radius=R, window=window, noise_bias=2, photons_per_adu=gain)
    op0 = oracle.Params(patch=N, v_radius=R, window=window)
    S = oracle.bispectrum_set(op.u_cut, R)[1]
    truth = oracle.accumulate_patch((lam / gain)[None], op0, S)      # spectra of E[p]
    cor, raw = [], []
    for _ in range(nb):
        cube = _photon_frames(rng, lam, per, gain)
        cor.append(oracle.accumulate_patch(cube, op, S))
        raw.append(oracle.accumulate_patch(cube, op0, S))
    return S, truth, cor, raw


def _zscores(est, truth):
    est = np.array(est)
    se = np.std(est, axis=0, ddof=1) / np.sqrt(len(est))
    with np.errstate(divide="ignore", invalid="ignore"):      # P(0) = 0 exactly; the callers mask it
        return np.abs(est.mean(axis=0) - truth) / se


def _near_origin(ux, uy, window):
    """Frequencies where the taper's transform is non-zero."""
    if window:
        return (np.abs(ux) <= 1) & (np.abs(uy) <= 1)
    return (ux == 0) & (uy == 0)


@pytest.mark.parametrize("window,gain", [(0, 1.0), (1, 2.0)])
def test_photon_corrected_spectra_are_unbiased(window, gain):
    """40 x 1000 Poisson frames of a fixed scene: the corrected P and B
    agree with those of the noise-free frame within the Monte Carlo error,
    where the uncorrected ones are far off.  With the Hann taper the samples
    with a side next to the origin are left out (the mean removal adds
    terms there that the estimate does not carry)."""
    S, truth, cor, raw = _mc(window, gain)
    N = truth["P"].shape[0]
    wx, wy, vx, vy = S.T
    near = (_near_origin(wx, wy, window) | _near_origin(vx, vy, window)
            | _near_origin(wx - vx, wy - vy, window))
    zc = _zscores([c["B"] for c in cor], truth["B"])[~near]
    zr = _zscores([r["B"] for r in raw], truth["B"])[~near]
    assert len(zc) > 300
    assert zc.max() < 5.0 and zc.mean() < 1.2
    assert np.median(zr) > 5.0
    k = np.fft.fftfreq(N) * N
    ux, uy = np.meshgrid(k, k)
    off = ~_near_origin(ux, uy, window)
    pc = _zscores([c["P"] for c in cor], truth["P"])[off]
    pr = _zscores([r["P"] for r in raw], truth["P"])[off]
    assert pc.max() < 6.0
    assert pr.min() > 20.0


# ---------------------------------------------------------------------------
# The whole composition (tile, accumulate, seeds, Eq. 1, phase, synthesis,
# mosaic) against a closed form: identical noiseless frames.
# ---------------------------------------------------------------------------
def _band_limited_periodic(N, radius, H, W, seed, mean=3.0):
    """An N-periodic real image whose spectrum lies inside |u| <= radius,
    tiled over H x W (every N x N cut is a circular shift of one period)."""
    rng = _rng(seed)
    k = np.fft.fftfreq(N) * N
    ux, uy = np.meshgrid(k, k)
    X = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    X[ux ** 2 + uy ** 2 > radius * radius] = 0.0
    X[0, 0] = 0.0
    base = np.real(np.fft.ifft2(X)) * N
    base = mean + 0.3 * base / base.std()
    reps = (-(-H // N), -(-W // N))
    return np.tile(base, reps)[:H, :W]


def _closed_form_case(window):
    """F identical noiseless frames of a band-limited image, STF = 1.

    Every frame has the spectrum I of its (tapered, mean-removed) patch, so
    P = |I|^2, M = I and B(w, v) = I(w - v) I(v) conj I(w): Eq. 1 gives
    |I| and the recursion, seeded by M(1,0) and M(0,1), gives arg I on W.
    When I lies inside |u| <= u_cut the inverse transform returns the tapered
    patch exactly, and the normalised overlap-add returns the image wherever
    the summed taper is nonzero.
    * window 0: one 32 x 32 patch, content inside |u| <= u_cut = 15.
    * window 1: a 72 x 88 crop cut into 4 x 5 patches of 32 at stride 16
      (the last row and column clamped flush with the edge).  The Hann taper
      spreads each frequency by one step per axis, so the content is kept
      inside |u| <= u_cut - 2 (13 + sqrt 2 < 15).
    """
    N, uc, R = 32, 15, 5
    if window == 0:
        H, W, radius, stride = 32, 32, uc, 32
    else:
        H, W, radius, stride = 72, 88, uc - 2, 16
    img = _band_limited_periodic(N, radius, H, W, seed=41 + window)
    frames = np.repeat(img[None], 3, axis=0)
    p = oracle.Params(patch=N, stride=stride, u_cut=uc, v_radius=R, window=window)
    stf = np.ones((N, N))
    return img, frames, p, stf


@pytest.mark.parametrize("window", [0, 1])
def test_reconstruct_returns_identical_noiseless_frames(window):
    img, frames, p, stf = _closed_form_case(window)
    out = oracle.reconstruct(frames, p, stf)
    ys, xs = out["ys"], out["xs"]
    if window == 0:
        np.testing.assert_allclose(out["image"], img, rtol=0, atol=1e-10)
    else:
        assert ys == [0, 16, 32, 40] and xs == [0, 16, 32, 48, 56]
        # summed taper: 0 on row 0 and column 0, below 1e-3 only next to them
        h = 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(32) / 32)
        den = np.zeros(img.shape)
        for y0 in ys:
            for x0 in xs:
                den[y0:y0 + 32, x0:x0 + 32] += np.outer(h, h)
        ok = den >= 1e-3
        assert ok.sum() > 0.99 * (71 * 87)
        np.testing.assert_allclose(out["image"][ok], img[ok], rtol=0, atol=1e-10)
        assert np.all(out["image"][~ok] == 0)


def _swap_seeds(acc):
    acc["M10"], acc["M01"] = acc["M01"], acc["M10"]


def _conjugate_bispectrum(acc):
    acc["B"] = np.conj(acc["B"])


def _drop_mean_level(acc):
    acc["mu"] = 0.0


def _transpose_power(acc):
    acc["P"] = acc["P"].T.copy()


@pytest.mark.parametrize("window", [0, 1])
@pytest.mark.parametrize("mistake", [_swap_seeds, _conjugate_bispectrum, _drop_mean_level, _transpose_power])
def test_closed_form_catches_planted_mistakes(monkeypatch, window, mistake):
    """Negative controls: the closed form above fails when a plausible
    mistake is planted in a copy of the composition (the seeds M(1,0) and
    M(0,1) swapped, the bispectrum conjugated, the mean level not restored,
    the power spectrum transposed)."""
    import oracle.speckle as sp
    img, frames, p, stf = _closed_form_case(window)
    real = sp.accumulate_patch

    def planted(cube, params, S=None):
        acc = real(cube, params, S)
        mistake(acc)
        return acc

    monkeypatch.setattr(sp, "accumulate_patch", planted)
    out = sp.reconstruct(frames, p, stf)
    err = np.max(np.abs(out["image"][1:, 1:] - img[1:, 1:]))
    assert err > 1e-2, err
