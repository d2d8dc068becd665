"""Pins of the model speckle transfer function (oracle/seeing.py) against
facts outside it: the random generator's published known answers, normal
moments, the Kolmogorov structure function, the diffraction limit, the
band limit of the pupil, and the speckle-regime asymptote of the STF."""
import numpy as np
import pytest

import oracle


def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors of its published definition
    (counter, key -> output)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
        ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
        ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
         (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
    ]
    for ctr, key, want in cases:
        got = oracle.philox4x32(*[np.array([c], np.uint32) for c in ctr], key[0], key[1])
        assert tuple(int(g[0]) for g in got) == want


def test_normals_moments():
    g = oracle.normals(2024, 3, 1, 400000)
    n = g.size
    assert abs(g.mean()) < 4 / np.sqrt(n)
    assert abs(g.var() - 1.0) < 4 * np.sqrt(2.0 / n)
    assert abs(np.mean(g ** 4) - 3.0) < 0.05
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.mean(g[0::2] * g[1::2])) < 4 / np.sqrt(n / 2)


def test_screens_follow_the_kolmogorov_structure_function():
    """<(phi(x + r) - phi(x))^2> = 6.88 (r / r0)^(5/3) for separations well
    inside the grid, for both screens of a pair, which are uncorrelated.  FFT
    screens with three subharmonic levels reach 0.8-0.9 of it there (the
    grid's Nyquist limit and finite size remove some power); a wrong
    normalisation would miss by far more."""
    N, r0 = 128, 8.0
    d = {r: [] for r in (2, 4, 8)}
    cross = []
    for j in range(24):
        a, b = oracle.screen_pair(N, r0, 77, j, 0)
        cross.append(np.mean((a - a.mean()) * (b - b.mean())) / np.sqrt(a.var() * b.var()))
        for s in (a, b):
            for r in d:
                # differences inside the grid (the subharmonics are not periodic on it)
                d[r].append(0.5 * (np.mean((s[:, r:] - s[:, :-r]) ** 2) + np.mean((s[r:, :] - s[:-r, :]) ** 2)))
    for r, v in d.items():
        ratio = np.mean(v) / (6.88 * (r / r0) ** (5.0 / 3.0))
        assert 0.75 < ratio < 1.05, (r, ratio)
    assert abs(np.mean(cross)) < 0.15


def test_no_turbulence_gives_the_pupil_otf():
    """D/r0 -> 0: every OTF is the bare pupil's, so <OTF> = T and the STF is
    T^2 (T computed from the pupil by an explicit autocorrelation)."""
    N = 32
    P = oracle.pupil(N)
    # autocorrelation of the pupil, brute force over all lags
    T = np.zeros((N, N))
    for dy in range(N):
        for dx in range(N):
            T[dy, dx] = np.sum(P * np.roll(np.roll(P, -dy, 0), -dx, 1))
    T /= T[0, 0]
    A, S = oracle.model(N, 1e-9, 4, 5)
    assert np.max(np.abs(A - T)) < 1e-6
    assert np.max(np.abs(S - T * T)) < 1e-6


@pytest.mark.parametrize("x", [4.0, 16.0])
def test_stf_is_normalised_symmetric_and_band_limited(x):
    N = 64
    A, S = oracle.model(N, x, 8, 11)
    assert S[0, 0] == pytest.approx(1.0, abs=1e-12)
    assert np.all(S <= 1.0 + 1e-12) and np.all(S >= 0.0)
    Sm = S[(-np.arange(N)) % N][:, (-np.arange(N)) % N]
    assert np.max(np.abs(S - Sm)) < 1e-12 * S.max()
    # nothing beyond the diffraction cut-off |u| = D = N/2 px (+1 px for the
    # discrete pupil's extent)
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    assert np.max(S[r > N / 2 + 1.5]) < 1e-12


def test_stf_speckle_regime_plateau():
    """Between the seeing and diffraction limits the STF is the pupil OTF
    times the coherence area of the wave over the pupil area:
    int exp(-6.88 (r/r0)^(5/3)) d^2r / (pi D^2 / 4) = 0.4356 (r0/D)^2 for
    Kolmogorov phase.  The screens carry 0.8-0.9 of that structure function
    and resolve r0 by only 4-5 px here, both of which enlarge the coherence
    area, so the plateau lies above 0.4356 but well within a factor of 2.5."""
    from scipy.integrate import quad
    area = 2 * np.pi * quad(lambda s: np.exp(-6.88 * s ** (5 / 3)) * s, 0, np.inf)[0]
    assert area / (np.pi / 4) == pytest.approx(0.4356, abs=2e-4)
    N, x = 128, 14.0
    _, S = oracle.model(N, x, 80, 13)
    T = oracle.otf(np.zeros((N, N)), oracle.pupil(N)).real
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    band = (r > 0.35 * N / 2) & (r < 0.7 * N / 2)
    ratio = np.mean(S[band] / (T[band] * (1.0 / x) ** 2))
    assert 0.4356 < ratio < 2.5 * 0.4356, ratio


# ---------------------------------------------------------------------------
# Spectral ratio and the seeing fit.
# ---------------------------------------------------------------------------
def test_spectral_ratio_of_identical_frames_is_one():
    """Frames that do not change have |<I>|^2 = <|I|^2>: the finite-burst
    corrected ratio is 1 wherever there is power."""
    rng = np.random.default_rng(3)
    img = rng.random((32, 32))
    eps, P = oracle.spectral_ratio(np.repeat(img[None], 7, axis=0), 1)
    nz = P > 1e-12 * P.max()
    assert np.max(np.abs(eps[nz] - 1.0)) < 1e-9


def test_spectral_ratio_numerator_is_unbiased_for_random_frames():
    """Frames = fixed image + independent white noise of power sigma^2 per
    frequency: E|m|^2 = |S|^2 + sigma^2 / F and E P = |S|^2 + sigma^2, so
    eps P = (|m|^2 - P / F) / (1 - 1/F) averages to |S|^2 (the uncorrected
    |m|^2 sits sigma^2 / F above it)."""
    N, F, B = 16, 8, 400
    rng = np.random.default_rng(9)
    base = rng.standard_normal((N, N))
    S2 = np.abs(np.fft.fft2(base - base.mean())) ** 2
    sigma2 = S2[1:, 1:].mean()
    num, raw = [], []
    for _ in range(B):
        fr = base[None] + rng.standard_normal((F, N, N)) * np.sqrt(sigma2 / (N * N))
        eps, P = oracle.spectral_ratio(fr, 0)
        num.append(eps * P)
        I = np.fft.fft2(fr - fr.mean(axis=(1, 2), keepdims=True), axes=(1, 2))
        raw.append(np.abs(I.mean(axis=0)) ** 2)
    m = np.ones((N, N), bool)
    m[0, 0] = False
    se = sigma2 * np.sqrt(4.0 / (F * B))              # rough standard error of the mean numerator
    assert abs(np.mean(np.mean(num, axis=0)[m] - S2[m])) < 3 * se / np.sqrt(m.sum())
    assert np.mean(np.mean(raw, axis=0)[m] - S2[m]) == pytest.approx(sigma2 / F, rel=0.1)


def test_weighted_model_curve_without_taper_is_the_annular_mean():
    rng = np.random.default_rng(4)
    N, Q = 32, 6
    rho = rng.random((N, N))
    rho[0, 0] = 0.0
    P = rng.random((N, N)) + 0.1
    annuli = oracle.half_plane_annuli(Q)
    got = oracle.weighted_model_curve(rho, P, 0, annuli)
    want = np.array([np.mean([rho[uy % N, ux % N] for (uy, ux) in mem]) for mem in annuli])
    assert np.allclose(got, want, rtol=0, atol=1e-15)
    # the half-plane annuli hold one of each +-u: counts are half the full annuli
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    for q, mem in enumerate(annuli, 1):
        assert 2 * len(mem) == np.count_nonzero((r >= q - 0.5) & (r < q + 0.5))


def test_seeing_recovers_the_generators_d_over_r0():
    """A 384 x 384 burst of 60 frames made by the test generator at
    D/r0 = 15 (its own Kolmogorov screens): the spectral-ratio estimate lies
    within 10 % (measured 14.5)."""
    import dataclasses
    import synth
    cfg = dataclasses.replace(synth.CONFIGS["burst1024"], index=300, H=384, W=384)
    fr = synth.make_burst(cfg, frames=60).astype(np.float64)
    r = oracle.seeing(fr, 128, 1, screens=200, seed=5, lo=6.0, hi=40.0, J=12, Q=12)
    assert abs(r["d_over_r0"] / cfg.d_over_r0 - 1.0) < 0.10, r["d_over_r0"]
    assert r["stf"][0, 0] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("tstar", [7.3, 11.85, 4.0, 0.2])
def test_fit_curve_vertex_of_an_exact_parabola(tstar):
    """Model curves c_j = c + (j - t*) d make the squared distance to c an
    exact parabola (j - t*)^2 |d|^2 in the grid index; the fit must return
    D/r0 = lo (hi/lo)^(t*/(J-1)) (a sign slip in the vertex gives 2j - t*).
    At the grid's ends (no neighbour on one side) the grid point itself."""
    rng = np.random.default_rng(9)
    J, Q, lo, hi = 20, 12, 2.0, 50.0
    grid = oracle.fit_grid(lo, hi, J)
    c = rng.random(Q)
    d = rng.standard_normal(Q)
    curves = c[None, :] + (np.arange(J)[:, None] - tstar) * d[None, :]
    got = oracle.fit_curve(c, curves, grid)
    j = int(round(tstar))
    want_t = tstar if 0 < j < J - 1 else float(j)
    assert got == pytest.approx(lo * (hi / lo) ** (want_t / (J - 1.0)), rel=1e-12)
    # the minimum at the last point: the fit stops there
    curves = c[None, :] + (np.arange(J)[:, None] - (J + 3.0)) * d[None, :]
    assert oracle.fit_curve(c, curves, grid) == pytest.approx(hi, rel=1e-12)


def test_weighted_model_curve_through_the_taper():
    """The tapered branch, by hand.  With rho = c everywhere (rho(0) = 0 is
    left out of both sums) every annulus reads c.  With the power spectrum
    at two frequencies only, P(u) = 1 at k = (0, 0) from u and P = 16 at
    k = (ky, kx) = (1, -1) (squared taper weights 1/4 * 1/4 = 1/16 and
    1/16 * 1/16 = 1/256), u reads (rho1 / 16 + rho2 / 16) / (1/16 + 1/16),
    the mean of the two ratios; a power at the origin adds nothing."""
    N = 32
    rho = np.full((N, N), 0.37)
    rho[0, 0] = 0.0
    P = np.random.default_rng(2).random((N, N)) + 0.5
    annuli = oracle.half_plane_annuli(8)
    got = oracle.weighted_model_curve(rho, P, 1, annuli)
    np.testing.assert_allclose(got, 0.37, rtol=0, atol=1e-15)
    uy, ux = 3, 5
    rho = np.zeros((N, N))
    P = np.zeros((N, N))
    rho[uy, ux], P[uy, ux] = 0.2, 1.0
    rho[uy - 1, ux + 1], P[uy - 1, ux + 1] = 0.9, 16.0
    got = oracle.weighted_model_curve(rho, P, 1, [[(uy, ux)]])
    assert got[0] == pytest.approx(0.55, abs=1e-15)
    # u = (0, 1): the neighbour k = (0, 1) is the origin, left out
    rho2 = np.zeros((N, N))
    P2 = np.zeros((N, N))
    rho2[0, 1], P2[0, 1] = 0.3, 2.0
    P2[0, 0], rho2[0, 0] = 50.0, 0.0
    rho2[1, 2], P2[1, 2] = 0.7, 8.0           # k = (-1, -1): weight 1/256
    got = oracle.weighted_model_curve(rho2, P2, 1, [[(0, 1)]])
    want = (2.0 / 16 * 0.3 + 8.0 / 256 * 0.7) / (2.0 / 16 + 8.0 / 256)
    assert got[0] == pytest.approx(want, abs=1e-15)
