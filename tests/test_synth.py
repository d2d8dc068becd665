"""Statistics of the synthetic burst generator (textbook closed forms)."""
import numpy as np

import synth


def test_kolmogorov_structure_function():
    """D(r) = 6.88 (r / r0)^(5/3) (Fried) for r well inside the screen."""
    r0, M = 8.0, 256
    D = []
    for j in range(30):
        s = synth.phase_screen(M, r0, np.random.default_rng(j))
        D.append([np.mean((s[:, r:] - s[:, :-r]) ** 2) for r in (2, 4, 8, 16, 32)])
    D = np.mean(D, axis=0)
    ref = 6.88 * (np.array([2, 4, 8, 16, 32]) / r0) ** (5.0 / 3.0)
    ratio = D / ref
    assert np.all(ratio > 0.75) and np.all(ratio < 1.15), ratio
    # the log-log slope is 5/3
    slope = np.polyfit(np.log([2, 4, 8, 16]), np.log(D[:4]), 1)[0]
    assert abs(slope - 5.0 / 3.0) < 0.12, slope


def test_object_power_law_mean_and_contrast():
    obj = synth.make_object(512, 512, np.random.default_rng(0))
    assert abs(obj.mean() - 1.0) < 1e-12 and abs(obj.std() - 0.1) < 1e-12
    P = np.abs(np.fft.fft2(obj - obj.mean())) ** 2
    k = np.hypot(*np.meshgrid(np.fft.fftfreq(512), np.fft.fftfreq(512)))
    bins = np.geomspace(4 / 512, 0.25, 12)
    idx = np.digitize(k, bins)
    kk = [k[idx == i].mean() for i in range(1, len(bins))]
    pp = [P[idx == i].mean() for i in range(1, len(bins))]
    slope = np.polyfit(np.log(kk), np.log(pp), 1)[0]
    assert abs(slope + 3.0) < 0.15, slope


def test_psf_unit_sum_and_nyquist_cutoff():
    s = synth.phase_screen(64, 3.2, np.random.default_rng(1))
    psf = synth.pupil_psf(s)
    assert abs(psf.sum() - 1.0) < 1e-12 and psf.min() >= 0
    otf = np.abs(np.fft.fft2(psf))
    k = np.fft.fftfreq(64) * 64
    r = np.hypot(k[None, :], k[:, None])
    # the autocorrelation of a pupil of diameter M/2 ends at M/2
    assert otf[r > 32.5].max() < 1e-12


def test_poisson_and_12bit_frames():
    cfg = synth.CONFIGS["burst1024"]
    f = synth.make_burst(cfg, frames=2)
    assert f.dtype == np.uint16 and f.shape == (2, 1024, 1024)
    assert f.max() <= 4095
    assert abs(f.mean() - 2048) < 10
    # photon noise: variance of the difference of a frame from its smooth
    # version exceeds the ADU quantisation floor and follows Poisson scaling
    g = cfg.photons / 2048.0
    d = f[0].astype(np.float64)[:, 1:] - f[0].astype(np.float64)[:, :-1]
    assert d.var() > 2 * 2048 / g * 0.5


def test_poisson_moments_float_frames():
    cfg = synth.CONFIGS["single64"]
    a = synth.make_burst(cfg, frames=3)
    assert a.dtype == np.float32
    assert np.all(a == np.round(a))
    assert abs(a.mean() / cfg.photons - 1.0) < 0.01


def test_stf_table_normalisation_and_symmetry():
    cfg = synth.CONFIGS["single64"]
    stf = synth.stf_table(cfg, screens=40)
    assert stf[0, 0] == 1.0
    N = stf.shape[0]
    idx = (-np.arange(N)) % N
    np.testing.assert_allclose(stf, stf[np.ix_(idx, idx)], rtol=1e-10, atol=1e-15)
    assert np.all(stf >= 0) and stf.max() <= 1.0 + 1e-12
