"""Synthetic speckle bursts and speckle-transfer-function tables.

The paper reconstructs NVST TiO bursts (2560x2160 and 1024x1024 pixels,
~100 short exposures of granulation and sunspots, 16-bit camera; Table 1,
Section 4).  Those data are not available, so bursts are simulated:

* object: periodic Gaussian random field, power spectrum |k|^-3, scaled to
  mean 1 and 10 % RMS contrast (granulation-like);
* per frame: an independent Kolmogorov phase screen (FFT method with Lane
  et al. 1992 subharmonics, phase PSD 0.023 r0^(-5/3) f^(-11/3)) over a
  circular pupil of diameter M/2 pixels in an MxM grid, so that the PSF
  |FFT(pupil exp(i phi))|^2 is Nyquist sampled (pixel = lambda / 2D);
* frame = object (*) PSF (circular convolution, isoplanatic);
* photon noise Poisson(frame * photons_per_px); 12-bit ADU frames
  (gain photons/2048, clipped to [0, 4095], uint16) or float32 photon counts.

The speckle transfer function table is the Monte Carlo mean of |OTF|^2 over
independent screens, resampled onto the patch frequency grid.

Seeds: stream k of config c starts from ``170100581 + 1000*c + k``
(k = 0 object, 1 screens, 2 noise, 3 STF); frame f (or STF screen j) draws
from ``numpy.random.default_rng([base, f])``, so frames can be generated
independently and in any order.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import os

import numpy as np
import scipy.fft as sfft

SEED_BASE = 170100581


@dataclasses.dataclass(frozen=True)
class BurstConfig:
    name: str
    index: int          # config index c used in the seeds
    H: int
    W: int
    F: int
    dtype: str          # "f32" photon counts or "u16" 12-bit ADU
    d_over_r0: float
    M: int              # PSF grid; pupil diameter M/2 px
    photons: float      # mean photons per pixel
    patch: int          # reconstruction patch size N
    v_radius: int       # bispectrum |v| limit R
    window: int         # 0 none, 1 periodic Hann

    @property
    def r0_px(self) -> float:
        return (self.M / 2) / self.d_over_r0


CONFIGS = {
    # one 64x64 subimage, 100 float32 frames, D/r0 = 10, pupil 32 in 64
    "single64": BurstConfig("single64", 0, 64, 64, 100, "f32", 10.0, 64, 1e4, 64, 8, 0),
    # 1024x1024 x 100 uint16, D/r0 = 15, 128 px patches at 50 % overlap
    "burst1024": BurstConfig("burst1024", 1, 1024, 1024, 100, "u16", 15.0, 256, 1e4, 128, 10, 1),
    # 2560x2160 x 100 uint16, D/r0 = 20, 5e3 photons/px
    "burst2560": BurstConfig("burst2560", 2, 2160, 2560, 100, "u16", 20.0, 256, 5e3, 128, 12, 1),
}


def config_by_name(name: str) -> BurstConfig:
    return CONFIGS[name]


def burst_seed(cfg: BurstConfig, stream: int) -> int:
    return SEED_BASE + 1000 * cfg.index + stream


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def make_object(H: int, W: int, rng: np.random.Generator, slope: float = -3.0,
                mean: float = 1.0, rms: float = 0.10) -> np.ndarray:
    """Periodic Gaussian random field with power spectrum |k|^slope."""
    white = rng.standard_normal((H, W))
    ky = np.fft.fftfreq(H)[:, None]
    kx = np.fft.rfftfreq(W)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (slope / 2.0)
    field = sfft.irfft2(sfft.rfft2(white, workers=_workers()) * amp, s=(H, W),
                        workers=_workers())
    field -= field.mean()
    field *= rms / field.std()
    return field + mean


def _psd(f: np.ndarray, r0: float) -> np.ndarray:
    out = np.zeros_like(f)
    nz = f > 0
    out[nz] = 0.023 * r0 ** (-5.0 / 3.0) * f[nz] ** (-11.0 / 3.0)
    return out


def phase_screen(M: int, r0: float, rng: np.random.Generator,
                 subharmonics: int = 3) -> np.ndarray:
    """Kolmogorov phase screen [rad] on an MxM grid of 1-px spacing.

    FFT method plus ``subharmonics`` levels of Lane, Glindemann & Dainty
    (1992) low-frequency compensation.  Returns float64 (M, M).
    """
    df = 1.0 / M
    fy = np.fft.fftfreq(M)[:, None]
    fx = np.fft.fftfreq(M)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    c = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    c *= np.sqrt(_psd(f, r0)) * df
    scr = np.real(sfft.fft2(c, workers=1))
    if subharmonics:
        n = np.arange(M, dtype=np.float64)
        sh = np.zeros((M, M))
        for p in range(1, subharmonics + 1):
            dfp = df / 3.0 ** p
            for iy in (-1, 0, 1):
                for ix in (-1, 0, 1):
                    if ix == 0 and iy == 0:
                        continue
                    fxp, fyp = ix * dfp, iy * dfp
                    fr = np.hypot(fxp, fyp)
                    cc = (rng.standard_normal() + 1j * rng.standard_normal())
                    cc *= np.sqrt(0.023 * r0 ** (-5.0 / 3.0) * fr ** (-11.0 / 3.0)) * dfp
                    ex = np.exp(2j * np.pi * fxp * n)
                    ey = np.exp(2j * np.pi * fyp * n)
                    sh += np.real(cc * np.outer(ey, ex))
        scr = scr + sh - sh.mean()
    return scr


def _pupil(M: int) -> np.ndarray:
    y, x = np.mgrid[0:M, 0:M].astype(np.float64)
    c = (M - 1) / 2.0
    return ((x - c) ** 2 + (y - c) ** 2 <= (M / 4.0) ** 2).astype(np.float64)


def pupil_psf(screen: np.ndarray) -> np.ndarray:
    """Unit-sum PSF |FFT(pupil exp(i phi))|^2, origin at [0, 0] (wrapped)."""
    M = screen.shape[0]
    field = _pupil(M) * np.exp(1j * screen)
    psf = np.abs(sfft.fft2(field, workers=1)) ** 2
    return psf / psf.sum()


def _embed(psf: np.ndarray, H: int, W: int) -> np.ndarray:
    M = psf.shape[0]
    if M == H and M == W:
        return psf
    h = M // 2
    big = np.zeros((H, W))
    big[:h, :h] = psf[:h, :h]
    big[:h, W - h:] = psf[:h, h:]
    big[H - h:, :h] = psf[h:, :h]
    big[H - h:, W - h:] = psf[h:, h:]
    return big


def make_burst(cfg: BurstConfig, frames: int | None = None,
               return_object: bool = False):
    """Frames [F][H][W] (uint16 ADU or float32 photons) for ``cfg``.

    ``frames`` overrides the frame count (the first ``frames`` frames of the
    same seeded sequence).
    """
    F = cfg.F if frames is None else frames
    obj = make_object(cfg.H, cfg.W, np.random.default_rng(burst_seed(cfg, 0)))
    ospec = sfft.rfft2(obj, workers=_workers())
    out = np.empty((F, cfg.H, cfg.W), np.uint16 if cfg.dtype == "u16" else np.float32)
    gain = cfg.photons / 2048.0

    def one(f):
        srng = np.random.default_rng([burst_seed(cfg, 1), f])
        psf = pupil_psf(phase_screen(cfg.M, cfg.r0_px, srng))
        otf = sfft.rfft2(_embed(psf, cfg.H, cfg.W), workers=1)
        img = sfft.irfft2(ospec * otf, s=(cfg.H, cfg.W), workers=1)
        np.maximum(img, 0.0, out=img)
        nrng = np.random.default_rng([burst_seed(cfg, 2), f])
        photons = nrng.poisson(img * cfg.photons)
        if cfg.dtype == "u16":
            out[f] = np.clip(np.rint(photons / gain), 0, 4095).astype(np.uint16)
        else:
            out[f] = photons.astype(np.float32)

    with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(one, range(F)))
    if return_object:
        return out, obj
    return out


def stf_table(cfg: BurstConfig, screens: int = 1000, patch: int | None = None) -> np.ndarray:
    """Monte Carlo speckle transfer function <|OTF|^2> on the patch grid.

    Returns float64 [N][N] in DFT order (index k <-> frequency k mod N),
    with value 1 at the origin.  The PSF grid M samples frequency at 1/M
    cycles/px, the patch grid at 1/N, so STF_patch(u) = STF_M(u M / N).
    """
    N = cfg.patch if patch is None else patch
    M = cfg.M
    def one(j):
        rng = np.random.default_rng([burst_seed(cfg, 3), j])
        psf = pupil_psf(phase_screen(M, cfg.r0_px, rng))
        return np.abs(sfft.fft2(psf, workers=1)) ** 2

    acc = np.zeros((M, M))
    with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
        for a in ex.map(one, range(screens)):
            acc += a
    acc /= screens
    acc /= acc[0, 0]
    step = M // N
    k = (np.fft.fftfreq(N) * N).astype(np.int64) * step % M
    return acc[np.ix_(k, k)].copy()
