"""FP64 reference of the model speckle transfer function (Sections 2 and 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy,
written to be checked by eye.

The paper divides the mean power spectrum by a model STF <|H|^2> chosen by
the seeing parameter r0 (no point source can be observed on the Sun), and
gives no formulas for it.  The reading taken here:

* A Monte Carlo over Kolmogorov phase screens: phase spectrum
  0.023 r0^(-5/3) f^(-11/3), FFT method with three levels of subharmonics
  after Lane, Glindemann and Dainty (1992), across a circular pupil of
  diameter N/2 pixels in the N x N patch grid, so that the point spread
  function |FFT2(pupil exp(i phi))|^2 is Nyquist sampled on the patch grid
  (D/r0 fixes r0 = (N/2) / (D/r0) pixels).  The OTF is FFT2(PSF) / OTF(0);
  the model STF is <|OTF|^2> over the screens.
* A screen pair comes from one complex FFT (its real and imaginary parts).
* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw 2011) with
  key (seed mod 2^32, seed div 2^32) and counter (screen pair j, word w,
  stream m, 0); the four words of a counter give two normal pairs by
  Box-Muller with u = (x + 1/2) 2^-32.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["philox4x32", "normals", "screen_pair", "pupil", "otf", "model", "long_exposure_otf", "annulus_mean"]

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x32 (Salmon et al. 2011), element-wise over uint32 arrays:
    each round multiplies words 0 and 2 by fixed constants, keeps the low
    halves and xors the high halves into words 1 and 3 with the key; the
    key is raised by the Weyl constants between rounds."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for r in range(rounds):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = np.uint64(_M0) * c[0]
        p1 = np.uint64(_M1) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _MASK, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _MASK]
    return [x.astype(np.uint32) for x in c]


def normals(seed, j, m, n):
    """n standard normals (n a multiple of 4) of screen pair j, stream m:
    words w = 0 .. n/4 - 1, each two Box-Muller pairs (cos, sin)."""
    w = np.arange(n // 4, dtype=np.uint64)
    x = philox4x32(np.full_like(w, j), w, np.full_like(w, m), np.zeros_like(w),
                   seed & _MASK, (seed >> 32) & _MASK)
    u = [(xi.astype(np.float64) + 0.5) * 2.0 ** -32 for xi in x]
    out = np.empty((n // 4, 4))
    for a in (0, 2):
        r = np.sqrt(-2.0 * np.log(u[a]))
        t = 2.0 * np.pi * u[a + 1]
        out[:, a] = r * np.cos(t)
        out[:, a + 1] = r * np.sin(t)
    return out.reshape(-1)


def _psd(f, r0):
    return 0.023 * r0 ** (-5.0 / 3.0) * f ** (-11.0 / 3.0)


def screen_pair(N, r0, seed, j, m):
    """Two Kolmogorov phase screens [rad] on the N x N grid (1-px spacing,
    r0 in pixels).  Coefficients c(f) = sqrt(PSD(f)) df (g + i g') on the DFT
    frequencies f (df = 1/N, none at f = 0), normals 2e and 2e + 1 for
    element e = y N + x; z = FFT2(c) (forward, unnormalised); then three
    subharmonic levels p: for the 8 neighbours (iy, ix) of the origin in
    the order iy, ix = -1, 0, 1, at frequency (ix, iy) df / 3^p, coefficient
    sqrt(PSD) df / 3^p (g + i g') (normals 2 N^2 + 2 s, + 1, s = 8 (p - 1) + k),
    z += c exp(+2 pi i f.x).  Returns (Re z, Im z)."""
    g = normals(seed, j, m, 2 * N * N + 48)
    df = 1.0 / N
    fy = np.fft.fftfreq(N)[:, None]
    fx = np.fft.fftfreq(N)[None, :]
    f = np.hypot(fx, fy)
    sig = np.zeros((N, N))
    nz = f > 0
    sig[nz] = np.sqrt(_psd(f[nz], r0)) * df
    c = sig * (g[0:2 * N * N:2].reshape(N, N) + 1j * g[1:2 * N * N:2].reshape(N, N))
    z = np.fft.fft2(c)
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    s = 0
    for p in range(1, 4):
        dfp = df / 3.0 ** p
        for iy in (-1, 0, 1):
            for ix in (-1, 0, 1):
                if ix == 0 and iy == 0:
                    continue
                fr = math.hypot(ix * dfp, iy * dfp)
                cs = math.sqrt(_psd(fr, r0)) * dfp * complex(g[2 * N * N + 2 * s], g[2 * N * N + 2 * s + 1])
                z = z + cs * np.exp(2j * np.pi * (ix * dfp * x + iy * dfp * y))
                s += 1
    return z.real, z.imag


def pupil(N):
    """Circular pupil of diameter N/2 px centred in the N x N grid."""
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    c = (N - 1) / 2.0
    return ((x - c) ** 2 + (y - c) ** 2 <= (N / 4.0) ** 2).astype(np.float64)


def otf(phi, P):
    """FFT2 of the PSF |FFT2(P exp(i phi))|^2, normalised to 1 at u = 0."""
    psf = np.abs(np.fft.fft2(P * np.exp(1j * phi))) ** 2
    o = np.fft.fft2(psf)
    return o / o[0, 0].real


def model(N, d_over_r0, screens, seed, m=0):
    """Monte Carlo <OTF> (complex) and <|OTF|^2> (the model STF) over
    ``screens`` screens (an even number: screens / 2 pairs) at D/r0 with
    D = N/2 px, stream m."""
    r0 = (N / 2.0) / d_over_r0
    P = pupil(N)
    A = np.zeros((N, N), dtype=np.complex128)
    S = np.zeros((N, N))
    for j in range(screens // 2):
        for phi in screen_pair(N, r0, seed, j, m):
            o = otf(phi, P)
            A += o
            S += np.abs(o) ** 2
    return A / screens, S / screens


def long_exposure_otf(N, d_over_r0):
    """T(u) exp(-3.44 (|u| / r0)^(5/3)) (Fried 1966; T the OTF of pupil(N),
    r0 = (N/2) / (D/r0) px, |u| the wrapped DFT lag): the mean OTF of
    Kolmogorov turbulence of unlimited outer scale."""
    T = otf(np.zeros((N, N)), pupil(N)).real
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    r0 = (N / 2.0) / d_over_r0
    return T * np.exp(-3.44 * (r / r0) ** (5.0 / 3.0))


def annulus_mean(E, Q):
    """Means of E [N][N] (DFT order) over q - 1/2 <= |u| < q + 1/2, q = 1..Q."""
    N = E.shape[0]
    k = np.fft.fftfreq(N) * N
    r = np.hypot(k[None, :], k[:, None])
    return np.array([E[(r >= q - 0.5) & (r < q + 0.5)].mean() for q in range(1, Q + 1)])
