"""FP64 reference of the seeing estimate by the spectral ratio and of the
model speckle transfer function (Sections 2 and 3.2).

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

The seeing D/r0 comes from the burst itself by the spectral ratio, on the
full N x N cubes of the frame on a grid of step N (the paper's
non-overlapping cubes):
* Per cube, with the taper and mean removal of the reconstruction, F frames,
  m = <I_f> and P = <|I_f|^2>:
      eps(u) = (|m(u)|^2 - P(u) / F) / (P(u) (1 - 1/F)),
  the ratio |E I|^2 / E|I|^2 = |<OTF>|^2 / <|OTF|^2> with the finite-burst
  term of |m|^2 removed; eps is averaged over annuli q - 1/2 <= |u| < q + 1/2,
  q = 1..Q (over the half plane uy > 0 or uy = 0 < ux, which holds one of
  each pair +-u).
* Model curves on a geometric grid of J values of D/r0 (model point m = j):
  rho_j = |<OTF>|^2 / <|OTF|^2> from the Monte Carlo.  The taper mixes each
  frequency with its neighbours (transform weights 1/2, -1/4 per axis, so
  |w|^2 = 1/4, 1/16); with |O|^2 = P / STF the measured ratio is then
      sum_k |w(k)|^2 P(u - k) rho_j(u - k) / sum_k |w(k)|^2 P(u - k)
  (P of the cube, rho_j(0) = 0: the mean removal takes out the origin),
  averaged over the same annuli.  (A flat object instead of the measured P
  read D/r0 14-25 % low on 128-px cubes of the test bursts; this 2-12 %.)
* The cube's D/r0 minimises sum_q (eps(q) - curve_j(q))^2 (first minimum,
  then the vertex of the parabola through it and its neighbours, in grid
  index); the burst's value is 1 / <1 / (D/r0)> over the cubes (the mean r0),
  and its model STF is the Monte Carlo at that value (model point m = J).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["philox4x32", "normals", "screen_pair", "pupil", "otf", "model", "seeing_cubes", "fit_grid",
           "half_plane_annuli", "spectral_ratio", "weighted_model_curve", "fit_curve", "seeing"]

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


def seeing_cubes(H, W, N):
    """Origins (y, x) of the full N x N cubes on a grid of step N, row-major."""
    return [(i * N, j * N) for i in range(H // N) for j in range(W // N)]


def fit_grid(lo, hi, J):
    """D/r0 grid lo (hi/lo)^(j/(J-1)), j = 0..J-1."""
    return lo * (hi / lo) ** (np.arange(J) / (J - 1.0))


def half_plane_annuli(Q):
    """For q = 1..Q the frequencies (uy, ux) of the half plane (uy > 0, or
    uy = 0 < ux) with q - 1/2 <= |u| < q + 1/2."""
    out = []
    for q in range(1, Q + 1):
        m = []
        for uy in range(0, Q + 1):
            for ux in range(-Q, Q + 1):
                if uy == 0 and ux <= 0:
                    continue
                r = math.hypot(ux, uy)
                if q - 0.5 <= r < q + 0.5:
                    m.append((uy, ux))
        out.append(m)
    return out


def spectral_ratio(cube, window):
    """(eps [N][N], P [N][N]) of one cube [F][N][N] (F >= 2)."""
    from .speckle import patch_spectra
    I, _ = patch_spectra(np.asarray(cube, dtype=np.float64), window)
    F = I.shape[0]
    P = np.mean(np.abs(I) ** 2, axis=0)
    m2 = np.abs(np.mean(I, axis=0)) ** 2
    eps = np.zeros_like(P)
    nz = P > 0
    eps[nz] = (m2[nz] - P[nz] / F) / (P[nz] * (1.0 - 1.0 / F))
    return eps, P


def weighted_model_curve(rho, P, window, annuli):
    """Annular means of sum_k |w(k)|^2 P(u - k) rho(u - k) / sum_k |w(k)|^2
    P(u - k) (the identity without a taper), rho(0) taken as 0."""
    N = P.shape[0]
    w = {-1: 1.0 / 16.0, 0: 1.0 / 4.0, 1: 1.0 / 16.0} if window else {0: 1.0}
    out = []
    for members in annuli:
        vals = []
        for (uy, ux) in members:
            num = den = 0.0
            for ky in w:
                for kx in w:
                    vy, vx = uy - ky, ux - kx
                    if vy == 0 and vx == 0:
                        continue
                    wt = w[ky] * w[kx] * P[vy % N, vx % N]
                    num += wt * rho[vy % N, vx % N]
                    den += wt
            vals.append(num / den if den > 0 else 0.0)
        out.append(np.mean(vals))
    return np.array(out)


def fit_curve(curve, curves, grid):
    """D/r0 of a ratio curve against the model curves [J][Q] on ``grid``."""
    J = len(grid)
    e = np.sum((np.asarray(curves) - np.asarray(curve)[None, :]) ** 2, axis=1)
    j = int(np.argmin(e))
    t = float(j)
    if 0 < j < J - 1:
        den = e[j - 1] - 2.0 * e[j] + e[j + 1]
        if den > 0:
            t = j + 0.5 * (e[j - 1] - e[j + 1]) / den
    lo, hi = float(grid[0]), float(grid[-1])
    return lo * (hi / lo) ** (t / (J - 1.0))


def seeing(frames, N, window, screens, seed, lo, hi, J, Q):
    """The estimate for a burst [F][H][W]: per cube the ratio curve and D/r0,
    the burst's D/r0, and the model STF (and mean OTF) there."""
    F, H, W = frames.shape
    grid = fit_grid(lo, hi, J)
    rhos = []
    for m, x in enumerate(grid):
        A, S = model(N, x, screens, seed, m)
        r = np.abs(A) ** 2 / S
        r[0, 0] = 0.0
        rhos.append(r)
    annuli = half_plane_annuli(Q)
    curves, xs = [], []
    for (y0, x0) in seeing_cubes(H, W, N):
        eps, P = spectral_ratio(frames[:, y0:y0 + N, x0:x0 + N], window)
        c = np.array([np.mean([eps[uy % N, ux % N] for (uy, ux) in mem]) for mem in annuli])
        table = np.array([weighted_model_curve(r, P, window, annuli) for r in rhos])
        curves.append(c)
        xs.append(fit_curve(c, table, grid))
    xs = np.array(xs)
    x = 1.0 / np.mean(1.0 / xs)
    A, S = model(N, x, screens, seed, J)
    return dict(curves=np.array(curves), d_over_r0_cubes=xs, d_over_r0=x, stf=S, mean_otf=A, grid=grid)
