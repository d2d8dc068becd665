"""FP64 reference implementation of the speckle-masking reconstruction.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in
complex128 / float64, written to be checked against the paper by eye.

Conventions (the paper is silent on them; these are the readings used):
* frames are [F][H][W], x (width) fastest; a frequency u = (ux, uy) lives at
  array index [uy mod N, ux mod N];
* forward transform exp(-2 pi i u.x / N), unnormalised (numpy.fft.fft2);
  inverse includes 1/N^2 (numpy.fft.ifft2);
* <.> is the mean over the frames of the burst.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "tiling", "hann", "window2d", "patch_spectra", "frequency_half_disk",
    "bispectrum_set", "accumulate_patch", "bispectrum", "noise_bias",
    "photon_noise_terms", "debias_bispectrum",
    "amplitude", "phase_recursion", "phase_least_squares", "diffraction_filter",
    "synthesize_patch", "mosaic", "reconstruct", "Params",
]


class Params:
    """Reconstruction parameters (defaults follow the patch size N)."""

    def __init__(self, patch=128, stride=None, u_cut=None, v_radius=10,
                 window=1, noise_bias=0, filter=0, stf_floor=1e-6,
                 phase_method=0, lsq_iters=10, photons_per_adu=1.0):
        self.patch = int(patch)
        self.stride = int(patch // 2 if stride is None else stride)
        self.u_cut = int(patch // 2 - 1 if u_cut is None else u_cut)
        self.v_radius = int(v_radius)
        self.window = int(window)
        self.noise_bias = int(noise_bias)      # 0 off, 1 corner level, 2 photon model
        self.photons_per_adu = float(photons_per_adu)
        self.filter = int(filter)
        self.stf_floor = float(stf_floor)
        self.phase_method = int(phase_method)   # 0 recursion, 1 + least squares
        self.lsq_iters = int(lsq_iters)


# ---------------------------------------------------------------------------
# Division into overlapping subimages (Section 3.2).
# ---------------------------------------------------------------------------
def tiling(H, W, N, s, clamp=True):
    """Origins of the overlapping N x N subimages of an H x W frame.

    The paper cuts a burst into partially overlapping subimage cubes
    (Section 3.2; 1110 cubes of 256^2 for 2560x2160, Section 4).  With
    ``clamp`` the grid is k*s for k < ceil((L-N)/s) and a last subimage
    flush with the edge (min(k*s, L-N)), so every pixel is covered; without
    it only the full steps floor((L-N)/s)+1 are kept.
    Returns (ys, xs) lists of row and column origins.
    """
    def axis(L):
        if L < N:
            raise ValueError("frame smaller than a patch")
        if clamp:
            n = -(-(L - N) // s) + 1
            return [min(k * s, L - N) for k in range(n)]
        n = (L - N) // s + 1
        return [k * s for k in range(n)]
    return axis(H), axis(W)


def hann(N):
    """Periodic Hann taper h[n] = 1/2 - 1/2 cos(2 pi n / N)."""
    n = np.arange(N, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / N)


def window2d(N, window):
    if window == 0:
        return np.ones((N, N))
    h = hann(N)
    return np.outer(h, h)


def patch_spectra(cube, window):
    """Spectra of one subimage cube [F][N][N] (float64).

    For each frame: weighted mean mu_f = sum(w p)/sum(w), apodised
    q = (p - mu_f) w, I_f = FFT2(q).  Returns (I [F][N][N] complex128,
    mu [F]).
    """
    F, N, _ = cube.shape
    w = window2d(N, window)
    mu = np.array([np.sum(w * cube[f]) / np.sum(w) for f in range(F)])
    q = (cube - mu[:, None, None]) * w[None]
    return np.fft.fft2(q, axes=(1, 2)), mu


# ---------------------------------------------------------------------------
# Bispectrum index sets.
# ---------------------------------------------------------------------------
def frequency_half_disk(u_cut):
    """W: frequencies 0 < |w| <= u_cut in the upper half plane.

    Upper half plane means wy > 0, or wy == 0 and wx > 0.  Order: by |w|^2,
    then wy, then wx (the order in which the phase recursion visits them).
    Returns int64 [|W|][2] as (wx, wy).
    """
    out = []
    for wy in range(0, u_cut + 1):
        for wx in range(-u_cut, u_cut + 1):
            r2 = wx * wx + wy * wy
            if r2 == 0 or r2 > u_cut * u_cut:
                continue
            if wy > 0 or wx > 0:
                out.append((wx, wy))
    out.sort(key=lambda w: (w[0] * w[0] + w[1] * w[1], w[1], w[0]))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def bispectrum_set(u_cut, R):
    """The bispectrum samples used by the phase recursion.

    For each w in W (in recursion order) the v with 0 < |v|^2 < |w|^2,
    |v| <= R and 0 < |w - v|^2 < |w|^2, ordered by (vy, vx): each sample is
    a triangle (w - v) + v = w whose two shorter sides are already known
    when w is reached.
    Returns (Wset [|W|][2], S [|S|][4] = (wx, wy, vx, vy), woff [|W|+1]).
    """
    Wset = frequency_half_disk(u_cut)
    rows = []
    woff = [0]
    for wx, wy in Wset:
        n2 = wx * wx + wy * wy
        for vy in range(-R, R + 1):
            for vx in range(-R, R + 1):
                a = vx * vx + vy * vy
                if a == 0 or a > R * R or a >= n2:
                    continue
                dx, dy = wx - vx, wy - vy
                b = dx * dx + dy * dy
                if b == 0 or b >= n2:
                    continue
                rows.append((wx, wy, vx, vy))
        woff.append(len(rows))
    S = np.array(rows, dtype=np.int64).reshape(-1, 4)
    return Wset, S, np.array(woff, dtype=np.int64)


# ---------------------------------------------------------------------------
# Accumulation over the burst (Eq. 1 numerator; speckle masking bispectrum).
# ---------------------------------------------------------------------------
def bispectrum(I, wv):
    """Mean bispectrum <I(w - v) I(v) conj(I(w))> over frames.

    ``I`` is [F][N][N] complex; ``wv`` is [n][4] of (wx, wy, vx, vy) with
    any signs (indices are taken mod N).  This is B(u1, u2) =
    <I(u1) I(u2) conj(I(u1 + u2))> with u1 = w - v, u2 = v.
    """
    F, N, _ = I.shape
    wx, wy, vx, vy = (wv[:, i] for i in range(4))
    iw = (wy % N) * N + (wx % N)
    iv = (vy % N) * N + (vx % N)
    id_ = ((wy - vy) % N) * N + ((wx - vx) % N)
    acc = np.zeros(len(wv), dtype=np.complex128)
    for f in range(F):
        flat = I[f].reshape(-1)
        acc += flat[id_] * flat[iv] * np.conj(flat[iw])
    return acc / F


def photon_noise_terms(cube, window, gain):
    """Photon-noise terms of the power spectrum and bispectrum of a cube.

    Model (the paper gives none): a pixel value is p = c / G with c photon
    counts, Poisson given the noise-free image, and G = ``gain`` photons per
    unit of p.  Per pixel the noise then has variance E[p] / G and third
    cumulant E[p] / G^2, both estimated without bias by the data itself.
    With t the taper, I = FFT2((p - mu) t) as in ``patch_spectra`` and
    Q(u) = FFT2(t^2 p)(u) / G, per frame:
        C(u) = conj(I(u)) Q(u),   q0 = sum(t^2 p) / G,   T = sum(t^3 p) / G^2.
    The noise adds q0 (in expectation) to |I(u)|^2 and
        C(w) + conj C(v) + conj C(w - v) - 2 T
    to I(w - v) I(v) conj I(w), where the taper's transform vanishes at
    the three frequencies (for the Hann taper: each has a component of
    modulus >= 2; with no taper: each is non-zero); there the mean removal
    adds terms that these estimates leave out.
    Returns (C [N][N] complex = <C(u)>, q0 = <q0>, T = <T>) over frames.
    """
    cube = np.asarray(cube, dtype=np.float64)
    F, N, _ = cube.shape
    t = window2d(N, window)
    I, _ = patch_spectra(cube, window)
    Q = np.fft.fft2(cube * (t * t)[None], axes=(1, 2)) / gain
    C = np.mean(np.conj(I) * Q, axis=0)
    q0 = float(np.mean(np.sum(cube * (t * t)[None], axis=(1, 2)))) / gain
    T = float(np.mean(np.sum(cube * (t * t * t)[None], axis=(1, 2)))) / (gain * gain)
    return C, q0, T


def debias_bispectrum(B, C, T, wv):
    """B(w, v) - [C(w) + conj C(v) + conj C(w - v)] + 2 T on the samples
    ``wv`` ([n][4] of (wx, wy, vx, vy)); C on the N x N grid (DFT order)."""
    N = C.shape[0]
    wx, wy, vx, vy = (np.asarray(wv)[:, i] for i in range(4))
    cw = C[wy % N, wx % N]
    cv = C[vy % N, vx % N]
    cd = C[(wy - vy) % N, (wx - vx) % N]
    return B - (cw + np.conj(cv) + np.conj(cd)) + 2.0 * T


def accumulate_patch(cube, params, S=None):
    """Power spectrum, mean spectrum, mean level and bispectrum of a cube.

    Returns dict with P [N][N] = <|I|^2>, M10 = <I(1,0)>, M01 = <I(0,1)>,
    mu = <mu_f>, B [|S|] complex (None when S is None).  With the photon
    noise model (noise_bias 2) P and B are the corrected means of
    ``photon_noise_terms`` (P - q0, and ``debias_bispectrum``).
    """
    I, mu = patch_spectra(np.asarray(cube, dtype=np.float64), params.window)
    P = np.mean(np.abs(I) ** 2, axis=0)
    M = np.mean(I, axis=0)
    out = dict(P=P, M10=M[0, 1], M01=M[1, 0], mu=float(np.mean(mu)), B=None)
    if S is not None:
        out["B"] = bispectrum(I, S)
    if params.noise_bias == 2:
        C, q0, T = photon_noise_terms(cube, params.window, params.photons_per_adu)
        out["P"] = P - q0
        if S is not None:
            out["B"] = debias_bispectrum(out["B"], C, T, S)
    return out


# ---------------------------------------------------------------------------
# Fourier modulus, Eq. 1.
# ---------------------------------------------------------------------------
def noise_bias(P):
    """Flat noise level: mean of P over the corners |u| > N/2 + 2.

    A Nyquist-sampled telescope transfers nothing beyond |u| = N/2, so the
    corners of the power spectrum hold only the (white) photon-noise bias.
    """
    N = P.shape[0]
    k = np.fft.fftfreq(N) * N
    r2 = k[None, :] ** 2 + k[:, None] ** 2
    mask = r2 > (N / 2 + 2) ** 2
    return float(P[mask].mean())


def amplitude(P, stf, Wset, nbias=0.0, floor=1e-6):
    """|O(w)| = sqrt(<|I(w)|^2> / <|H(w)|^2>) on W (Eq. 1).

    The bias ``nbias`` is removed first and negative values clip to 0;
    where the STF is below ``floor`` the modulus is set to 0.
    """
    N = P.shape[0]
    out = np.zeros(len(Wset))
    for i, (wx, wy) in enumerate(Wset):
        s = stf[wy % N, wx % N]
        if s < floor:
            continue
        out[i] = math.sqrt(max(P[wy % N, wx % N] - nbias, 0.0) / s)
    return out


# ---------------------------------------------------------------------------
# Fourier phase by speckle masking (recursive solution).
# ---------------------------------------------------------------------------
def _unit(z):
    a = abs(z)
    return complex(1.0, 0.0) if a == 0.0 else z / a


def phase_recursion(B, M10, M01, Wset, S, woff, N):
    """Object phasors e(w) on W from the mean bispectrum.

    Since B(w, v) ~ O(w - v) O(v) conj(O(w)) times a real transfer factor,
    phi(w) = phi(w - v) + phi(v) - arg B(w, v).  Every w (in increasing
    |w|) takes the phase of the |B|-weighted phasor sum
        z(w) = sum_v e(w - v) e(v) conj(B(w, v)),  e(w) = z / |z|,
    over its samples; e(-u) = conj(e(u)), e(0) = 1.  The two lowest
    frequencies (1,0) and (0,1) fix the translation and are seeded from the
    mean spectrum: e = M / |M| (1 when M == 0).
    Returns complex128 [|W|].
    """
    E = np.zeros((N, N), dtype=np.complex128)
    known = np.zeros((N, N), dtype=bool)

    def put(ux, uy, val):
        E[uy % N, ux % N] = val
        E[(-uy) % N, (-ux) % N] = np.conj(val)
        known[uy % N, ux % N] = True
        known[(-uy) % N, (-ux) % N] = True

    put(0, 0, 1.0)
    put(1, 0, _unit(complex(M10)))
    put(0, 1, _unit(complex(M01)))
    out = np.zeros(len(Wset), dtype=np.complex128)
    for i, (wx, wy) in enumerate(Wset):
        if (wx, wy) in ((1, 0), (0, 1)):
            out[i] = E[wy % N, wx % N]
            continue
        s = S[woff[i]:woff[i + 1]]
        vx, vy = s[:, 2], s[:, 3]
        a = E[(wy - vy) % N, (wx - vx) % N]
        b = E[vy % N, vx % N]
        assert known[(wy - vy) % N, (wx - vx) % N].all() and known[vy % N, vx % N].all()
        z = np.sum(a * b * np.conj(B[woff[i]:woff[i + 1]]))
        out[i] = _unit(z)
        put(wx, wy, out[i])
    return out


def phase_least_squares(B, e0, Wset, S, woff, iters):
    """Least-squares refinement of the phasors (an alternative to the
    recursion named in the paper's description of the phase step).

    Every sample is a closure phi(w - v) + phi(v) - phi(w) = arg B(w, v);
    the refinement raises the |B|-weighted closure agreement
        J(e) = sum_S Re[ e(w - v) e(v) conj(e(w)) conj(B(w, v)) ]
    over unit phasors with e(-u) = conj(e(u)), keeping the two seeds
    (1,0) and (0,1) (they fix the translation).  For fixed other phasors J is
    largest at e(u) = g(u) / |g(u)|, where g(u) sums, over every sample in
    which u appears:
        as w:        e(w - v) e(v) conj(B)
        as w - v:    conj(e(v)) e(w) B
        as v:        conj(e(w - v)) e(w) B
    (conjugated where the sample holds -u).  One step moves every phasor
    halfway to that target, all at once from the previous phasors:
        e'(u) = unit(unit(g(u)) + e(u))   (e(u) kept where g(u) = 0).
    ``iters`` steps from ``e0`` (normally the recursion's phasors).
    Returns complex128 [|W|].
    """
    Wset = np.asarray(Wset)
    S = np.asarray(S)
    pos = {(int(x), int(y)): i for i, (x, y) in enumerate(Wset)}

    def index_of(x, y):
        """W index of +-(x, y) and whether the sample holds the conjugate."""
        j = np.empty(len(x), dtype=np.int64)
        cj = np.empty(len(x), dtype=bool)
        for k, (a, b) in enumerate(zip(x.tolist(), y.tolist())):
            if (a, b) in pos:
                j[k], cj[k] = pos[(a, b)], False
            else:
                j[k], cj[k] = pos[(-a, -b)], True
        return j, cj

    wx, wy, vx, vy = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    iw = np.array([pos[(int(a), int(b))] for a, b in zip(wx, wy)], dtype=np.int64)
    ia, ca = index_of(wx - vx, wy - vy)
    ib, cb = index_of(vx, vy)
    seeds = [pos[(1, 0)], pos[(0, 1)]]
    e = np.array(e0, dtype=np.complex128)
    for _ in range(iters):
        ea = np.where(ca, np.conj(e[ia]), e[ia])
        eb = np.where(cb, np.conj(e[ib]), e[ib])
        ec = e[iw]
        g = np.zeros(len(Wset), dtype=np.complex128)
        np.add.at(g, iw, ea * eb * np.conj(B))
        t = np.conj(eb) * ec * B
        np.add.at(g, ia, np.where(ca, np.conj(t), t))
        t = np.conj(ea) * ec * B
        np.add.at(g, ib, np.where(cb, np.conj(t), t))
        new = e.copy()
        nz = np.abs(g) > 0
        new[nz] = g[nz] / np.abs(g[nz]) + e[nz]
        new[nz] = new[nz] / np.abs(new[nz])
        new[seeds] = e[seeds]
        e = new
    return e


# ---------------------------------------------------------------------------
# Inverse transform and mosaic (Section 3.2).
# ---------------------------------------------------------------------------
def diffraction_filter(Wset, N):
    """Diffraction-limited OTF of a circular pupil at rho = |w| / (N/2).

    T(rho) = (2/pi) (acos rho - rho sqrt(1 - rho^2)), 0 for rho >= 1.
    """
    rho = np.hypot(Wset[:, 0], Wset[:, 1]) / (N / 2)
    rho = np.minimum(rho, 1.0)
    return (2.0 / np.pi) * (np.arccos(rho) - rho * np.sqrt(1.0 - rho * rho))


def synthesize_patch(amp, phasor, Wset, N, mu, window, filt=None):
    """Reconstructed subimage from modulus and phase on W.

    O(w) = filt(w) |O(w)| e(w) on W, O(-w) = conj(O(w)), zero elsewhere;
    r = Re IFFT2(O) + mu * window (the mean level removed before the
    transform is put back under the same taper).
    """
    spec = np.zeros((N, N), dtype=np.complex128)
    val = amp * phasor
    if filt is not None:
        val = val * filt
    wx, wy = Wset[:, 0], Wset[:, 1]
    spec[wy % N, wx % N] = val
    spec[(-wy) % N, (-wx) % N] = np.conj(val)
    return np.real(np.fft.ifft2(spec)) + mu * window2d(N, window)


def mosaic(patches, ys, xs, H, W, window):
    """Merge overlapping subimages: sum r_k / sum w_k (0 where sum w < 1e-3).

    ``patches`` is [len(ys)][len(xs)][N][N], each r_k being the subimage
    times the taper, so the normalised overlap-add restores the image.
    """
    N = patches.shape[-1]
    w = window2d(N, window)
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    for i, y in enumerate(ys):
        for j, x in enumerate(xs):
            num[y:y + N, x:x + N] += patches[i, j]
            den[y:y + N, x:x + N] += w
    out = np.zeros((H, W))
    ok = den >= 1e-3
    out[ok] = num[ok] / den[ok]
    return out


def reconstruct(frames, params, stf, patch_list=None, keep=False):
    """Full path: tile, accumulate, modulus, phase, synthesis, mosaic.

    ``patch_list`` restricts the work to the given (row, col) tiles (the
    mosaic is then not formed).  Returns a dict with per-stage results.
    """
    F, H, W = frames.shape
    N = params.patch
    ys, xs = tiling(H, W, N, params.stride)
    Wset, S, woff = bispectrum_set(params.u_cut, params.v_radius)
    filt = diffraction_filter(Wset, N) if params.filter else None
    tiles = patch_list if patch_list is not None else [
        (i, j) for i in range(len(ys)) for j in range(len(xs))]
    res = {}
    for (i, j) in tiles:
        cube = frames[:, ys[i]:ys[i] + N, xs[j]:xs[j] + N]
        acc = accumulate_patch(cube, params, S)
        nb = noise_bias(acc["P"]) if params.noise_bias == 1 else 0.0
        amp = amplitude(acc["P"], stf, Wset, nb, params.stf_floor)
        ph = phase_recursion(acc["B"], acc["M10"], acc["M01"], Wset, S, woff, N)
        if params.phase_method == 1:
            ph = phase_least_squares(acc["B"], ph, Wset, S, woff, params.lsq_iters)
        r = synthesize_patch(amp, ph, Wset, N, acc["mu"], params.window, filt)
        res[(i, j)] = dict(acc, amp=amp, phasor=ph, patch=r, nbias=nb)
    out = dict(tiles=res, ys=ys, xs=xs, Wset=Wset, S=S, woff=woff)
    if patch_list is None:
        pat = np.stack([np.stack([res[(i, j)]["patch"] for j in range(len(xs))])
                        for i in range(len(ys))])
        out["image"] = mosaic(pat, ys, xs, H, W, params.window)
    if not keep:
        for v in res.values():
            v.pop("B", None)
    return out
