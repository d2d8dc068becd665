"""Shared helpers of the GPU parity tests: inputs, metrics, tolerances."""
import functools
import sys

import numpy as np

import oracle
import synth

# Tolerances.  Bispectrum: 1e-4 relative, both normwise per patch and
# against A(w,v) = <|I(w-v)||I(v)||I(w)|> per sample (a near-cancelling mean
# makes the plain elementwise ratio ill-conditioned).  Phase: 1e-3 rad RMS of
# the wrapped difference.  Power spectrum: 1e-5 normwise (FP32 FFT +
# compensated sums are ~1e-6).  Mosaic: 1e-3 of the interior RMS contrast.
BISPEC_TOL = 1e-4
PHASE_RMS_TOL = 1e-3
POWER_TOL = 1e-5
MOSAIC_TOL = 1e-3
# Mean spectrum at the two seed frequencies, relative: it only sets the
# seeds' phases, which a relative error d moves by at most d rad, so it is
# held 10x under the phase tolerance.
MEAN_SPEC_TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=4)
def burst(name, F=None, H=None, W=None):
    cfg = synth.CONFIGS[name]
    fr = synth.make_burst(cfg, frames=F)
    if H is not None or W is not None:
        fr = np.ascontiguousarray(fr[:, :H, :W])
    return fr


@functools.lru_cache(maxsize=4)
def stf(name, screens=200):
    return synth.stf_table(synth.CONFIGS[name], screens=screens)


def to_device(fr):
    import torch
    if fr.dtype == np.uint16:
        return torch.from_numpy(fr.view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(fr)).cuda()


def oparams(p):
    return oracle.Params(patch=p.patch, stride=p.stride, u_cut=p.u_cut, v_radius=p.v_radius,
                         window=p.window, noise_bias=p.noise_bias, filter=p.filter, stf_floor=p.stf_floor,
                         phase_method=p.phase_method, lsq_iters=p.lsq_iters, photons_per_adu=p.photons_per_adu)


def cube(frames, p, k):
    F, H, W = frames.shape
    ys, xs = oracle.tiling(H, W, p.patch, p.stride)
    i, j = divmod(k, len(xs))
    return frames[:, ys[i]:ys[i] + p.patch, xs[j]:xs[j] + p.patch].astype(np.float64)


def abs_bispectrum(I, S):
    """A(w,v) = <|I(w-v)| |I(v)| |I(w)|>, the scale of each sample."""
    return oracle.bispectrum(np.abs(I).astype(np.complex128), S).real


def bispec_errors(bg, bo, A):
    d = np.abs(bg - bo)
    return float(np.linalg.norm(d) / np.linalg.norm(bo)), float(np.max(d / np.maximum(A, 1e-300)))


def phase_rms(eg, eo):
    d = np.angle(eg * np.conj(eo))
    return float(np.sqrt(np.mean(d * d))), float(np.max(np.abs(d)))


def as_complex(t):
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _align(n):
    return (n + 255) // 256 * 256


def reconstruct_views(ws, P, N, nW, S):
    """The intermediates nvsm_reconstruct and nvsm_reconstruct_batch leave at
    the start of their workspace (the layout the header documents): power,
    mean spectrum, mean level, bispectrum, modulus, phasors, subimages of the
    P patches of the last launch group, each 256-byte aligned."""
    import torch
    out, off = {}, 0
    for name, n, dt, shape in (("power", P * N * N * 4, torch.float32, (P, N, N)),
                               ("mean_spec", P * 16, torch.float32, (P, 2, 2)),
                               ("mu", P * 4, torch.float32, (P,)),
                               ("bispec", P * S * 8, torch.float32, (P, S, 2)),
                               ("amp", P * nW * 8, torch.float64, (P, nW)),
                               ("phasor", P * nW * 16, torch.float64, (P, nW, 2)),
                               ("patches", P * N * N * 4, torch.float32, (P, N, N))):
        out[name] = ws[off:off + n].view(dt).view(shape)
        off += _align(n)
    return out
