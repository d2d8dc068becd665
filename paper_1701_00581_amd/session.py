"""Device-buffer plumbing around the C entry points (no computation)."""
from __future__ import annotations

from . import _lib


class Session:
    """Owns a context and the torch buffers of one burst shape.

    ``accumulate``, ``solve``, ``synthesize`` and ``reconstruct`` call the
    C entry points of the same names on the current torch stream.
    """

    def __init__(self, params, H, W, F, device=0):
        import torch
        self.torch = torch
        self.params = params
        self.H, self.W, self.F = int(H), int(W), int(F)
        self.dev = torch.device("cuda", device)
        self.ctx = _lib.nvsm_create(device)
        self.info = _lib.nvsm_plan(params, H, W, F)
        _lib.nvsm_prepare(self.ctx, params)
        N = params.patch
        P, nW, S = self.info.patches, self.info.w_count, self.info.s_count
        e = lambda *shape, dt=torch.float32: torch.empty(shape, dtype=dt, device=self.dev)  # noqa: E731
        self.power = e(P, N, N)
        self.mean_spec = e(P, 2, 2)
        self.mu = e(P)
        self.bispec = e(P, S, 2)
        self.amp = e(P, nW, dt=torch.float64)
        self.phasor = e(P, nW, 2, dt=torch.float64)
        self.patches = e(P, N, N)
        self.image = e(self.H, self.W)
        self.ws_acc = e(max(1, self.info.ws_accumulate), dt=torch.uint8)
        self._ws_rec = None

    def accumulate(self, frames, with_bispectrum=True):
        _lib.nvsm_accumulate(self.ctx, self.params, frames, self.power, self.mean_spec, self.mu,
                             self.bispec if with_bispectrum else None, self.ws_acc)

    def solve(self, stf, power=None, mean_spec=None, bispec=None):
        _lib.nvsm_solve(self.ctx, self.params, self.info.patches,
                        self.power if power is None else power,
                        self.mean_spec if mean_spec is None else mean_spec,
                        self.bispec if bispec is None else bispec, stf, self.amp, self.phasor)

    def synthesize(self, amp=None, phasor=None, mu=None):
        _lib.nvsm_synthesize(self.ctx, self.params, self.H, self.W,
                             self.amp if amp is None else amp, self.phasor if phasor is None else phasor,
                             self.mu if mu is None else mu, self.patches, self.image)

    def reconstruct(self, frames, stf, out=None):
        if self._ws_rec is None:
            self._ws_rec = self.torch.empty(self.info.ws_reconstruct, dtype=self.torch.uint8, device=self.dev)
        _lib.nvsm_reconstruct(self.ctx, self.params, frames, stf, self.image if out is None else out,
                              self._ws_rec)
        return self.image if out is None else out

    def close(self):
        if self.ctx:
            _lib.nvsm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
