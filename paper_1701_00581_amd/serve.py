"""Serving loop: bursts from several detector channels arrive frame by frame
and are reconstructed as they complete (continuous batching).

Each channel has a compute stream and a copy stream (both of default
priority; frames move host to device on the copy stream while the channel's
earlier work computes), two device staging buffers of one group of frames
each and a workspace (group scratch and final buffers).  Per-burst
device memory comes from a pool of slots sized to an HBM budget; a burst is admitted when its first frame
arrives and a slot of its channel's shape is free, otherwise its frames
wait on the host until one frees (admission by HBM footprint).  Work of
different channels overlaps on the device through their streams.

Two policies.  Every result depends only on its own frames and on where
its running sums were folded, never on the other bursts: with fixed groups
(max_group == group) a burst gives the same image, bit for bit, alone or in
any mix; adaptive groups change only the fold points, within the parity
tolerances.

* ``stream`` -- the burst's running sums live in its slot
  (``nvsm_stream_*``): arriving frames are copied to the device at once (into
  the channel's staging buffer being filled; the other holds the group in
  flight) and are ingested and added in groups, so only the last group, the
  phase solve and the synthesis remain after the last frame.  A group is launched once ``group`` frames wait and the GPU
  has finished everything launched so far (every channel's last launch),
  once ``max_group`` frames wait, or with the burst's last frame: an idle
  GPU gets small groups (low latency), a busy one larger groups (fewer
  passes over the running sums; a burst whose frames have all arrived
  while the GPU was busy goes in one group, which reads and writes no
  running sums at all).
* ``plain`` -- frames are kept on the device and the burst is reconstructed
  with one ``nvsm_reconstruct`` after its last frame.

All computation is in the library's HIP kernels; this module moves frames,
orders launches and keeps time.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import _lib


@dataclasses.dataclass
class ChannelSpec:
    name: str
    H: int
    W: int
    params: object            # _lib.Params
    stf: object               # device float64 [N][N]


@dataclasses.dataclass
class Done:
    channel: str
    burst: int
    frames: int
    image: object             # device float32 [H][W] (owned by the caller after poll)
    t_last_frame: float       # host clock when the last frame was submitted
    t_done: float             # host clock when the image was seen ready
    groups: int = 1           # device passes over the burst's running sums
    @property
    def latency_ms(self):
        return (self.t_done - self.t_last_frame) * 1e3


class _Burst:
    def __init__(self, ch, bid):
        self.ch, self.bid = ch, bid
        self.pending = []          # host frames not yet on the device
        self.count = 0             # frames handed to the device
        self.total = 0             # frame count once the last frame arrived
        self.staged = 0            # frames in the channel's filling staging buffer
        self.slot = None
        self.t_last = None
        self.event = None
        self.image = None
        self.groups = 0            # device passes over the running sums


class Server:
    """policy: "stream" or "plain"; budget: bytes of HBM for burst slots;
    max_frames: the largest burst (plain policy keeps every frame)."""

    def __init__(self, channels, policy="stream", group=10, budget=64 << 30, max_frames=150, device=0,
                 max_group=None):
        import torch
        self.torch = torch
        self.policy = policy
        self.group = int(group)
        self.max_group = int(max_group or group)
        self.dev = torch.device("cuda", device)
        self.ctx = _lib.nvsm_create(device)
        self.ch = {}
        need = []
        for c in channels:
            _lib.nvsm_prepare(self.ctx, c.params)
            st = torch.cuda.Stream(device=self.dev)           # default priority
            cp = torch.cuda.Stream(device=self.dev)           # host-to-device copies, default priority
            if policy == "stream":
                slot_b, gws_b = _lib.nvsm_stream_plan(c.params, c.H, c.W, self.max_group)
                gws = torch.empty(gws_b, dtype=torch.uint8, device=self.dev)
                stage = [torch.empty((self.max_group, c.H, c.W), dtype=torch.int16, device=self.dev)
                         for _ in range(2)]
            else:
                info = _lib.nvsm_plan(c.params, c.H, c.W, max_frames)
                slot_b = max_frames * c.H * c.W * 2
                gws = torch.empty(info.ws_reconstruct, dtype=torch.uint8, device=self.dev)
                stage = None
            self.ch[c.name] = dict(spec=c, stream=st, copy=cp, gws=gws, stage=stage, fill=0, read_ev=[None, None],
                                   slot_bytes=slot_b, free=[], active={}, order=collections.deque(), last_ev=None)
            need.append((c.name, slot_b))
        # slots: one per channel first, then round robin while the budget lasts
        used = 0
        k = 0
        while True:
            added = False
            for name, b in need:
                if used + b <= budget or k == 0:
                    self.ch[name]["free"].append(torch.empty(b, dtype=torch.uint8, device=self.dev))
                    used += b
                    added = True
            k += 1
            if not added or k > 64:
                break
        self.slots_bytes = used
        self.done = []
        self.inflight = []

    # -- frames in ------------------------------------------------------
    def submit(self, channel, burst, frame, last=False):
        """Hand over one frame (host uint16 [H][W], ideally pinned) of a
        burst; last=True with the burst's final frame."""
        c = self.ch[channel]
        b = c["active"].get(burst)
        if b is None:
            b = _Burst(channel, burst)
            c["active"][burst] = b
            c["order"].append(b)
        b.pending.append(frame)
        if last:
            b.total = b.count + b.staged + len(b.pending)
            b.t_last = time.perf_counter()
        self._advance(c)

    def _admit(self, c, b):
        if b.slot is None and c["free"] and c["order"] and c["order"][0] is b:
            b.slot = c["free"].pop()
            c["order"].popleft()
        return b.slot is not None

    def _gpu_idle(self):
        """Every channel's last launch has finished on the device."""
        return all(c["last_ev"] is None or c["last_ev"].query() for c in self.ch.values())

    def _copies_done(self, c):
        """The channel's compute stream waits for the copies issued so far."""
        ev = self.torch.cuda.Event()
        ev.record(c["copy"])
        c["stream"].wait_event(ev)

    def _advance(self, c):
        torch = self.torch
        spec = c["spec"]
        for b in list(c["active"].values()):
            if not self._admit(c, b):
                break                                  # bursts are admitted in arrival order
            if self.policy == "stream":
                while True:
                    # arrived frames go to the filling buffer at once, on the
                    # copy stream (which waited for that buffer's last
                    # reader when it became the filling one)
                    stage = c["stage"][c["fill"]]
                    with torch.cuda.stream(c["copy"]):
                        while b.pending and b.staged < self.max_group:
                            stage[b.staged].copy_(torch.from_numpy(b.pending.pop(0).view(np.int16)),
                                                  non_blocking=True)
                            b.staged += 1
                    g = b.staged
                    last = bool(b.total) and not b.pending
                    if not (g and (last or g >= self.max_group or (g >= self.group and self._gpu_idle()))):
                        break
                    self._copies_done(c)
                    b.count += g
                    b.staged = 0
                    final = b.total if last else 0
                    with torch.cuda.stream(c["stream"]):
                        _lib.nvsm_stream_add(self.ctx, spec.params, stage[:g], b.count - g, final, b.slot, c["gws"])
                        rd = torch.cuda.Event()
                        rd.record(c["stream"])
                        c["read_ev"][c["fill"]] = rd
                        b.groups += 1
                        if final:
                            b.image = torch.empty((spec.H, spec.W), dtype=torch.float32, device=self.dev)
                            _lib.nvsm_stream_finish(self.ctx, spec.params, spec.H, spec.W, spec.stf, b.image,
                                                    c["gws"])
                        c["last_ev"] = torch.cuda.Event()
                        c["last_ev"].record(c["stream"])
                    # the other buffer fills next, once its last group was read
                    c["fill"] ^= 1
                    if c["read_ev"][c["fill"]] is not None:
                        c["copy"].wait_event(c["read_ev"][c["fill"]])
                    if final:
                        break
            else:
                frames = b.slot.view(torch.int16)
                with torch.cuda.stream(c["copy"]):
                    for fr in b.pending:
                        frames[b.count * spec.H * spec.W:(b.count + 1) * spec.H * spec.W].copy_(
                            torch.from_numpy(fr.view(np.int16)).reshape(-1), non_blocking=True)
                        b.count += 1
                b.pending.clear()
                if b.total and b.count == b.total:
                    self._copies_done(c)
                    with torch.cuda.stream(c["stream"]):
                        b.image = torch.empty((spec.H, spec.W), dtype=torch.float32, device=self.dev)
                        fv = frames[: b.total * spec.H * spec.W].view(b.total, spec.H, spec.W)
                        _lib.nvsm_reconstruct(self.ctx, spec.params, fv, spec.stf, b.image, c["gws"])
                        c["last_ev"] = torch.cuda.Event()
                        c["last_ev"].record(c["stream"])
            with torch.cuda.stream(c["stream"]):
                if b.total and b.count == b.total and b.event is None:
                    b.event = torch.cuda.Event()
                    b.event.record(c["stream"])
                    self.inflight.append(b)
                    del c["active"][b.bid]

    # -- results out ----------------------------------------------------
    def poll(self):
        """Completed bursts since the last call (their slots are freed)."""
        out = []
        keep = []
        now = time.perf_counter()
        for b in self.inflight:
            if b.event.query():
                c = self.ch[b.ch]
                c["free"].append(b.slot)
                b.slot = None
                out.append(Done(b.ch, b.bid, b.total, b.image, b.t_last, now, max(1, b.groups)))
            else:
                keep.append(b)
        self.inflight = keep
        for c in self.ch.values():
            if c["active"]:
                self._advance(c)
        return out

    def drain(self):
        out = []
        while self.inflight or any(c["active"] for c in self.ch.values()):
            out += self.poll()
            time.sleep(0.0002)
        return out

    def close(self):
        self.torch.cuda.synchronize()
        if self.ctx:
            _lib.nvsm_destroy(self.ctx)
            self.ctx = None


def schedule(channels, seconds, fps=10.0, fmin=70, fmax=130, gap_s=2.0, seed=0):
    """Frame arrivals.  Per channel (a detector records one burst at a time)
    bursts arrive as a Poisson stream: the idle time before each burst,
    the first included, is exponential with mean gap_s (0: back to back);
    F is uniform in [fmin, fmax] and the frames come every 1/fps s.  The
    channels are independent, so their bursts cluster at random.  Returns
    sorted (t, channel, burst, frame index, F) tuples."""
    rng = np.random.default_rng(seed)
    ev = []
    for ci, name in enumerate(channels):
        t = float(rng.exponential(gap_s)) if gap_s > 0 else 0.0
        k = 0
        while t < seconds:
            F = int(rng.integers(fmin, fmax + 1))
            for f in range(F):
                ev.append((t, ci, name, k, f, F))
                t += 1.0 / fps
            if gap_s > 0:
                t += float(rng.exponential(gap_s))
            k += 1
    ev.sort()
    return [(t, name, k, f, F) for t, _, name, k, f, F in ev]


def run(server, events, frames_of, compress=1.0, pace=True):
    """Feeds the schedule to the server (time divided by compress; pace=False
    hands frames over as fast as possible) and returns the Done records.
    frames_of(channel, burst, f) gives the host frame."""
    t0 = time.perf_counter()
    done = []
    for t, name, k, f, F in events:
        if pace:
            target = t0 + t / compress
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                done += server.poll()
                time.sleep(min(0.0005, target - now))
        server.submit(name, k, frames_of(name, k, f), last=(f == F - 1))
        done += server.poll()
    done += server.drain()
    return done, time.perf_counter() - t0
