#!/usr/bin/env python3
"""Throughput of the speckle-masking reconstruction on one MI355X.

One step = one whole burst through the library: ingest (tile cut, taper,
FFT, power/mean sums), bispectrum accumulation, FP64 modulus and phase
solve, inverse transforms and mosaic -- nvsm_reconstruct, frames already in
HBM, image written to HBM.  Default workload: one 2560x2160 burst of 100
12-bit frames, 128x128 patches at 50 % overlap (39x33 patches), |v| <= 12.

Prints one JSON line (rank 0).  Stage times come from HIP events the
library records on the launch stream during the timed steps.  The CPU
baseline is the FP64 oracle on a sample of patches, in a process pool over
the host cores, extrapolated to the whole burst.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reconstructed bursts/s (2560×2160×100 frames); bispectrum GB/s; p99 latency"
FLOP_PER_TERM = 14          # I(w-v) I(v): 6, times conj I(w): 6, accumulate: 2
BYTES_PER_TERM = 8          # one complex64 bispectrum term per frame
# Peaks.  The bispectrum kernel is bound by FP32 vector FMA issue; packed
# FP32 instructions are disabled in this build, so its ceiling is
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s (the
# published 157.3 TFLOP/s counts packed FP32).
PEAK_FP32_UNPACKED = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_FP32_PACKED = 157.3
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "burst2560": dict(v_radius=12, patch=128, noise_bias=1, filter=1),
    "burst1024": dict(v_radius=10, patch=128, noise_bias=1, filter=1),
    "single64": dict(v_radius=8, patch=64, window=0, noise_bias=1, filter=1),
    "batch16": None,
    "serve3": None,
    "model_stf": None,
    "seeing2560": None,
}

TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_bispec_burst2560_traffic.md")

_FR = None
_STF = None
_OP = None


def measured_traffic(workload):
    """HBM bytes per k_bispec launch from the committed counter summary, or
    None when it does not cover this workload or the kernel sources have
    changed since the counters were taken."""
    import hashlib
    if workload != "burst2560" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for f in kv["source_files"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != kv["source_sha256_16"]:
            return None
        return float(kv["k_bispec_traffic_bytes"])
    except (KeyError, OSError, ValueError):
        return None


def _oracle_worker(tiles):
    import oracle
    t = time.perf_counter()
    oracle.reconstruct(_FR, _OP, _STF, patch_list=tiles)
    return time.perf_counter() - t


def cpu_baseline(frames, stf, op, n_patches_total, ny, nx, workers):
    """FP64 oracle on a stratified sample of tiles, one pool worker per core."""
    global _FR, _STF, _OP
    _FR, _STF, _OP = frames, stf, op
    per = 2
    n = workers * per
    idx = np.linspace(0, n_patches_total - 1, n).round().astype(int)
    tiles = [(int(k // nx), int(k % nx)) for k in idx]
    chunks = [tiles[i::workers] for i in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        cpu_s = pool.map(_oracle_worker, chunks)
    wall = time.perf_counter() - t0
    per_burst_s = wall * n_patches_total / n
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=1.0 / per_burst_s, unit="bursts/s", cores=workers, kind="oracle",
                host_cores=os.cpu_count(), cpu_model=cpu_model,
                sample=f"{n} of {n_patches_total} patches (stratified, full frame count), FP64 NumPy oracle, "
                       f"{workers} worker processes, {wall:.1f} s wall / {sum(cpu_s):.1f} s CPU, "
                       f"extrapolated x{n_patches_total / n:.1f} to the whole burst (mosaic excluded)",
                wall_s=wall)


def batch16(args):
    """16 bursts of uneven shape: 8 x 2560x2160 and 8 x 1024x1024, uint16,
    frame counts uniform in [80, 150], 128^2 patches.  The v radius of each
    class is tuned on its first burst (nvsm_tune_radius: the smallest R in
    6..12 resp. 6..10 whose phases agree with the largest R's within
    --tune-tol rad).  Three ways, same images at that schedule: one
    nvsm_reconstruct per burst (plain launches); nvsm_reconstruct_batch per
    class (eager); the two batch calls captured once in a HIP graph and
    replayed."""
    import dataclasses
    import synth
    import torch
    import paper_1701_00581_amd as nv
    rng = np.random.default_rng(170100581)
    Fs = rng.integers(80, 151, size=16)
    classes = []
    t = time.perf_counter()
    for c, (base, R, n0) in enumerate((("burst2560", 12, 0), ("burst1024", 10, 8))):
        cfg0 = synth.CONFIGS[base]
        stf = torch.from_numpy(synth.stf_table(cfg0, screens=args.stf_screens)).cuda()
        p = nv.default_params(128, v_radius=R, noise_bias=1, filter=1)
        items = []
        for i in range(8):
            cfg = dataclasses.replace(cfg0, name=f"{base}-{i}", index=100 + n0 + i, F=int(Fs[n0 + i]))
            fr = synth.make_burst(cfg)
            d = torch.from_numpy(fr.view(np.int16)).cuda()
            items.append((d, stf, torch.empty((cfg.H, cfg.W), device="cuda")))
            del fr
        classes.append((p, items))
    print(f"[bench] generated 16 bursts (F = {list(map(int, Fs))}) in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    ctx = nv.nvsm_create(0)
    # the v-radius schedule: one R per class, tuned on the class's first burst
    schedule = []
    for p, items in classes:
        d, stf, _ = items[0]
        F, H, W = d.shape
        r_max = p.v_radius
        wt = torch.empty(nv.nvsm_tune_radius_plan(p, H, W, F, r_max), dtype=torch.uint8, device="cuda")
        r, meas = nv.nvsm_tune_radius(ctx, p, d, stf, 6, r_max, args.tune_tol, wt)
        del wt
        schedule.append({"r_max": r_max, "v_radius": r, "phase_rms_vs_r_max": {k: round(v, 4) for k, v in meas.items()}})
        p.v_radius = r
    print(f"[bench] v-radius schedule (tol {args.tune_tol} rad): {schedule}", file=sys.stderr, flush=True)
    terms = 0
    cap = int(args.batch_ws_gib * (1 << 30))
    ws_need = 0
    for p, items in classes:
        nv.nvsm_prepare(ctx, p)
        info = nv.nvsm_plan(p, 128, 128, 1)
        for d, _, _ in items:
            F, H, W = d.shape
            terms += nv.nvsm_plan(p, H, W, F).patches * info.s_count * F
        lo, hi = nv.nvsm_batch_plan(p, [tuple(d.shape) for d, _, _ in items])
        ws_need = max(ws_need, lo)
    ws = torch.empty(max(ws_need, min(cap, ws_need * 16)), dtype=torch.uint8, device="cuda")
    # tuned launch choices (identical outputs), one burst per class
    tuned = []
    for p, items in classes:
        d = items[0][0]
        info = nv.nvsm_plan(p, d.shape[1], d.shape[2], d.shape[0])
        wt = ws if ws.numel() >= info.ws_reconstruct else torch.empty(info.ws_reconstruct, dtype=torch.uint8,
                                                                          device="cuda")
        tuned.append(nv.nvsm_autotune(ctx, p, d, wt))
        del wt
    wsr = {}

    def plain():
        for p, items in classes:
            for d, stf, out in items:
                F, H, W = d.shape
                need = nv.nvsm_plan(p, H, W, F).ws_reconstruct
                nv.nvsm_reconstruct(ctx, p, d, stf, out, ws if ws.numel() >= need else wsr.setdefault(
                    need, torch.empty(need, dtype=torch.uint8, device="cuda")))

    def batched():
        for p, items in classes:
            nv.nvsm_reconstruct_batch(ctx, p, items, ws)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    plain()
    ref = [o.clone() for _, items in classes for _, _, o in items]
    t_plain = timed(plain, args.steps)
    batched()
    same_b = all(torch.equal(o, r) for o, r in zip([o for _, items in classes for _, _, o in items], ref))
    t_batch = timed(batched, args.steps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batched()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batched()
    t_graph = timed(g.replay, args.steps)
    same_g = all(torch.equal(o, r) for o, r in zip([o for _, items in classes for _, _, o in items], ref))
    stage = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        nv.nvsm_profile_read(ctx)
        nv.nvsm_profile_enable(ctx, True)
        fn()
        torch.cuda.synchronize()
        nv.nvsm_profile_enable(ctx, False)
        stage[name] = {k: round(v[0], 3) for k, v in nv.nvsm_profile_read(ctx).items()}
    out = {
        "metric": "bursts/s of a 16-burst uneven batch (8 x 2560x2160 + 8 x 1024x1024, F in [80,150])",
        "value": 16 / t_graph, "unit": "bursts/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_graph * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch16: 8 x 2560x2160 (|v|<={classes[0][0].v_radius}) + 8 x 1024x1024 "
                               f"(|v|<={classes[1][0].v_radius}) uint16 bursts, F = {list(map(int, Fs))}, 128x128 "
                               f"patches, v radii tuned at {args.tune_tol} rad, one HIP graph of two batch calls",
                   "v_radius_schedule": schedule,
                   "terms": int(terms), "workspace_GiB": ws.numel() / (1 << 30),
                   "tuned_launch": [{"slots": k, "form": f} for k, f in tuned], "parallelism": "single GPU"},
        "per_burst_plain": {"bursts_per_s": 16 / t_plain, "ms": t_plain * 1e3},
        "batched_eager": {"bursts_per_s": 16 / t_batch, "ms": t_batch * 1e3, "identical": bool(same_b)},
        "batched_graph": {"bursts_per_s": 16 / t_graph, "ms": t_graph * 1e3, "identical": bool(same_g)},
        "terms_per_s": terms / t_graph,
        "stage_ms_per_batch": stage,
    }
    print(json.dumps(out), flush=True)
    del g
    nv.nvsm_destroy(ctx)


def serve3(args):
    """Three channels (2 x 2560x2160 |v|<=12, 1 x 1024x1024 |v|<=10) deliver
    bursts of F uniform in [70, 130] frames at 10 frames/s each, the idle
    time before each burst exponential with mean --gap-s (a Poisson stream
    of bursts per detector), on a simulated clock divided by --compress.  The same schedule is served by
    the streaming policy (running sums on the device, adaptive groups) and
    by the plain policy (one reconstruction after each burst's last frame);
    latency runs from a burst's last frame to its image being ready."""
    import synth
    import torch
    import paper_1701_00581_amd as nv
    from paper_1701_00581_amd import serve
    specs, pool = [], {}
    t = time.perf_counter()
    for name, base, R in (("ch0", "burst2560", 12), ("ch1", "burst2560", 12), ("ch2", "burst1024", 10)):
        cfg = synth.CONFIGS[base]
        cfg = type(cfg)(**{**cfg.__dict__, "index": cfg.index + 200 + len(specs)})
        stf = torch.from_numpy(synth.stf_table(cfg, screens=args.stf_screens)).cuda()
        specs.append(serve.ChannelSpec(name, cfg.H, cfg.W, nv.default_params(128, v_radius=R, noise_bias=1, filter=1),
                                       stf))
        fr = synth.make_burst(cfg, frames=130)
        pinned = torch.from_numpy(fr.view(np.int16)).pin_memory()     # a new pinned tensor
        pool[name] = pinned.numpy().view(np.uint16)
    print(f"[bench] generated frame pools in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    events = serve.schedule([s.name for s in specs], seconds=args.sim_seconds, fps=10.0, fmin=70, fmax=130,
                            gap_s=args.gap_s, seed=1)
    frames_of = lambda c, k, f: pool[c][f]  # noqa: E731
    results = {}
    for policy, kw in (("plain", {}), ("stream", dict(group=args.group, max_group=args.max_group))):
        srv = serve.Server(specs, policy=policy, budget=int(args.serve_budget_gib * (1 << 30)), max_frames=130, **kw)
        done, wall = serve.run(srv, events, frames_of, compress=args.compress)
        lat = np.array([d.latency_ms for d in done])
        results[policy] = {
            "bursts": len(done), "wall_s": wall, "bursts_per_s": len(done) / wall,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "groups_per_burst": float(np.mean([d.groups for d in done])),
            "slots_GiB": srv.slots_bytes / (1 << 30),
        }
        print(f"[bench] {policy}: {results[policy]}", file=sys.stderr, flush=True)
        srv.close()
        del srv
        torch.cuda.empty_cache()
    # as fast as frames can be handed over (no pacing): throughput bound
    sat = {}
    ev2 = [e for e in events if e[2] < args.sat_bursts]
    for policy, kw in (("plain", {}), ("stream", dict(group=args.group, max_group=args.max_group))):
        srv = serve.Server(specs, policy=policy, budget=int(args.serve_budget_gib * (1 << 30)), max_frames=130, **kw)
        done, wall = serve.run(srv, ev2, frames_of, pace=False)
        sat[policy] = {"bursts": len(done), "wall_s": wall, "bursts_per_s": len(done) / wall,
                       "groups_per_burst": float(np.mean([d.groups for d in done]))}
        print(f"[bench] saturated {policy}: {sat[policy]}", file=sys.stderr, flush=True)
        srv.close()
        del srv
        torch.cuda.empty_cache()
    st, pl = results["stream"], results["plain"]
    out = {
        "metric": "served bursts/s and p99 burst latency, 3 channels (2 x 2560x2160 + 1 x 1024x1024) at 10 fps",
        "value": st["bursts_per_s"], "unit": "bursts/s", "n_gpus": 1, "steps": st["bursts"], "warmup": 0,
        "ms_per_step": st["wall_s"] * 1e3 / max(1, st["bursts"]), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve3: {args.sim_seconds:.0f} s of arrivals at 10 fps per channel, F in [70,130], "
                               f"Poisson bursts (exponential idle time, mean {args.gap_s:g} s), "
                               f"clock / {args.compress:g}, streaming groups {args.group}..{args.max_group}",
                   "parallelism": "single GPU"},
        "paced": results, "saturated": sat,
        "p99_ratio_plain_over_stream": pl["latency_ms"]["p99"] / st["latency_ms"]["p99"],
    }
    print(json.dumps(out), flush=True)


def model_stf(args):
    """Model STF tables: 128 x 128 patch grid, D/r0 = 20, --model-screens
    Kolmogorov screens per table (Monte Carlo; a reading of the model STF the
    paper chooses by r0)."""
    import oracle
    N, x, K = 128, 20.0, args.model_screens
    cpu = None
    if not args.no_cpu_baseline:
        ks = 20
        t = time.perf_counter()
        oracle.model(N, x, ks, 99)
        dt = time.perf_counter() - t
        cpu = {"value": ks / K / dt, "unit": "tables/s", "cores": 1, "kind": "oracle",
               "sample": f"{ks} of {K} screens of one table (FP64 NumPy oracle, one process), scaled to {K}"}
    import torch
    import paper_1701_00581_amd as nv
    p = nv.default_params(N)
    ctx = nv.nvsm_create(0)
    ws = torch.empty(nv.nvsm_model_stf_plan(p, K), dtype=torch.uint8, device="cuda")
    stf = torch.empty((N, N), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        nv.nvsm_model_stf(ctx, p, x, K, 1, stf, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(args.steps):
        nv.nvsm_model_stf(ctx, p, x, K, 1 + k, stf, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nv.nvsm_destroy(ctx)
    # per screen: half of the pair's transform (one per pair of screens) and
    # the transforms of the field and the PSF, 5 N^2 log2(N^2) flop each
    flop = K * 2.5 * 5 * N * N * math.log2(N * N)
    out = {
        "metric": f"model STF tables/s ({N}x{N} patch grid, D/r0 {x:g}, {K} screens)",
        "value": 1e3 / ms, "unit": "tables/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": f"model_stf: N {N}, D/r0 {x:g}, {K} screens per table"},
        "screens_per_s": K * 1e3 / ms,
        "fft_tflops": flop / (ms * 1e-3) / 1e12,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def seeing2560(args):
    """Seeing estimate by the spectral ratio of the 2560x2160x100 burst (320
    cubes of 128^2) with the default settings: 40 model points of 1000
    screens, 12 annuli; then its model STF."""
    import oracle
    import synth
    cfg = synth.CONFIGS["burst2560"]
    frames = synth.make_burst(cfg)
    F, H, W = frames.shape
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's two parts on a sample: one model point of 20 screens,
        # and the ratio of 2 cubes, scaled to 41 model points of 1000 screens
        # and 320 cubes (the per-cube fit is left out of the sample)
        t = time.perf_counter()
        oracle.model(128, 20.0, 20, 1, 0)
        t_model = (time.perf_counter() - t) * (1000 / 20) * 41
        t = time.perf_counter()
        for (y0, x0) in oracle.seeing_cubes(H, W, 128)[:2]:
            oracle.spectral_ratio(frames[:, y0:y0 + 128, x0:x0 + 128].astype(np.float64), 1)
        t_ratio = (time.perf_counter() - t) * 320 / 2
        cpu = {"value": 1.0 / (t_model + t_ratio), "unit": "estimates/s", "cores": 1, "kind": "oracle",
               "sample": "one model point of 20 screens and the ratio of 2 cubes, scaled to 41 x 1000 screens and "
                         "320 cubes (FP64 NumPy oracle, one process; the fit is not included)"}
    import torch
    import paper_1701_00581_amd as nv
    p = nv.default_params(128)
    sp = nv.seeing_default_params()
    ws_b, cubes = nv.nvsm_seeing_plan(p, sp, H, W, F)
    ctx = nv.nvsm_create(0)
    d = torch.from_numpy(frames.view(np.int16)).cuda()
    x = torch.empty(1 + cubes, dtype=torch.float64, device="cuda")
    stf = torch.empty((128, 128), dtype=torch.float64, device="cuda")
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        nv.nvsm_seeing(ctx, p, sp, d, x, stf, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        nv.nvsm_seeing(ctx, p, sp, d, x, stf, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    est = float(x[0].item())
    nv.nvsm_destroy(ctx)
    out = {
        "metric": "seeing estimates/s (2560x2160x100, 320 cubes of 128^2, 40 model points x 1000 screens)",
        "value": 1e3 / ms, "unit": "estimates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": "seeing2560: the 2560x2160x100 burst, D/r0 20 in the generator"},
        "d_over_r0_estimate": est, "d_over_r0_generator": cfg.d_over_r0, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="burst2560", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=None, help="override the frame count")
    ap.add_argument("--stf-screens", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase-method", type=int, default=0, choices=(0, 1),
                    help="0: the recursion; 1: the recursion followed by least-squares steps")
    ap.add_argument("--lsq-iters", type=int, default=10, help="least-squares steps with --phase-method 1")
    ap.add_argument("--noise-bias", type=int, default=None, choices=(0, 1, 2),
                    help="override the workload's noise term: 0 none, 1 corner level, 2 photon-noise model")
    ap.add_argument("--model-screens", type=int, default=1000, help="model_stf: screens per table")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference for traffic counters)")
    ap.add_argument("--batch-ws-gib", type=float, default=96.0, help="workspace cap of the batch16 workload")
    ap.add_argument("--tune-tol", type=float, default=0.1,
                    help="batch16: phase agreement (rad, RMS weighted by the power above the noise floor) that sets each class's v radius")
    ap.add_argument("--sim-seconds", type=float, default=600.0, help="serve3: simulated seconds of arrivals")
    ap.add_argument("--compress", type=float, default=20.0, help="serve3: simulated clock / wall clock")
    ap.add_argument("--group", type=int, default=10, help="serve3: frames per streaming group when the GPU is idle")
    ap.add_argument("--max-group", type=int, default=130, help="serve3: largest streaming group")
    ap.add_argument("--gap-s", type=float, default=2.0,
                    help="serve3: mean idle time before each burst of a channel (exponential; 0: back to back)")
    ap.add_argument("--serve-budget-gib", type=float, default=160.0, help="serve3: HBM for burst slots")
    ap.add_argument("--sat-bursts", type=int, default=8, help="serve3: bursts per channel of the unpaced run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs the path on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    if args.workload == "batch16":
        batch16(args)
        return
    if args.workload == "serve3":
        serve3(args)
        return
    if args.workload == "model_stf":
        model_stf(args)
        return
    if args.workload == "seeing2560":
        seeing2560(args)
        return

    import oracle
    import synth
    cfg = synth.CONFIGS[args.workload]
    t = time.perf_counter()
    frames = synth.make_burst(cfg, frames=args.frames)
    stf = synth.stf_table(cfg, screens=args.stf_screens)
    F, H, W = frames.shape
    gen_s = time.perf_counter() - t
    print(f"[bench] generated {args.workload} {F}x{H}x{W} {frames.dtype} in {gen_s:.1f} s", file=sys.stderr,
          flush=True)
    wl = dict(WORKLOADS[args.workload])
    if args.noise_bias is not None:
        wl["noise_bias"] = args.noise_bias
    # photon-noise gain of the synthetic frames: 12-bit units of photons / 2048, or photon counts
    gain = cfg.photons / 2048.0 if frames.dtype == np.uint16 else 1.0

    # CPU baseline first, before the GPU runtime exists in this process
    cpu = None
    ys, xs = oracle.tiling(H, W, wl["patch"], wl["patch"] // 2)
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or max(1, min(16, os.cpu_count() or 1))
        op = oracle.Params(patch=wl["patch"], v_radius=wl["v_radius"], window=wl.get("window", 1),
                           noise_bias=wl["noise_bias"], filter=wl["filter"], phase_method=args.phase_method,
                           lsq_iters=args.lsq_iters, photons_per_adu=gain)
        cpu = cpu_baseline(frames, stf, op, len(ys) * len(xs), len(ys), len(xs), workers)
        print(f"[bench] cpu baseline {cpu['value']:.3e} bursts/s ({cpu['sample']})", file=sys.stderr, flush=True)

    import torch
    import paper_1701_00581_amd as nv
    dev = torch.device("cuda", 0)
    p = nv.default_params(wl["patch"], v_radius=wl["v_radius"], window=wl.get("window", 1),
                          noise_bias=wl["noise_bias"], filter=wl["filter"])
    p.phase_method = args.phase_method
    p.lsq_iters = args.lsq_iters
    p.photons_per_adu = gain
    s = nv.Session(p, H, W, F)
    # host -> device upload of the burst (pinned), reported beside the value
    raw = frames.view(np.int16) if frames.dtype == np.uint16 else frames
    pinned = torch.from_numpy(raw).pin_memory()
    d_frames = torch.empty(pinned.shape, dtype=pinned.dtype, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h2d = []
    for _ in range(3):
        e0.record()
        d_frames.copy_(pinned, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        h2d.append(e0.elapsed_time(e1))
    h2d_ms = float(np.median(h2d))
    d_stf = torch.from_numpy(stf).to(dev)

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        s.reconstruct(d_frames, d_stf)
    torch.cuda.synchronize()
    if not torch.isfinite(s.image).all():
        raise RuntimeError("non-finite output")

    nv.nvsm_profile_read(s.ctx)          # drop anything recorded so far
    nv.nvsm_profile_enable(s.ctx, True)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        s.reconstruct(d_frames, d_stf)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nv.nvsm_profile_enable(s.ctx, False)
    stages = nv.nvsm_profile_read(s.ctx)
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    elapsed = t1 - t0
    value = args.steps / elapsed

    info = s.info
    P, S = info.patches, info.s_count
    terms = P * S * F
    # per step: the library records each launch of a stage (the bispectrum
    # runs its patch ranges back to back on the launch stream; the solve of
    # each range runs on a second stream, overlapping the next range's
    # bispectrum)
    bis_launches = stages["bispectrum"][1] / args.steps
    bis_ms = stages["bispectrum"][0] / max(1, stages["bispectrum"][1])       # per launch
    achieved = terms * FLOP_PER_TERM / bis_launches / (bis_ms * 1e-3) / 1e12
    stage_ms = {k: v[0] / args.steps for k, v in stages.items()}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bursts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {W}x{H} x {F} {'uint16 12-bit' if frames.dtype == np.uint16 else 'float32'} "
                        f"frames, {p.patch}x{p.patch} patches at stride {p.stride} ({info.patches_x}x{info.patches_y}), "
                        f"|v|<={p.v_radius}, u_cut {p.u_cut}, FP32 compensated accumulation, FP64 solve"
                        + (f", {p.lsq_iters} least-squares phase steps" if p.phase_method == 1 else "")
                        + (", photon-noise terms" if p.noise_bias == 2 else ""),
            "frames": F, "height": H, "width": W, "patch": p.patch, "v_radius": p.v_radius,
            "patches": P, "bispectrum_samples_per_patch": S, "parallelism": "single GPU",
        },
        "bispectrum_GBps": terms * BYTES_PER_TERM / (stage_ms["bispectrum"] * 1e-3) / 1e9,
        "bispectrum_terms_per_s": terms / (stage_ms["bispectrum"] * 1e-3),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "stage_ms": stage_ms,
        "h2d": {"ms": h2d_ms, "GBps": frames.nbytes / (h2d_ms * 1e-3) / 1e9,
                "bursts_per_s_with_h2d": 1.0 / (elapsed / args.steps + h2d_ms * 1e-3)},
        "roofline": {
            "bound": "alu",
            "kernel": "k_bispec",
            "achieved": achieved,
            "peak": PEAK_FP32_UNPACKED,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_UNPACKED,
            "traffic": measured_traffic(args.workload),
            "traffic_unit": "bytes per launch (HBM read+write, copy-calibrated FETCH_SIZE/WRITE_SIZE)",
            "frac_vs_packed_fp32_peak": achieved / PEAK_FP32_PACKED,
            "algorithmic_flop_per_launch": terms * FLOP_PER_TERM / bis_launches,
            "avg_launch_ms": bis_ms,
            "launches_per_step": bis_launches,
        },
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                                      "host_cores", "cpu_model")},
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
