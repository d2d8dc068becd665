"""The FP64 oracle over many patches in a process pool (test infrastructure).

Workers are spawned fresh (they never touch the GPU) and read the frames
from a memory-mapped .npy file, so a full burst is not copied per worker.
Each worker runs ``oracle.reconstruct`` on its share of the tiles; the
parent merges the subimages with ``oracle.mosaic``.
"""
import multiprocessing as mp
import os
import shutil
import tempfile
import time

import numpy as np


def workers():
    """Pool size: the host's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def _work(job):
    import oracle
    path, stf_path, kw, tiles, keep = job
    fr = np.load(path, mmap_mode="r")
    stf = np.load(stf_path)
    op = oracle.Params(**kw)
    r = oracle.reconstruct(fr, op, stf, patch_list=tiles, keep=True)
    out = {}
    for t, v in r["tiles"].items():
        d = {"patch": v["patch"]}
        if t in keep:
            d.update(B=v["B"], phasor=v["phasor"], amp=v["amp"], P=v["P"], mu=v["mu"])
        out[t] = d
    return out


def reconstruct(frames, op, stf, keep=(), n_workers=None, say=print):
    """oracle.reconstruct of every tile, in a pool.  Returns dict(image,
    tiles: {(i, j): {patch[, B, phasor, amp, P, mu] for tiles in keep}},
    ys, xs)."""
    import oracle
    F, H, W = frames.shape
    N = op.patch
    ys, xs = oracle.tiling(H, W, N, op.stride)
    tiles = [(i, j) for i in range(len(ys)) for j in range(len(xs))]
    n = n_workers or workers()
    keep = set(keep)
    tmp = tempfile.mkdtemp(prefix="oracle_pool_")
    try:
        path = os.path.join(tmp, "frames.npy")
        stf_path = os.path.join(tmp, "stf.npy")
        np.save(path, np.ascontiguousarray(frames))
        np.save(stf_path, np.asarray(stf, dtype=np.float64))
        kw = dict(vars(op))
        # small jobs, dealt round-robin, so the pool stays busy to the end
        per = max(1, len(tiles) // (4 * n))
        jobs = [(path, stf_path, kw, tiles[a:a + per], keep & set(tiles[a:a + per]))
                for a in range(0, len(tiles), per)]
        res = {}
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(n) as pool:
            for k, r in enumerate(pool.imap_unordered(_work, jobs)):
                res.update(r)
                if k % max(1, len(jobs) // 8) == 0:
                    say(f"[oracle pool] {len(res)}/{len(tiles)} tiles, {time.perf_counter() - t0:.0f} s")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    pat = np.stack([np.stack([res[(i, j)]["patch"] for j in range(len(xs))]) for i in range(len(ys))])
    return dict(image=oracle.mosaic(pat, ys, xs, H, W, op.window), tiles=res, ys=ys, xs=xs)
