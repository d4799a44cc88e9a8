"""The oracle's FP64 dense association of every pair job of a large problem, in the
layout of the kernels' fixed association (bf_params.fixed_association: per job and
source pixel, word 0 = target pixel << 2 | photometric << 1 | geometric, word 1 =
first pixel of the bilinear footprint).

Computed in spawned worker processes (the calling test process holds a GPU
context and must not fork), each returning the encoded words of a range of jobs,
which the caller copies into one device tensor.  Test infrastructure only."""
import os

import numpy as np

_W = {}


def _init(depth, intensity, intr, params, pairs, poses):
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    _W.update(depth=depth, intensity=intensity, intr=intr, params=params, pairs=pairs, poses=poses, frames={})


def _frame(f):
    from oracle.frames import prepare_frame
    fr = _W["frames"]
    if f not in fr:
        fr[f] = prepare_frame(_W["depth"][f], _W["intensity"][f], _W["intr"], _W["params"])
    return fr[f]


def _run(rng):
    from oracle.pairs import relative_pose64
    from oracle.terms import associate
    lo, hi = rng
    W, HW = _W["intr"][4], _W["intr"][4] * _W["intr"][5]
    poses = _W["poses"]
    out = np.zeros((hi - lo, HW, 2), np.int32)
    for k in range(lo, hi):
        i, j = (int(v) for v in _W["pairs"][k])
        R, t = relative_pose64(poses[i], poses[j])
        a = associate(_frame(i), _frame(j), R, t, _W["intr"], _W["params"])
        geo, ph = a["geo"], a["photo"]
        out[k - lo, :, 0] = np.where(geo, ((a["yh"] * W + a["xh"]) << 2) | 1 | np.where(ph, 2, 0), 0)
        out[k - lo, :, 1] = np.where(ph, a["y0"] * W + a["x0"], 0)
    return lo, hi, out


def oracle_association(prob, pairs, poses, params, workers=None, device="cuda"):
    """[jobs, H*W, 2] int32 tensor on `device`."""
    import multiprocessing as mp

    import torch
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    n = len(pairs)
    out = torch.empty((n, prob.width * prob.height, 2), dtype=torch.int32, device=device)
    step = max(1, min(512, (n + 8 * workers - 1) // (8 * workers)))
    ranges = [(lo, min(n, lo + step)) for lo in range(0, n, step)]
    done = 0
    with mp.get_context("spawn").Pool(workers, initializer=_init,
                                      initargs=(prob.depth, prob.intensity, tuple(prob.intrinsics), params,
                                                np.asarray(pairs), poses)) as pool:
        for lo, hi, words in pool.imap_unordered(_run, ranges):
            out[lo:hi] = torch.from_numpy(words).to(device)
            done += hi - lo
    assert done == n
    return out
