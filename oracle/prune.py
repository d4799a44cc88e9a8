"""Residual pruning after the solve (paper Sec. 4.4.1, last paragraph).

Test infrastructure: the plain FP64 reference of the GPU path's pruning loop.

After each solve the largest residual over the active sparse correspondences is
found; if it exceeds the threshold, every correspondence between the two frames
of that correspondence is removed, a frame that had correspondences and has none
left is marked invalid (removed from the problem: its dense pairs go, its pose
stays), and the problem is solved again, warm-started from the current poses.
The residual of a correspondence is the length (metres) of T_i p - T_j q; ties
go to the smallest correspondence index.  The dense pair set is the one of the
first round.
"""
import numpy as np

from .gn import Setup, solve


def residual_norms(poses, ci, cj, p, q):
    """|T_i p - T_j q| for every correspondence (FP64)."""
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    a = np.einsum("nab,nb->na", poses[ci, :3, :3], p) + poses[ci, :3, 3]
    b = np.einsum("nab,nb->na", poses[cj, :3, :3], q) + poses[cj, :3, 3]
    return np.linalg.norm(a - b, axis=1)


def solve_pruned(depth, intensity, intr, ci, cj, p, q, init_poses, params, r_prune=0.05, max_rounds=100,
                 linear="pcg", pairs=None):
    ci = np.asarray(ci, np.int64)
    cj = np.asarray(cj, np.int64)
    F = depth.shape[0]
    M = len(ci)
    active = np.ones(M, bool)
    had = np.bincount(np.concatenate([ci, cj]), minlength=F) > 0
    if pairs is None:
        pairs = Setup(depth, intensity, intr, ci[:0], cj[:0], np.zeros((0, 3)), np.zeros((0, 3)), init_poses,
                      params).pairs
    pairs = np.asarray(pairs, np.int64).reshape(-1, 2)
    poses = np.array(init_poses, np.float64, copy=True)
    removed = []
    rmax = -1.0
    valid = np.ones(F, bool)
    while True:
        cnt = np.bincount(np.concatenate([ci[active], cj[active]]), minlength=F)
        valid = ~(had & (cnt == 0))
        keep = valid[pairs[:, 0]] & valid[pairs[:, 1]]
        res = solve(depth, intensity, intr, ci[active], cj[active], np.asarray(p)[active], np.asarray(q)[active],
                    poses, params, linear=linear, pairs=pairs[keep])
        poses = res["poses"]
        if not active.any():
            rmax = -1.0
            break
        r = residual_norms(poses, ci, cj, p, q)
        r[~active] = -1.0
        k = int(np.argmax(r))
        rmax = float(r[k])
        if rmax <= r_prune or len(removed) >= max_rounds:
            break
        a, b = ci[k], cj[k]
        active &= ~(((ci == a) & (cj == b)) | ((ci == b) & (cj == a)))
        removed.append((int(min(a, b)), int(max(a, b))))
    return {"poses": poses, "energy": res["energy"], "active": active, "valid": valid, "removed": removed,
            "rmax": rmax}
