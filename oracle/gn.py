"""Gauss-Newton solve of E_align (paper Sec. 4.3-4.4).

E_align = w_sparse E_sparse + w_d (w_geo E_geo + w_photo E_photo), written as
a sum of squared residuals (no factor 1/2).  Each iteration k linearises the
residuals at the current poses, assembles J^T J and J^T F, removes the fixed
reference frame and unconstrained frames (and holds frames that no residual
touches at these poses), solves for the increment and applies it by
T_f <- T_f Exp(dx_f) (``se3``).  w_d is ramped linearly over the
iterations.  The dense pair set is computed once from the initial poses.  The
returned energy is evaluated at the returned poses with the last iteration's
w_d.  There is no damping (the paper's solver is plain Gauss-Newton).
"""
import time

import numpy as np

from .frames import prepare_frames
from .pairs import dense_pairs, edge_list, group_correspondences
from .params import Params
from .se3 import exp_se3
from .system import (assemble, dense_pair_blocks, free_frames, inert_frames, reduce_system, solve_cholesky,
                     solve_pcg, sparse_pair_blocks)


class Setup:
    """Per-solve structures: prepared frames, pair set, correspondence groups, edges."""

    def __init__(self, depth, intensity, intr, corr_i, corr_j, p, q, init_poses, params, pairs=None):
        self.intr = tuple(intr)
        self.params = params
        self.F = depth.shape[0]
        self.frames = prepare_frames(depth, intensity, self.intr, params) if params.use_dense else None
        if not params.use_dense:
            self.pairs = np.zeros((0, 2), np.int32)
        elif pairs is None:
            self.pairs = dense_pairs(depth, init_poses, self.intr, params)
        else:
            self.pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
        if params.use_sparse and len(corr_i):
            self.skeys, self.sptr, self.sperm, self.pa, self.qb = group_correspondences(
                corr_i, corr_j, np.asarray(p, np.float64), np.asarray(q, np.float64), self.F)
        else:
            self.skeys = np.zeros((0, 2), np.int32)
            self.sptr = np.zeros(1, np.int64)
            self.sperm = np.zeros(0, np.int64)
            self.pa = self.qb = np.zeros((0, 3))
        self.edges, self.edge_dense, self.edge_sparse = edge_list(self.pairs, self.skeys)
        self.free = free_frames(self.F, self.edges)


def edge_blocks(setup, poses, wd, assoc=None):
    """Per-edge dicts with the sparse and dense contributions and their sum.
    `assoc` optionally maps edge index -> a fixed dense association."""
    prm = setup.params
    out = []
    for e, (i, j) in enumerate(setup.edges):
        tot = {"Hii": np.zeros((6, 6)), "Hij": np.zeros((6, 6)), "Hjj": np.zeros((6, 6)),
               "gi": np.zeros(6), "gj": np.zeros(6)}
        rec = {"sparse": None, "dense": None}
        s = setup.edge_sparse[e]
        if s >= 0:
            lo, hi = setup.sptr[s], setup.sptr[s + 1]
            b = sparse_pair_blocks(poses[i], poses[j], setup.pa[lo:hi], setup.qb[lo:hi], prm.w_sparse)
            rec["sparse"] = b
        d = setup.edge_dense[e]
        rec["dense_rev"] = None
        if d >= 0:
            b = dense_pair_blocks(setup.frames[i], setup.frames[j], poses[i], poses[j], setup.intr, prm, wd,
                                  assoc=None if assoc is None else assoc[e])
            rec["dense"] = b
            if prm.bidirectional:
                # the sums over the pixels of frame j as well (j -> i), roles swapped
                r = dense_pair_blocks(setup.frames[j], setup.frames[i], poses[j], poses[i], setup.intr, prm, wd,
                                      assoc=None if assoc is None else assoc.get(("rev", e)))
                rec["dense_rev"] = dict(r, Hii=r["Hjj"], Hjj=r["Hii"], Hij=r["Hij"].T, gi=r["gj"], gj=r["gi"])
        for part in ("sparse", "dense", "dense_rev"):
            if rec[part] is not None:
                for k in tot:
                    tot[k] = tot[k] + rec[part][k]
        rec.update(tot)
        out.append(rec)
    return out


def energies(blocks):
    dense = [b[k] for b in blocks for k in ("dense", "dense_rev") if b.get(k) is not None]
    es = sum(b["sparse"]["E"] for b in blocks if b["sparse"] is not None)
    eg = sum(d["Egeo"] for d in dense)
    ep = sum(d["Ephoto"] for d in dense)
    ng = sum(d["ngeo"] for d in dense)
    npp = sum(d["nphoto"] for d in dense)
    ns = sum(b["sparse"]["n"] for b in blocks if b["sparse"] is not None)
    return {"total": es + eg + ep, "sparse": es, "geo": eg, "photo": ep,
            "n_sparse": ns, "n_geo": ng, "n_photo": npp}


def build_system(setup, poses, wd, assoc=None):
    """Full H, g (FP64, 6F) and per-edge blocks and energies at `poses` with dense weight wd."""
    blocks = edge_blocks(setup, poses, wd, assoc)
    H, g = assemble(setup.F, setup.edges, blocks)
    return H, g, blocks, energies(blocks)


def evaluate(setup, poses, wd, assoc=None):
    blocks = edge_blocks(setup, poses, wd, assoc)
    return energies(blocks)


def solve(depth, intensity, intr, corr_i, corr_j, p, q, init_poses, params=None, linear="cholesky",
          pairs=None, setup=None, record=False, freeze_association=False):
    """Run params.num_gn Gauss-Newton iterations; returns a result dict.

    With `freeze_association` the dense pixel association is decided once at the
    initial poses and kept (a smooth energy, used to check convergence); otherwise
    it is re-decided at every iteration."""
    params = params or Params()
    t0 = time.perf_counter()
    if setup is None:
        setup = Setup(depth, intensity, intr, corr_i, corr_j, p, q, init_poses, params, pairs)
    poses = np.array(init_poses, np.float64, copy=True)
    trace = []
    steps = []
    assoc = None
    for k in range(params.num_gn):
        wd = params.dense_weight(k)
        H, g, blocks, en = build_system(setup, poses, wd, assoc)
        if freeze_association and assoc is None:
            keep = ("geo", "photo", "xh", "yh", "x0", "y0")
            assoc = {e: {k: b["dense"]["terms"][k] for k in keep} for e, b in enumerate(blocks)
                     if b["dense"] is not None}
            assoc.update({("rev", e): {k: b["dense_rev"]["terms"][k] for k in keep} for e, b in enumerate(blocks)
                          if b["dense_rev"] is not None})
        inert = inert_frames(H, setup.free)
        active = setup.free[~inert]
        Hr, gr, _ = reduce_system(H, g, active)
        if linear == "cholesky":
            dxa = solve_cholesky(Hr, gr)
            st = {}
        else:
            dxa, st = solve_pcg(Hr, gr, params.num_pcg, preconditioner=params.preconditioner)
        dx = np.zeros(6 * len(setup.free))
        dx.reshape(-1, 6)[~inert] = dxa.reshape(-1, 6)
        trace.append(en)
        steps.append({"dx": dx, **st, **({"H": Hr, "g": gr} if record else {})})
        for n, f in enumerate(setup.free):
            poses[f] = poses[f] @ exp_se3(dx[6 * n:6 * n + 6])
    final = evaluate(setup, poses, params.dense_weight(params.num_gn - 1), assoc)
    return {"poses": poses, "energy": final, "trace": trace, "steps": steps, "setup": setup,
            "assoc": assoc, "seconds": time.perf_counter() - t0}


def solve_problem(prob, params=None, linear="cholesky", **kw):
    """Convenience wrapper for a ``synth.Problem``-like object."""
    if params is None:
        params = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    return solve(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
                 prob.corr_q, prob.init_poses, params, linear=linear, **kw)
