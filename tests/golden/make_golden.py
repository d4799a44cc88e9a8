"""Write oracle results for workloads too large to solve inside a GPU test.

Calls only the oracle and the input generator.  Usage:
    python tests/golden/make_golden.py global200
    python tests/golden/make_golden.py global2000
Each file stores a digest of the generated inputs so a test can tell when the
generator no longer reproduces them.
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Params  # noqa: E402
from oracle.gn import solve_problem  # noqa: E402
from synth import make_problem  # noqa: E402


def input_digest(prob):
    h = hashlib.sha256()
    for a in (prob.depth, prob.intensity, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q, prob.init_poses):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def global200():
    prob = make_problem(1)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    res = solve_problem(prob, prm, linear="pcg")
    s = res["setup"]
    # trajectory X_0..X_n and the per-iteration increments (reduced, free frames in order)
    from oracle.se3 import exp_se3
    traj = [prob.init_poses.copy()]
    X = prob.init_poses.copy()
    for st in res["steps"]:
        for n, f in enumerate(s.free):
            X[f] = X[f] @ exp_se3(st["dx"][6 * n:6 * n + 6])
        traj.append(X.copy())
    np.savez_compressed(
        os.path.join(HERE, "global200_oracle.npz"),
        digest=np.array(input_digest(prob)),
        poses=res["poses"], pairs=s.pairs, edges=s.edges, free=s.free,
        traj=np.array(traj), steps=np.array([st["dx"] for st in res["steps"]]),
        energy=np.array([res["energy"][k] for k in ("total", "sparse", "geo", "photo")]),
        counts=np.array([res["energy"][k] for k in ("n_sparse", "n_geo", "n_photo")]),
        trace=np.array([[t[k] for k in ("total", "sparse", "geo", "photo")] for t in res["trace"]]),
        seconds=np.array(res["seconds"]))
    print("global200: oracle solve took", round(res["seconds"], 1), "s")


_G = {}


def _edge_block_range(rng_):
    """Oracle edge blocks of edges [lo, hi) (run in a worker process)."""
    from oracle.gn import edge_blocks
    lo, hi = rng_
    s = _G["setup"]
    sub = type(s).__new__(type(s))
    sub.__dict__.update(s.__dict__)
    sub.edges = s.edges[lo:hi]
    sub.edge_dense = s.edge_dense[lo:hi]
    sub.edge_sparse = s.edge_sparse[lo:hi]
    out = edge_blocks(sub, _G["poses"], _G["wd"])
    keys = ("Hii", "Hij", "Hjj", "gi", "gj")
    packed = {k: np.array([b[k] for b in out]) for k in keys}
    from oracle.gn import energies
    return packed, energies(out)


def _oracle_system(setup, poses, wd, workers):
    """H, g and energies of the oracle at `poses`: the oracle's own edge blocks,
    computed for contiguous edge ranges in worker processes and assembled here in
    edge order (the same sums as oracle.gn.build_system)."""
    import multiprocessing as mp
    from oracle.system import assemble
    E = len(setup.edges)
    step = (E + 8 * workers - 1) // (8 * workers)
    ranges = [(lo, min(E, lo + step)) for lo in range(0, E, step)]
    _G.update(setup=setup, poses=poses, wd=wd)
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_edge_block_range, ranges)
    blocks = []
    en = {k: 0.0 for k in ("total", "sparse", "geo", "photo", "n_sparse", "n_geo", "n_photo")}
    for packed, e in parts:
        n = len(packed["gi"])
        for t in range(n):
            blocks.append({k: packed[k][t] for k in packed})
        for k in en:
            en[k] += e[k]
    H, g = assemble(setup.F, setup.edges, blocks)
    return H, g, en


def global2000(workers=8):
    """Oracle at the 2000-keyframe workload: pair set, variables, energy at the
    initial poses and the first two Gauss-Newton increments (20 PCG iterations,
    block-Jacobi), i.e. one-step references at X_0 and X_1."""
    import time
    from oracle.gn import Setup
    from oracle.se3 import exp_se3
    from oracle.system import inert_frames, reduce_system, solve_pcg
    prob = make_problem(4)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    t0 = time.perf_counter()
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm)
    print("global2000: setup", round(time.perf_counter() - t0, 1), "s,", len(s.pairs), "pairs", flush=True)
    X = prob.init_poses.copy()
    traj, steps, traces, inert_sets = [X.copy()], [], [], []
    for k in range(2):
        t1 = time.perf_counter()
        H, g, en = _oracle_system(s, X, prm.dense_weight(k), workers)
        inert = inert_frames(H, s.free)
        active = s.free[~inert]
        Hr, gr, _ = reduce_system(H, g, active)
        dxa, st = solve_pcg(Hr, gr, prm.num_pcg)
        dx = np.zeros(6 * len(s.free))
        dx.reshape(-1, 6)[~inert] = dxa.reshape(-1, 6)
        for n, f in enumerate(s.free):
            X[f] = X[f] @ exp_se3(dx[6 * n:6 * n + 6])
        traj.append(X.copy())
        steps.append(dx)
        traces.append([en[key] for key in ("total", "sparse", "geo", "photo", "n_sparse", "n_geo", "n_photo")])
        inert_sets.append(inert)
        print(f"global2000: step {k} took {time.perf_counter() - t1:.1f} s, energy {en['total']:.6g}, "
              f"{int(inert.sum())} frames held", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "global2000_oracle.npz"),
        digest=np.array(input_digest(prob)), pairs=s.pairs, free=s.free, traj=np.array(traj),
        steps=np.array(steps), trace=np.array(traces), inert=np.array(inert_sets),
        seconds=np.array(time.perf_counter() - t0))


if __name__ == "__main__":
    for name in sys.argv[1:] or ["global200"]:
        globals()[name]()
