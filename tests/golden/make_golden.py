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
from oracle.gn import solve, solve_problem  # noqa: E402
from synth import make_problem  # noqa: E402


def input_digest(prob):
    h = hashlib.sha256()
    for a in (prob.depth, prob.intensity, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q, prob.init_poses):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _trajectory(res):
    """Poses X_0 .. X_n of an oracle run and its increments (free frames in order)."""
    from oracle.se3 import exp_se3
    s = res["setup"]
    X = res["init"].copy()
    traj = [X.copy()]
    for st in res["steps"]:
        for n, f in enumerate(s.free):
            X[f] = X[f] @ exp_se3(st["dx"][6 * n:6 * n + 6])
        traj.append(X.copy())
    return np.array(traj), np.array([st["dx"] for st in res["steps"]])


def converge_sparse(prob, tol=1e-11, max_iters=400):
    """Gauss-Newton with dense Cholesky on the sparse term alone (a smooth energy: no
    association decisions) from the initial poses until the largest increment is
    below `tol` (the outliers make it a large-residual problem, so Gauss-Newton
    converges linearly here, at about 0.77 per iteration at 200 keyframes); returns
    (poses, iterations, largest increment per iteration)."""
    from oracle.gn import Setup, build_system
    from oracle.se3 import exp_se3
    from oracle.system import reduce_system, solve_cholesky
    prm = Params(num_gn=1, num_pcg=1, use_dense=False, dense_ramp=False)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm)
    X = prob.init_poses.copy()
    hist = []
    for _ in range(max_iters):
        H, g, _, _ = build_system(s, X, 0.0)
        Hr, gr, _ = reduce_system(H, g, s.free)
        dx = solve_cholesky(Hr, gr)
        for n, f in enumerate(s.free):
            X[f] = X[f] @ exp_se3(dx[6 * n:6 * n + 6])
        hist.append(float(np.abs(dx).max()))
        if len(hist) % 10 == 0:
            print(f"  sparse-only Gauss-Newton {len(hist)}: largest increment {hist[-1]:.3e}", flush=True)
        if hist[-1] < tol:
            break
    return X, len(hist), np.array(hist)


def global200():
    """The 200-keyframe workload: the oracle's iteration-matched run (8 GN x 20 PCG,
    block-Jacobi, dense weight ramp), its trajectory and increments; the same run
    from initial poses moved by 1e-6 rad / 1e-6 m (seeded directions), which
    measures how far the iteration itself carries a rounding-sized difference; and
    the converged sparse-only solve (Cholesky)."""
    from oracle.se3 import exp_se3
    prob = make_problem(1)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    res = solve_problem(prob, prm, linear="pcg")
    res["init"] = prob.init_poses
    s = res["setup"]
    traj, steps = _trajectory(res)
    print("global200: oracle solve took", round(res["seconds"], 1), "s", flush=True)
    rng = np.random.Generator(np.random.PCG64(77))
    moved = prob.init_poses.copy()
    for f in s.free:
        xi = rng.normal(size=6)
        xi[:3] *= 1e-6 / np.linalg.norm(xi[:3])
        xi[3:] *= 1e-6 / np.linalg.norm(xi[3:])
        moved[f] = moved[f] @ exp_se3(xi)
    res_m = solve(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
                  moved, prm, linear="pcg", pairs=s.pairs)
    conv, n_conv, hist = converge_sparse(prob)
    np.savez_compressed(
        os.path.join(HERE, "global200_oracle.npz"),
        digest=np.array(input_digest(prob)),
        poses=res["poses"], pairs=s.pairs, edges=s.edges, free=s.free,
        traj=traj, steps=steps,
        energy=np.array([res["energy"][k] for k in ("total", "sparse", "geo", "photo")]),
        counts=np.array([res["energy"][k] for k in ("n_sparse", "n_geo", "n_photo")]),
        trace=np.array([[t[k] for k in ("total", "sparse", "geo", "photo")] for t in res["trace"]]),
        seconds=np.array(res["seconds"]),
        moved_init=moved, moved_poses=res_m["poses"], moved_size=np.array(1e-6),
        conv_sparse_poses=conv, conv_sparse_iters=np.array(n_conv), conv_sparse_hist=hist)


def global200_frozen():
    """Add to global200_oracle.npz the runs with the dense association decided once,
    at the initial poses, and held (a smooth energy): the 8 GN x 20 PCG run with the
    dense weight ramp, and the Gauss-Newton run with dense Cholesky and the full
    dense weight to increments below 1e-11."""
    from oracle.gn import Setup, build_system
    from oracle.se3 import exp_se3
    from oracle.system import inert_frames, reduce_system, solve_cholesky
    prob = make_problem(1)
    path = os.path.join(HERE, "global200_oracle.npz")
    g = dict(np.load(path, allow_pickle=False))
    assert str(g["digest"]) == input_digest(prob)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    res = solve_problem(prob, prm, linear="pcg", pairs=g["pairs"], freeze_association=True)
    print("global200 frozen association: 8 x 20 run took", round(res["seconds"], 1), "s", flush=True)
    s = res["setup"]
    assoc = res["assoc"]
    conv = Params(num_gn=1, num_pcg=1, dense_ramp=False)
    X = prob.init_poses.copy()
    hist = []
    for _ in range(200):
        H, gg, _, _ = build_system(s, X, conv.dense_weight(0), assoc)
        inert = inert_frames(H, s.free)
        act = s.free[~inert]
        Hr, gr, _ = reduce_system(H, gg, act)
        dx = solve_cholesky(Hr, gr)
        for n, f in enumerate(act):
            X[f] = X[f] @ exp_se3(dx[6 * n:6 * n + 6])
        hist.append(float(np.abs(dx).max()))
        print(f"  frozen association, Gauss-Newton {len(hist)}: largest increment {hist[-1]:.3e}", flush=True)
        if hist[-1] < 1e-11:
            break
    g.update(frozen_poses=res["poses"],
             frozen_energy=np.array([res["energy"][k] for k in ("total", "sparse", "geo", "photo")]),
             conv_frozen_poses=X, conv_frozen_iters=np.array(len(hist)), conv_frozen_hist=np.array(hist))
    np.savez_compressed(path, **g)


def global200_conv():
    """Recompute only the converged sparse-only solve in global200_oracle.npz."""
    prob = make_problem(1)
    path = os.path.join(HERE, "global200_oracle.npz")
    g = dict(np.load(path, allow_pickle=False))
    assert str(g["digest"]) == input_digest(prob)
    conv, n_conv, hist = converge_sparse(prob)
    g.update(conv_sparse_poses=conv, conv_sparse_iters=np.array(n_conv), conv_sparse_hist=hist)
    np.savez_compressed(path, **g)


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
    """Oracle at the 2000-keyframe workload: pair set, variables, and all 8
    Gauss-Newton iterations (20 PCG iterations, block-Jacobi, dense weight ramp):
    the energy and counts at each iterate, the increments, hence one-step
    references at X_0 .. X_7 and the final poses."""
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
    for k in range(prm.num_gn):
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
    _, _, en = _oracle_system(s, X, prm.dense_weight(prm.num_gn - 1), workers)
    final = [en[key] for key in ("total", "sparse", "geo", "photo", "n_sparse", "n_geo", "n_photo")]
    np.savez_compressed(
        os.path.join(HERE, "global2000_oracle.npz"),
        digest=np.array(input_digest(prob)), pairs=s.pairs, free=s.free, traj=np.array(traj),
        steps=np.array(steps), trace=np.array(traces), inert=np.array(inert_sets), poses=X, final=np.array(final),
        seconds=np.array(time.perf_counter() - t0))


def _pcg_fp32_storage(Hr, gr, iters):
    """The oracle's block-Jacobi PCG with the matrix and the vectors (x, r, z, p, Ap)
    rounded to binary32 after every operation, products summed exactly, dot
    products and alpha/beta in FP64: the arithmetic of a PCG that stores its
    matrix and vectors in FP32 with exact (compensated) accumulation."""
    from oracle.system import block_jacobi_inverse
    f32 = np.float32
    n = Hr.shape[0] // 6
    M = block_jacobi_inverse(Hr).astype(f32).astype(np.float64)
    H32 = Hr.astype(f32).astype(np.float64)

    def prec(r):
        return np.einsum("kab,kb->ka", M, r.reshape(n, 6)).ravel().astype(f32).astype(np.float64)

    x = np.zeros_like(gr)
    r = (-gr).astype(f32).astype(np.float64)
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    for _ in range(iters):
        if rz <= 1e-30:
            break
        Ap = (H32 @ p).astype(f32).astype(np.float64)
        alpha = rz / float(p @ Ap)
        x = (x + alpha * p).astype(f32).astype(np.float64)
        r = (r - alpha * Ap).astype(f32).astype(np.float64)
        z = prec(r)
        rzn = float(r @ z)
        p = (z + (rzn / rz) * p).astype(f32).astype(np.float64)
        rz = rzn
    return x


def global2000_fp32(workers=8):
    """Add to global2000_oracle.npz, for each of the oracle's iterates, how far the
    increment moves when the PCG stores its matrix and vectors in binary32 (with
    exact accumulation): the error that storage precision alone causes on this
    ill-conditioned system."""
    import time
    from oracle.gn import Setup
    from oracle.system import inert_frames, reduce_system, solve_pcg
    prob = make_problem(4)
    path = os.path.join(HERE, "global2000_oracle.npz")
    g = dict(np.load(path, allow_pickle=False))
    assert str(g["digest"]) == input_digest(prob)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm, pairs=g["pairs"])
    errs = []
    for k in range(prm.num_gn):
        t0 = time.perf_counter()
        H, gg, _ = _oracle_system(s, g["traj"][k], prm.dense_weight(k), workers)
        inert = inert_frames(H, s.free)
        Hr, gr, _ = reduce_system(H, gg, s.free[~inert])
        del H
        x64, _ = solve_pcg(Hr, gr, prm.num_pcg)
        x32 = _pcg_fp32_storage(Hr, gr, prm.num_pcg)
        errs.append(float(np.abs(x32 - x64).max()))
        print(f"global2000 step {k}: FP32-stored PCG moves the increment by {errs[-1]:.2e} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    g["fp32_storage_err"] = np.array(errs)
    np.savez_compressed(path, **g)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["global200"]:
        globals()[name]()
