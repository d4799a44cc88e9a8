"""Pins of the oracle's linear solvers and Gauss-Newton loop: library solves, the
Kabsch/Umeyama closed form, an independent least-squares minimiser with
finite-difference Jacobians, descent and quadratic convergence."""
import numpy as np
import pytest
import scipy.optimize

from oracle import Params
from oracle.gn import Setup, build_system, solve
from oracle.se3 import exp_se3, rotation_angle
from oracle.system import reduce_system, solve_cholesky, solve_pcg
from oracle.terms import dense_terms, sparse_terms
from synth import make_chunk


def _spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T


def test_cholesky_matches_library_solve():
    rng = np.random.default_rng(0)
    H = _spd(30, rng)
    g = rng.normal(size=30)
    assert np.allclose(solve_cholesky(H, g), np.linalg.solve(H, -g), rtol=1e-12, atol=1e-14)


def test_pcg_full_dimension_equals_cholesky():
    rng = np.random.default_rng(1)
    H = _spd(36, rng, cond=50.0)
    g = rng.normal(size=36)
    x, st = solve_pcg(H, g, 3 * 36)   # n steps suffice in exact arithmetic; allow for rounding
    ref = solve_cholesky(H, g)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_pcg_block_diagonal_one_iteration():
    rng = np.random.default_rng(2)
    H = np.zeros((24, 24))
    for k in range(4):
        H[6 * k:6 * k + 6, 6 * k:6 * k + 6] = _spd(6, rng)
    g = rng.normal(size=24)
    x, st = solve_pcg(H, g, 1)
    assert st["iters"] == 1
    assert np.allclose(x, solve_cholesky(H, g), rtol=1e-10, atol=1e-12)


def test_jacobi_pcg_full_dimension_equals_cholesky():
    rng = np.random.default_rng(3)
    H = _spd(36, rng, cond=50.0)
    g = rng.normal(size=36)
    x, st = solve_pcg(H, g, 4 * 36, preconditioner="jacobi")
    ref = solve_cholesky(H, g)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_jacobi_pcg_diagonal_one_iteration():
    """With H diagonal the Jacobi preconditioner is H^-1: one step is exact; the
    block-diagonal H of the block-Jacobi pin is not solved in one Jacobi step."""
    rng = np.random.default_rng(4)
    H = np.diag(rng.uniform(0.5, 20.0, 24))
    g = rng.normal(size=24)
    x, st = solve_pcg(H, g, 1, preconditioner="jacobi")
    assert st["iters"] == 1
    assert np.allclose(x, -g / np.diag(H), rtol=1e-14, atol=0)
    Hb = np.zeros((24, 24))
    for k in range(4):
        Hb[6 * k:6 * k + 6, 6 * k:6 * k + 6] = _spd(6, rng)
    x1, _ = solve_pcg(Hb, g, 1, preconditioner="jacobi")
    assert np.linalg.norm(x1 - solve_cholesky(Hb, g)) > 1e-3 * np.linalg.norm(x1)


def test_gn_with_jacobi_preconditioner_converges_to_same_minimum():
    """Both preconditioners reach the Cholesky GN result when PCG runs to
    convergence (association frozen, noise-free chunk)."""
    pr = make_chunk(num_frames=4, noise=False)
    args = (pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q, pr.init_poses)
    ref = solve(*args, Params(num_gn=6, num_pcg=10), linear="cholesky", freeze_association=True)
    jac = solve(*args, Params(num_gn=6, num_pcg=200, preconditioner="jacobi"), linear="pcg",
                freeze_association=True)
    assert np.abs(jac["poses"] - ref["poses"]).max() < 1e-8


def _sparse_only_solve(p, q, init, iters, linear="cholesky"):
    F = len(init)
    depth = np.zeros((F, 60, 80), np.float32)
    prm = Params(use_dense=False, num_gn=iters, num_pcg=12, dense_ramp=False)
    n = len(p)
    ci = np.zeros(n, np.int32)
    cj = np.ones(n, np.int32)
    return solve(depth, depth, (72.0, 72.0, 40.0, 30.0, 80, 60), ci, cj, p, q, init, prm, linear=linear)


def test_two_frame_sparse_equals_kabsch():
    """Sparse-only, two frames: the Gauss-Newton fixed point is the closed-form rigid
    least-squares fit (Kabsch / Umeyama without scale) of sum |p - T_1 q|^2."""
    rng = np.random.default_rng(3)
    T1 = exp_se3([0.1, -0.2, 0.05, 0.3, 0.1, -0.2])
    q = rng.uniform(-2, 2, size=(60, 3))
    p = q @ T1[:3, :3].T + T1[:3, 3] + 0.01 * rng.normal(size=(60, 3))
    init = np.stack([np.eye(4), T1 @ exp_se3([0.03, 0.02, -0.02, 0.05, -0.05, 0.02])])
    res = _sparse_only_solve(p, q, init, 12)
    mp, mq = p.mean(0), q.mean(0)
    S = (p - mp).T @ (q - mq)
    U, _, Vt = np.linalg.svd(S)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U) * np.linalg.det(Vt))])
    R = U @ D @ Vt
    t = mp - R @ mq
    assert np.abs(res["poses"][1][:3, :3] - R).max() < 1e-10
    assert np.abs(res["poses"][1][:3, 3] - t).max() < 1e-10
    assert np.array_equal(res["poses"][0], init[0])


def test_quadratic_convergence_noise_free_sparse():
    rng = np.random.default_rng(4)
    T1 = exp_se3([0.2, 0.1, -0.1, 0.5, -0.3, 0.2])
    q = rng.uniform(-2, 2, size=(40, 3))
    p = q @ T1[:3, :3].T + T1[:3, 3]
    init = np.stack([np.eye(4), T1 @ exp_se3([0.1, -0.08, 0.05, 0.1, 0.1, -0.1])])
    res = _sparse_only_solve(p, q, init, 6)
    steps = [np.linalg.norm(s["dx"]) for s in res["steps"]]
    for a, b in zip(steps, steps[1:]):
        if a > 1e-6:
            assert b <= 10.0 * a * a, steps
    assert steps[-1] < 1e-12


def _frozen_residuals(setup, poses, assoc, prm):
    out = []
    for e, (i, j) in enumerate(setup.edges):
        s = setup.edge_sparse[e]
        if s >= 0:
            lo, hi = setup.sptr[s], setup.sptr[s + 1]
            r = sparse_terms(poses[i], poses[j], setup.pa[lo:hi], setup.qb[lo:hi])[0]
            out.append(np.sqrt(prm.w_sparse) * r.ravel())
        if setup.edge_dense[e] >= 0:
            t = dense_terms(setup.frames[i], setup.frames[j], poses[i], poses[j], setup.intr, prm, assoc=assoc[e])
            out.append(np.sqrt(prm.w_geo) * t["rg"])
            out.append(np.sqrt(prm.w_photo) * t["rp"])
            if prm.bidirectional:
                t = dense_terms(setup.frames[j], setup.frames[i], poses[j], poses[i], setup.intr, prm,
                                assoc=assoc[("rev", e)])
                out.append(np.sqrt(prm.w_geo) * t["rg"])
                out.append(np.sqrt(prm.w_photo) * t["rp"])
    return np.concatenate(out)


@pytest.mark.parametrize("nframes,bidirectional", [(2, False), (3, False), (3, True)])
def test_gn_minimum_matches_least_squares(nframes, bidirectional):
    """All terms, association frozen at the converged poses: an independent
    trust-region least-squares minimiser with finite-difference Jacobians, started
    from several random perturbations, finds the same minimum as Gauss-Newton
    (also with the dense terms of both directions of every pair)."""
    prob = make_chunk(num_frames=nframes, noise=True, config=0, seed_offset=20 + nframes)
    prm = Params(num_gn=40, dense_ramp=False, bidirectional=bidirectional)
    res = solve(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
                prob.corr_q, prob.init_poses, prm, freeze_association=True)
    X = res["poses"]
    assert np.linalg.norm(res["steps"][-1]["dx"]) < 1e-10
    setup = res["setup"]
    assoc = res["assoc"]
    free = list(setup.free)

    def fun(z):
        P = X.copy()
        for n, f in enumerate(free):
            P[f] = X[f] @ exp_se3(z[6 * n:6 * n + 6])
        return _frozen_residuals(setup, P, assoc, prm)

    rng = np.random.default_rng(nframes)
    for start in range(3):
        z0 = rng.normal(size=6 * len(free)) * np.tile([0.01, 0.01, 0.01, 0.02, 0.02, 0.02], len(free))
        ls = scipy.optimize.least_squares(fun, z0, jac="3-point", method="trf", xtol=1e-15, ftol=1e-15,
                                          gtol=1e-15, max_nfev=200)
        for n, f in enumerate(free):
            T = X[f] @ exp_se3(ls.x[6 * n:6 * n + 6])
            assert rotation_angle(T[:3, :3].T @ X[f][:3, :3]) < 1e-7
            assert np.linalg.norm(T[:3, 3] - X[f][:3, 3]) < 1e-7


@pytest.mark.parametrize("noise", [False, True])
def test_monotone_descent(noise):
    """Association held fixed, ramp off, init within 3 cm / 2 deg: every Gauss-Newton
    step lowers the energy.  With re-association at every step the first steps (which
    carry almost all of the decrease) descend too; later ones may move by the energy
    of a few pixels entering or leaving the association."""
    prob = make_chunk(num_frames=6, noise=noise, config=0, seed_offset=30)
    prm = Params(num_gn=6, dense_ramp=False)
    args = (prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
            prob.corr_q, prob.init_poses, prm)
    res = solve(*args, freeze_association=True)
    E = [t["total"] for t in res["trace"]] + [res["energy"]["total"]]
    for a, b in zip(E, E[1:]):
        assert b <= a * (1 + 1e-12), E
    assert np.array_equal(res["poses"][0], prob.init_poses[0])
    res = solve(*args)
    E = [t["total"] for t in res["trace"]]
    assert E[1] < E[0] and E[2] < E[1]
    assert min(E) < E[0] and abs(E[-1] - min(E)) < 1e-3 * min(E)


def test_pcg_mode_approaches_cholesky_on_chunk():
    prob = make_chunk(num_frames=5, noise=True, config=0, seed_offset=40)
    prm = Params(num_gn=3, num_pcg=24, dense_ramp=False)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
              prob.corr_q, prob.init_poses, prm)
    H, g, _, _ = build_system(s, prob.init_poses, 1.0)
    Hr, gr, _ = reduce_system(H, g, s.free)
    x, st = solve_pcg(Hr, gr, 3 * Hr.shape[0])
    ref = solve_cholesky(Hr, gr)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def _drop_frame_data(pr, f):
    """Frame f with no valid depth and no correspondences: it is still a variable
    (lower frames' grid points fall in its view, so it has dense pairs), but no
    residual ever touches it."""
    import copy
    q = copy.copy(pr)
    q.depth = pr.depth.copy()
    q.depth[f] = 0.0
    keep = (pr.corr_i != f) & (pr.corr_j != f)
    q.corr_i, q.corr_j = pr.corr_i[keep], pr.corr_j[keep]
    q.corr_p, q.corr_q = pr.corr_p[keep], pr.corr_q[keep]
    return q


def _delete_frame(pr, f):
    import copy
    q = copy.copy(pr)
    sel = [k for k in range(pr.num_frames) if k != f]
    q.depth, q.intensity = pr.depth[sel], pr.intensity[sel]
    q.init_poses = pr.init_poses[sel]
    keep = (pr.corr_i != f) & (pr.corr_j != f)
    q.corr_i = (pr.corr_i[keep] - (pr.corr_i[keep] > f)).astype(np.int32)
    q.corr_j = (pr.corr_j[keep] - (pr.corr_j[keep] > f)).astype(np.int32)
    q.corr_p, q.corr_q = pr.corr_p[keep], pr.corr_q[keep]
    return q


@pytest.mark.parametrize("linear", ["cholesky", "pcg"])
def test_frame_without_residuals_is_held(linear):
    """A variable frame that no residual touches (its diagonal block is identically
    zero) keeps its pose, and every other frame moves exactly as in the problem
    where that frame does not exist."""
    pr = make_chunk(num_frames=6)
    f = 3
    prm = Params(num_gn=3, num_pcg=10)
    a = _drop_frame_data(pr, f)
    ra = solve(a.depth, a.intensity, a.intrinsics, a.corr_i, a.corr_j, a.corr_p, a.corr_q, a.init_poses, prm,
               linear=linear)
    assert any(f in (i, j) for i, j in ra["setup"].pairs), "frame must keep dense pairs"
    assert f in ra["setup"].free
    b = _delete_frame(pr, f)
    rb = solve(b.depth, b.intensity, b.intrinsics, b.corr_i, b.corr_j, b.corr_p, b.corr_q, b.init_poses, prm,
               linear=linear)
    assert np.array_equal(ra["poses"][f], pr.init_poses[f])
    others = [k for k in range(pr.num_frames) if k != f]
    assert np.abs(ra["poses"][others] - rb["poses"]).max() < 1e-10
    assert abs(ra["energy"]["total"] - rb["energy"]["total"]) <= 1e-10 * rb["energy"]["total"]


def _corrupt_pairs(pr, shifts):
    """Move the q point of every correspondence of the given pairs by a fixed
    offset (metres along x of camera j): whole frame pairs of gross outliers."""
    import copy
    q = copy.copy(pr)
    q.corr_q = pr.corr_q.copy()
    for (a, b), d in shifts.items():
        m = ((pr.corr_i == a) & (pr.corr_j == b)) | ((pr.corr_i == b) & (pr.corr_j == a))
        q.corr_q[m, 0] += d
    return q


def test_pruning_removes_exactly_the_corrupted_pairs():
    """Noise-free chunk with two frame pairs of gross outliers: pruning removes
    those two pairs and nothing else, the largest remaining residual is tiny, and
    the poses return to ground truth; without pruning they do not."""
    from oracle.prune import residual_norms, solve_pruned
    pr = make_chunk(num_frames=6, noise=False, outlier_rate=0.0)
    bad = {(1, 3): 0.6, (2, 4): 0.35}
    c = _corrupt_pairs(pr, bad)
    prm = Params(num_gn=8, num_pcg=30, use_dense=False, dense_ramp=False)
    args = (c.depth, c.intensity, c.intrinsics, c.corr_i, c.corr_j, c.corr_p, c.corr_q, c.init_poses, prm)
    out = solve_pruned(*args, r_prune=0.05, max_rounds=10)
    assert sorted(out["removed"]) == sorted(bad)
    assert out["rmax"] < 1e-6
    assert out["valid"].all()
    err = np.abs(out["poses"] - pr.gt_poses).max()
    plain = solve(*args, linear="pcg")
    assert err < 1e-6 < np.abs(plain["poses"] - pr.gt_poses).max()
    # the residual helper against a per-correspondence loop
    r = residual_norms(pr.gt_poses, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q)
    k = 17
    Ti, Tj = pr.gt_poses[pr.corr_i[k]], pr.gt_poses[pr.corr_j[k]]
    d = (Ti[:3, :3] @ pr.corr_p[k].astype(float) + Ti[:3, 3]) - (Tj[:3, :3] @ pr.corr_q[k].astype(float) + Tj[:3, 3])
    assert abs(r[k] - np.sqrt(d @ d)) < 1e-15


def _scramble_frame(pr, f, scale, seed):
    """Random offsets (uniform, +-scale metres) on the points of frame f in all its
    correspondences: no pose of f explains any of its pairs."""
    import copy
    q = copy.copy(pr)
    rng = np.random.default_rng(seed)
    q.corr_p, q.corr_q = pr.corr_p.copy(), pr.corr_q.copy()
    mi, mj = pr.corr_i == f, pr.corr_j == f
    q.corr_p[mi] += rng.uniform(-scale, scale, size=(mi.sum(), 3)).astype(np.float32)
    q.corr_q[mj] += rng.uniform(-scale, scale, size=(mj.sum(), 3)).astype(np.float32)
    return q


def test_pruning_invalidates_frames_left_without_correspondences():
    from oracle.prune import solve_pruned
    pr = make_chunk(num_frames=5, noise=False, outlier_rate=0.0)
    f = 4
    bad = {(o, f): None for o in range(4)}
    c = _scramble_frame(pr, f, 0.5, 8)
    prm = Params(num_gn=6, num_pcg=30, use_dense=False, dense_ramp=False)
    out = solve_pruned(c.depth, c.intensity, c.intrinsics, c.corr_i, c.corr_j, c.corr_p, c.corr_q, c.init_poses,
                       prm, r_prune=0.05, max_rounds=20)
    assert not out["valid"][f] and out["valid"][:f].all()
    assert sorted(out["removed"]) == sorted(bad)
    assert np.abs(out["poses"][:f] - pr.gt_poses[:f]).max() < 1e-6


def test_pruning_with_no_rounds_is_the_plain_solve():
    from oracle.prune import solve_pruned
    pr = make_chunk(num_frames=4)
    prm = Params(num_gn=3, num_pcg=10)
    args = (pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q, pr.init_poses, prm)
    out = solve_pruned(*args, r_prune=0.05, max_rounds=0)
    plain = solve(*args, linear="pcg")
    assert out["removed"] == []
    assert np.array_equal(out["poses"], plain["poses"])
