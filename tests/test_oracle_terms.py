"""Pins of the oracle's residuals, Jacobians, pair set and normal equations:
finite differences, zero residual at ground truth, explicit stacked-Jacobian
products, gauge invariance and hand-built camera configurations."""
import numpy as np
import pytest

from oracle import Params
from oracle.frames import prepare_frames
from oracle.gn import Setup, build_system
from oracle.pairs import dense_pairs, group_correspondences
from oracle.se3 import adjoint, exp_se3, inv
from oracle.system import assemble, dense_pair_blocks, free_frames, reduce_system
from oracle.terms import dense_terms, sparse_terms
from synth import make_chunk
from synth.trajectory import look_rotation, make_pose, quat_rot


@pytest.fixture(scope="module")
def clean3():
    return make_chunk(num_frames=3, noise=False, config=0, seed_offset=7)


@pytest.fixture(scope="module")
def noisy3():
    return make_chunk(num_frames=3, noise=True, config=0, seed_offset=11)


def _fd_columns(fun, Ti, Tj, h=1e-6):
    cols = []
    for which in (0, 1):
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            if which == 0:
                rp, rm = fun(Ti @ exp_se3(e), Tj), fun(Ti @ exp_se3(-e), Tj)
            else:
                rp, rm = fun(Ti, Tj @ exp_se3(e)), fun(Ti, Tj @ exp_se3(-e))
            cols.append((rp - rm) / (2 * h))
    J = np.stack(cols, axis=-1)
    return J[..., :6], J[..., 6:]


def _assert_close_cols(Jfd, J, rel=1e-6):
    Jfd = Jfd.reshape(-1, 6)
    J = J.reshape(-1, 6)
    for k in range(6):
        scale = np.linalg.norm(J[:, k]) + 1e-300
        assert np.linalg.norm(Jfd[:, k] - J[:, k]) <= rel * scale, (k, np.linalg.norm(Jfd[:, k] - J[:, k]) / scale)


def test_sparse_jacobian_fd():
    rng = np.random.default_rng(5)
    Ti = exp_se3(rng.normal(size=6) * 0.5)
    Tj = exp_se3(rng.normal(size=6) * 0.5)
    p = rng.normal(size=(40, 3)) * 2
    q = rng.normal(size=(40, 3)) * 2
    r, Ji, Jj = sparse_terms(Ti, Tj, p, q)
    Jfi, Jfj = _fd_columns(lambda A, B: sparse_terms(A, B, p, q)[0], Ti, Tj)
    _assert_close_cols(Jfi, Ji)
    _assert_close_cols(Jfj, Jj)


@pytest.mark.parametrize("pair", [(0, 1), (0, 2), (1, 2)])
def test_dense_jacobian_fd(noisy3, pair):
    prob = noisy3
    prm = Params()
    frames = prepare_frames(prob.depth, prob.intensity, prob.intrinsics, prm)
    i, j = pair
    Ti, Tj = prob.init_poses[i], prob.init_poses[j]
    base = dense_terms(frames[i], frames[j], Ti, Tj, prob.intrinsics, prm)
    assert base["geo"].sum() > 1000 and base["photo"].sum() > 1000
    for rk, Jik, Jjk in (("rg", "Jg_i", "Jg_j"), ("rp", "Jp_i", "Jp_j")):
        fun = lambda A, B: dense_terms(frames[i], frames[j], A, B, prob.intrinsics, prm, assoc=base)[rk]
        Jfi, Jfj = _fd_columns(fun, Ti, Tj)
        _assert_close_cols(Jfi, base[Jik])
        _assert_close_cols(Jfj, base[Jjk])


def test_dense_adjoint_identity(noisy3):
    """The two independently derived dense Jacobians satisfy J_i = -J_j Ad(T_j^-1 T_i)."""
    prob = noisy3
    prm = Params()
    frames = prepare_frames(prob.depth, prob.intensity, prob.intrinsics, prm)
    Ti, Tj = prob.init_poses[0], prob.init_poses[2]
    t = dense_terms(frames[0], frames[2], Ti, Tj, prob.intrinsics, prm)
    Ad = adjoint(inv(Tj) @ Ti)
    for a, b in (("Jg_i", "Jg_j"), ("Jp_i", "Jp_j")):
        scale = np.abs(t[a]).max()
        assert np.abs(t[a] + t[b] @ Ad).max() < 1e-12 * max(scale, 1.0)


def test_zero_residual_at_ground_truth_sparse():
    rng = np.random.default_rng(9)
    Ti = exp_se3(rng.normal(size=6))
    Tj = exp_se3(rng.normal(size=6))
    p = rng.uniform(-2, 2, size=(100, 3))
    Tji = inv(Tj) @ Ti
    q = p @ Tji[:3, :3].T + Tji[:3, 3]
    r, _, _ = sparse_terms(Ti, Tj, p, q)
    assert np.abs(r).max() < 1e-12


def test_duplicate_frame_dense_zero():
    """A frame paired with an identical copy of itself at the same pose: every dense
    residual vanishes and so does the gradient."""
    prob = make_chunk(num_frames=2, noise=True, config=0, seed_offset=3)
    depth = np.stack([prob.depth[0], prob.depth[0]])
    inten = np.stack([prob.intensity[0], prob.intensity[0]])
    prm = Params()
    frames = prepare_frames(depth, inten, prob.intrinsics, prm)
    T = prob.gt_poses[1]
    b = dense_pair_blocks(frames[0], frames[1], T, T, prob.intrinsics, prm, 1.0)
    t = b["terms"]
    assert t["geo"].sum() > 3000 and t["photo"].sum() > 3000
    assert np.abs(t["rg"]).max() < 1e-12 and np.abs(t["rp"]).max() < 1e-12
    assert np.abs(b["gi"]).max() < 1e-10 and np.abs(b["gj"]).max() < 1e-10


def test_planar_room_geometric_zero_at_gt():
    """Noise-free room without spheres: at ground truth the point-to-plane residuals of
    interior plane pixels vanish up to FP32 depth quantisation (|dz| <= 2^-24 z)."""
    prob = make_chunk(num_frames=3, noise=False, spheres=False, config=0, seed_offset=5)
    prm = Params()
    frames = prepare_frames(prob.depth, prob.intensity, prob.intrinsics, prm)
    Ti, Tj = prob.gt_poses[0], prob.gt_poses[2]
    t = dense_terms(frames[0], frames[2], Ti, Tj, prob.intrinsics, prm)
    geo = t["geo"]
    n_src = frames[0].N.reshape(-1, 3)[geo] @ Ti[:3, :3].T
    n_dst = frames[2].N[t["yh"][geo], t["xh"][geo]] @ Tj[:3, :3].T
    # interior: the source normal equals its 8 neighbours' and the target normal (world frame)
    N = frames[0].N
    H, W = N.shape[:2]
    flat = np.zeros((H, W), bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh = np.full_like(N, np.nan)
            sh[max(dy, 0):H + min(dy, 0), max(dx, 0):W + min(dx, 0)] = N[max(-dy, 0):H - max(dy, 0), max(-dx, 0):W - max(dx, 0)]
            flat = flat | ~(np.abs(sh - N).max(-1) < 1e-4)
    flat = ~flat.reshape(-1)[geo]
    interior = flat & (np.abs(n_src - n_dst).max(1) < 1e-4)
    assert interior.sum() > 2000
    assert np.abs(t["rg"][interior]).max() < 2e-6


def test_photometric_small_at_gt(clean3):
    """Sanity bound on rendered scenes: at ground truth only resampling error remains."""
    prob = clean3
    prm = Params(w_geo=0.0, w_sparse=0.0, dense_ramp=False)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
              prob.corr_q, prob.init_poses, prm)
    _, g_gt, _, e_gt = build_system(s, prob.gt_poses, 1.0)
    _, g_in, _, e_in = build_system(s, prob.init_poses, 1.0)
    assert e_gt["photo"] < 0.2 * e_in["photo"]
    assert np.linalg.norm(g_gt[6:]) < 0.4 * np.linalg.norm(g_in[6:])


def _shifted_plane_frames(shift_px):
    """Two views of a fronto-parallel plane at z=2 with texture L(X) = X^2/8 + X/2 + 1/2
    (X the plane coordinate along x, dL/dX > 0 over the view); camera 1 is translated along x so the image moves
    by exactly `shift_px` pixels.  All values are dyadic, hence exact in FP32, and the
    central-difference gradient G is linear in x, so bilinear interpolation of it is exact."""
    intr = (64.0, 64.0, 40.0, 30.0, 80, 60)
    fx, z = 64.0, 2.0
    tx = shift_px * z / fx
    xs = np.arange(80, dtype=np.float64)
    tex = lambda X: X * X / 8.0 + X / 2.0 + 0.5
    L0 = np.tile(tex((xs - 40.0) * z / fx), (60, 1))
    L1 = np.tile(tex((xs - 40.0) * z / fx + tx), (60, 1))
    depth = np.full((2, 60, 80), z, np.float32)
    inten = np.stack([L0, L1]).astype(np.float32)
    assert np.array_equal(inten.astype(np.float64), np.stack([L0, L1]))
    T1 = np.eye(4)
    T1[0, 3] = tx
    return depth, inten, intr, np.stack([np.eye(4), T1])


def test_photometric_exact_zero_on_shifted_plane():
    depth, inten, intr, poses = _shifted_plane_frames(0.375)
    prm = Params()
    frames = prepare_frames(depth, inten, intr, prm)
    t = dense_terms(frames[0], frames[1], poses[0], poses[1], intr, prm)
    assert t["photo"].sum() > 3000
    assert np.abs(t["rp"]).max() < 1e-12 and np.abs(t["rg"]).max() < 1e-12
    # a wrong pose leaves a clearly non-zero photometric residual
    bad = poses[1] @ exp_se3([0, 0, 0, 0.004, 0, 0])
    tb = dense_terms(frames[0], frames[1], poses[0], bad, intr, prm)
    assert np.abs(tb["rp"]).min() > 1e-5


@pytest.mark.parametrize("bidirectional", [False, True])
def test_assembly_matches_stacked_jacobian(noisy3, bidirectional):
    """Block-assembled H and g equal J^T J and J^T r of the explicitly stacked J
    (with both directions per pair: the j -> i rows, whose Jacobians are taken with
    respect to frame j as source and frame i as target, placed in their own columns)."""
    prob = noisy3
    prm = Params(dense_ramp=False, w_photo=0.7, w_sparse=0.3, bidirectional=bidirectional)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
              prob.corr_q, prob.init_poses, prm)
    H, g, blocks, _ = build_system(s, prob.init_poses, 1.0)
    F = prob.num_frames
    rows, res = [], []
    for (i, j), b in zip(s.edges, blocks):
        parts = []
        if b["sparse"] is not None:
            k = s.edge_sparse[list(map(tuple, s.edges)).index((i, j))]
            lo, hi = s.sptr[k], s.sptr[k + 1]
            r, Ji, Jj = sparse_terms(prob.init_poses[i], prob.init_poses[j], s.pa[lo:hi], s.qb[lo:hi])
            parts.append((np.sqrt(prm.w_sparse), r.reshape(-1), Ji.reshape(-1, 6), Jj.reshape(-1, 6)))
        if b["dense"] is not None:
            t = b["dense"]["terms"]
            parts.append((np.sqrt(prm.w_geo), t["rg"], t["Jg_i"], t["Jg_j"]))
            parts.append((np.sqrt(prm.w_photo), t["rp"], t["Jp_i"], t["Jp_j"]))
        if bidirectional and b["dense"] is not None:
            t = dense_terms(s.frames[j], s.frames[i], prob.init_poses[j], prob.init_poses[i], prob.intrinsics, prm)
            assert t["geo"].sum() > 0
            parts.append((np.sqrt(prm.w_geo), t["rg"], t["Jg_j"], t["Jg_i"]))
            parts.append((np.sqrt(prm.w_photo), t["rp"], t["Jp_j"], t["Jp_i"]))
        for sw, r, Ji, Jj in parts:
            Jr = np.zeros((len(r), 6 * F))
            Jr[:, 6 * i:6 * i + 6] = sw * Ji
            Jr[:, 6 * j:6 * j + 6] = sw * Jj
            rows.append(Jr)
            res.append(sw * r)
    J = np.vstack(rows)
    r = np.concatenate(res)
    JtJ = J.T @ J
    assert np.abs(H - JtJ).max() <= 1e-12 * np.abs(JtJ).max()
    assert np.abs(g - J.T @ r).max() <= 1e-12 * np.abs(J.T @ r).max()


def test_system_symmetry_psd_and_gauge(noisy3):
    prob = noisy3
    prm = Params()
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
              prob.corr_q, prob.init_poses, prm)
    H, g, _, _ = build_system(s, prob.init_poses, 1.0)
    assert (H == H.T).all()
    ev = np.linalg.eigvalsh(H)
    assert ev[0] >= -1e-10 * ev[-1]
    # The sparse residual T_i p - T_j q is expressed in world coordinates, so a global
    # rotation rotates it (|r| is invariant, r is not): J^T J keeps the 3 translation
    # null directions.  The dense residuals depend on relative poses only: 6.
    assert (ev < 1e-9 * ev[-1]).sum() == 3
    sd = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
               prob.corr_q, prob.init_poses, Params(use_sparse=False))
    Hd, _, _, _ = build_system(sd, prob.init_poses, 1.0)
    evd = np.linalg.eigvalsh(Hd)
    assert (evd < 1e-9 * evd[-1]).sum() == 6
    Hr, gr, _ = reduce_system(H, g, s.free)
    assert np.linalg.eigvalsh(Hr)[0] > 0
    # a global rigid motion leaves the energy unchanged: sum_f Ad(T_f^-1)^T g_f = 0
    tot = sum(adjoint(inv(prob.init_poses[f])).T @ g[6 * f:6 * f + 6] for f in range(prob.num_frames))
    assert np.abs(tot).max() < 1e-9 * np.abs(g).max()


def test_gauge_invariance_energy(noisy3):
    """E(G X) = E(X) for a rigid G applied to every pose, association frozen."""
    prob = noisy3
    prm = Params(dense_ramp=False)
    frames = prepare_frames(prob.depth, prob.intensity, prob.intrinsics, prm)
    X = prob.init_poses
    G = exp_se3([0.3, -0.2, 0.9, 1.5, -2.0, 0.7])
    for (i, j) in [(0, 1), (1, 2), (0, 2)]:
        a = dense_terms(frames[i], frames[j], X[i], X[j], prob.intrinsics, prm)
        b = dense_terms(frames[i], frames[j], G @ X[i], G @ X[j], prob.intrinsics, prm, assoc=a)
        assert abs(a["rg"] @ a["rg"] - b["rg"] @ b["rg"]) < 1e-12 * (a["rg"] @ a["rg"])
        assert abs(a["rp"] @ a["rp"] - b["rp"] @ b["rp"]) < 1e-12 * (a["rp"] @ a["rp"])
        p, q = prob.corr_p[:50].astype(np.float64), prob.corr_q[:50].astype(np.float64)
        ra = sparse_terms(X[i], X[j], p, q)[0]
        rb = sparse_terms(G @ X[i], G @ X[j], p, q)[0]
        assert abs((ra * ra).sum() - (rb * rb).sum()) < 1e-12 * (ra * ra).sum()


# ----------------------------------------------------------------------------- pairs

INTR = (72.0, 72.0, 40.0, 30.0, 80, 60)


def _wall_depth(T, intr, wall_x=3.0):
    """Depth image of the infinite plane x = wall_x seen from camera T."""
    fx, fy, cx, cy, W, H = intr
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    ray = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], -1) @ T[:3, :3].T
    t = (wall_x - T[0, 3]) / ray[..., 0]
    return np.where(t > 0, t, 0.0).astype(np.float32)


def _pair_case(yaw_deg, shift=0.0):
    """Camera 0 at the origin looking at the wall; camera 1 rotated by yaw about the
    wall point seen by camera 0's centre (plus an optional sideways shift)."""
    R0 = look_rotation(0.0, 0.0)
    T0 = make_pose(R0, np.zeros(3))
    Rz = quat_rot([0, 0, 1], np.deg2rad(yaw_deg))
    pivot = np.array([3.0, 0.0, 0.0])
    T1 = make_pose(Rz @ R0, pivot + Rz @ (-pivot) + np.array([0, shift, 0]))
    depth = np.stack([_wall_depth(T0, INTR), _wall_depth(T1, INTR)])
    return depth, np.stack([T0, T1])


@pytest.mark.parametrize("yaw,expect", [(0.0, True), (30.0, True), (59.9, True), (60.1, False), (180.0, False)])
def test_pair_angle_rule(yaw, expect):
    depth, poses = _pair_case(yaw)
    got = dense_pairs(depth, poses, INTR, Params())
    assert (len(got) == 1) == expect


def test_pair_needs_overlap():
    depth, poses = _pair_case(0.0, shift=40.0)     # same direction, looking at a far part of the wall
    assert len(dense_pairs(depth, poses, INTR, Params())) == 0


def test_correspondence_grouping_round_trip():
    rng = np.random.default_rng(4)
    F = 7
    n = 500
    ci = rng.integers(0, F, n)
    cj = (ci + rng.integers(1, F, n)) % F
    p = rng.normal(size=(n, 3))
    q = rng.normal(size=(n, 3))
    keys, ptr, perm, pa, qb = group_correspondences(ci, cj, p, q, F)
    assert (keys[:, 0] < keys[:, 1]).all()
    assert (np.diff(keys[:, 0] * F + keys[:, 1]) > 0).all()
    # every group holds exactly the correspondences of its pair, in input order
    for k, (a, b) in enumerate(keys):
        idx = perm[ptr[k]:ptr[k + 1]]
        assert (np.diff(idx) > 0).all()
        assert (np.minimum(ci[idx], cj[idx]) == a).all() and (np.maximum(ci[idx], cj[idx]) == b).all()
        sw = ci[idx] > cj[idx]
        assert np.array_equal(pa[ptr[k]:ptr[k + 1]], np.where(sw[:, None], q[idx], p[idx]))
    inv_perm = np.argsort(perm)
    assert np.array_equal(perm[inv_perm], np.arange(n))
    again = group_correspondences(ci, cj, p, q, F)
    assert all(np.array_equal(x, y) for x, y in zip((keys, ptr, perm), again[:3]))


def test_free_frames_rule():
    edges = np.array([[0, 2], [2, 3], [4, 5]])
    assert list(free_frames(7, edges)) == [2, 3, 4, 5]
