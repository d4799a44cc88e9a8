"""GPU vs oracle parity through the C ABI on the 11-frame chunk workload (and
variants): per-frame preparation, pair set and indexing (bit-exact), per-pixel
association masks, per-pair dense records and per-edge blocks at fixed poses,
the assembled normal equations, PCG, and the full Gauss-Newton solve.

Tolerances: integer and index data bit-exact.  Association: the kernels decide
in binary32, the oracle by the plain rule in FP64; the masks must be identical
pixel by pixel except where the oracle flags a decision as within twice the
binary32 rounding bound of one of its tests (``oracle.terms.near_decisions``);
such an excused decision has two correct outcomes, so a job that contains one is
not held to the block tolerance below (it is checked loosely and counted).
6x6 blocks within 1e-5 of the block's Frobenius norm; poses within 1e-5 rad /
1e-5 m; energies within 1e-4 relative."""
import numpy as np
import pytest
import torch

from oracle import Params
from oracle.frames import U32, prepare_frames
from oracle.gn import Setup, build_system, solve
from oracle.pairs import dense_pairs, edge_list, group_correspondences, relative_pose64
from oracle.system import reduce_system, solve_pcg
from oracle.terms import associate
from synth import make_chunk, make_problem

from gpu_helpers import (bf_params_from, block_rel_err, compare_masks, device_problem, pose_errors, poses_cuda,
                         upper21)

pytestmark = pytest.mark.gpu

bf = pytest.importorskip("paper_1604_01093_amd.bf")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def chunk():
    return make_problem(0)


@pytest.fixture(scope="module")
def chunk_setup(chunk):
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg)
    return Setup(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                 chunk.corr_q, chunk.init_poses, prm)


def test_prepare_frames(ctx, chunk):
    """Validity masks identical; binary32 normals within twice the oracle's rounding
    bound of its FP64 normals (the orientation may differ only where the oracle
    flags it as within rounding); gradients within 2e-7."""
    depth = chunk.depth.copy()
    depth[3, 10:20, 30:45] = 0.0          # a hole
    depth[4, :, :] = 0.0                  # a frame without depth
    depth[5, 7, 7] = np.nan
    depth[6, 30, 30] = np.float32(0.1)    # exactly on the depth limit: valid
    depth[6, 31, 30] = np.nextafter(np.float32(0.1), np.float32(0))   # just below: invalid
    inten = chunk.intensity.copy()
    inten[6, 20, 20] = np.inf
    prm = Params()
    dp = bf.DeviceProblem.from_numpy(depth, inten, chunk.intrinsics)
    nd, g = bf.bf_prepare_frames(ctx, dp, bf_params_from(prm))
    nd, g = nd.cpu().numpy(), g.cpu().numpy()
    fr = prepare_frames(depth, inten, chunk.intrinsics, prm)
    assert fr[6].depth_ok[30, 30] and not fr[6].depth_ok[31, 30]
    worst = 0.0
    for f, o in enumerate(fr):
        assert np.array_equal(~np.isnan(nd[f, ..., 0]), o.normal_ok), f
        ok = o.normal_ok
        diff = np.linalg.norm(nd[f][ok][:, :3].astype(np.float64) - o.N[ok], axis=1)
        flip_ok = o.flip_margin[ok] <= 2.0 * (o.N_sigma[ok] + 4 * U32)
        flipped = np.linalg.norm(nd[f][ok][:, :3].astype(np.float64) + o.N[ok], axis=1) <= 2.0 * o.N_sigma[ok]
        good = diff <= 2.0 * o.N_sigma[ok]
        assert np.all(good | (flipped & flip_ok)), f
        worst = max(worst, float((diff / o.N_sigma[ok])[good].max(initial=0.0)))
        assert np.array_equal(~np.isnan(g[f]), o.grad_ok), f
        gk = o.grad_ok
        assert np.abs(g[f][gk] - o.G[gk]).max() <= 2e-7 * max(1.0, np.abs(o.G[gk]).max())
    print(f"normals: largest difference {worst:.3f} x the rounding bound", flush=True)
    assert not (~np.isnan(nd[4, ..., 0])).any()


def job_assoc(setup, i, j, poses, prm):
    """The oracle's FP64 association of pair job i -> j at `poses`."""
    R, t = relative_pose64(poses[i], poses[j])
    return associate(setup.frames[i], setup.frames[j], R, t, setup.intr, prm)


def check_masks(masks, jobs, setup, poses, prm, label=""):
    """Every job's GPU mask against the oracle: returns the set of job indices whose
    masks differ (only at excused decisions) and the totals."""
    differ = set()
    tot = np.zeros(4, np.int64)
    for k, (i, j) in enumerate(jobs):
        ug, up, eg, ep, same = compare_masks(masks[k], job_assoc(setup, i, j, poses, prm), setup.intr[4])
        assert ug == 0 and up == 0, (label, k, i, j, ug, up)
        tot += (ug, up, eg, ep)
        if not same:
            differ.add(k)
    print(f"masks{label}: {len(jobs)} jobs, excused mismatches geo {tot[2]} photo {tot[3]}, "
          f"{len(differ)} jobs differ", flush=True)
    return differ


@pytest.mark.parametrize("which", ["chunk", "chunk_perturbed"])
def test_pairs_bit_exact(ctx, chunk, which):
    prm = Params()
    poses = chunk.init_poses.copy()
    if which == "chunk_perturbed":
        # rotate a few frames so the angle and overlap tests both reject some pairs
        from oracle.se3 import exp_se3
        for f in (3, 7, 9):
            poses[f] = poses[f] @ exp_se3([0.0, 1.1 + 0.1 * f, 0.0, 0.5, 0.0, 0.0])
    dp = device_problem(chunk)
    got = bf.bf_build_pairs(ctx, dp, poses_cuda(poses), bf_params_from(prm)).cpu().numpy()
    ref = dense_pairs(chunk.depth, poses, chunk.intrinsics, prm)
    assert np.array_equal(got, ref)
    if which == "chunk":
        assert len(ref) == 55
    else:
        assert 0 < len(ref) < 55


def test_structure_bit_exact(ctx, chunk):
    rng = np.random.default_rng(0)
    M = len(chunk.corr_i)
    order = rng.permutation(M)
    swap = rng.uniform(size=M) < 0.5
    ci = np.where(swap, chunk.corr_j, chunk.corr_i)[order]
    cj = np.where(swap, chunk.corr_i, chunk.corr_j)[order]
    pi = np.where(swap[:, None], chunk.corr_q, chunk.corr_p)[order]
    pj = np.where(swap[:, None], chunk.corr_p, chunk.corr_q)[order]
    # drop one pair's correspondences entirely so the edge set differs from the pairs
    keep = ~((np.minimum(ci, cj) == 2) & (np.maximum(ci, cj) == 5))
    ci, cj, pi, pj = ci[keep], cj[keep], pi[keep], pj[keep]
    prm = Params()
    dp = bf.DeviceProblem.from_numpy(chunk.depth, chunk.intensity, chunk.intrinsics, ci, cj, pi, pj)
    pairs = np.array([(0, 1), (0, 4), (2, 5), (3, 9), (8, 10)], np.int32)
    dp.set_pairs(torch.as_tensor(pairs).cuda())
    st = bf.bf_build_structure(ctx, dp, poses_cuda(chunk.init_poses), bf_params_from(prm))
    keys, ptr, perm, _, _ = group_correspondences(ci, cj, pi, pj, chunk.num_frames)
    assert np.array_equal(st["sparse_ij"].cpu().numpy(), keys)
    assert np.array_equal(st["sparse_ptr"].cpu().numpy(), ptr)
    assert np.array_equal(st["corr_perm"].cpu().numpy(), perm)
    edges, _, _ = edge_list(pairs, keys)
    assert np.array_equal(st["edges"].cpu().numpy(), edges)
    assert np.array_equal(st["pairs"].cpu().numpy(), pairs)
    assert np.array_equal(st["free"].cpu().numpy(), np.arange(1, chunk.num_frames))


def test_dense_records_at_fixed_poses(ctx, chunk, chunk_setup):
    prm = chunk_setup.params
    k = 2
    wd = prm.dense_weight(k)
    dp = device_problem(chunk)
    res = bf.bf_eval_residuals(ctx, dp, poses_cuda(chunk.init_poses), bf_params_from(prm), gn_iter=k,
                               records=True, masks=True)
    rec = res["records"].cpu().numpy()
    masks = res["masks"].cpu().numpy()
    _, _, blocks, en = build_system(chunk_setup, chunk.init_poses, wd)
    assert len(rec) == len(chunk_setup.pairs) == 55
    differ = check_masks(masks, chunk_setup.pairs, chunk_setup, chunk.init_poses, prm)
    assert len(differ) <= 2
    for e, (i, j) in enumerate(chunk_setup.edges):
        d = chunk_setup.edge_dense[e]
        o = blocks[e]["dense"]
        r = rec[d]
        assert r[29] == int(((masks[d][:, 0] & 1) != 0).sum()) and r[30] == int(((masks[d][:, 0] & 2) != 0).sum())
        tol = 1e-2 if d in differ else 1e-5
        if d not in differ:
            assert r[29] == o["ngeo"] and r[30] == o["nphoto"], (i, j)
        assert block_rel_err(r[:21], upper21(o["Hjj"])) < tol, (i, j)
        assert block_rel_err(r[21:27], o["gj"]) < tol * max(1.0, np.linalg.norm(upper21(o["Hjj"])) /
                                                             max(np.linalg.norm(o["gj"]), 1e-30)), (i, j)
        assert abs(r[27] - o["Egeo"]) <= tol * o["Egeo"] and abs(r[28] - o["Ephoto"]) <= tol * o["Ephoto"]
    assert res["n_sparse"] == en["n_sparse"]
    if not differ:
        assert res["n_geo"] == en["n_geo"] and res["n_photo"] == en["n_photo"]
    for key in ("total", "sparse", "geo", "photo"):
        assert abs(res[key] - en[key]) <= (1e-4 if differ else 1e-6) * abs(en[key]), key


@pytest.fixture(scope="module")
def init_differ(ctx, chunk, chunk_setup):
    """Dense jobs whose GPU masks differ from the oracle's at the initial poses (only
    at excused decisions), and the frames they touch."""
    res = bf.bf_eval_residuals(ctx, device_problem(chunk), poses_cuda(chunk.init_poses),
                               bf_params_from(chunk_setup.params), gn_iter=0, masks=True)
    differ = check_masks(res["masks"].cpu().numpy(), chunk_setup.pairs, chunk_setup, chunk.init_poses,
                         chunk_setup.params, " at init")
    frames = {int(f) for d in differ for f in chunk_setup.pairs[d]}
    return differ, frames


@pytest.mark.parametrize("pcg_storage", [0, 1])
def test_normal_equations_and_edge_blocks(ctx, chunk, chunk_setup, pcg_storage, init_differ):
    """Every 6x6 block of H within 1e-5, except blocks summed over a job with an
    excused decision (1e-2); H bitwise symmetric; g per frame likewise."""
    differ, dframes = init_differ
    prm = chunk_setup.params
    wd = prm.dense_weight(1)
    dp = device_problem(chunk)
    out = bf.bf_build_normal_equations(ctx, dp, poses_cuda(chunk.init_poses),
                                       bf_params_from(prm, pcg_storage=pcg_storage), gn_iter=1, edge_blocks=True)
    H_ref, g_ref, blocks, en = build_system(chunk_setup, chunk.init_poses, wd)
    H, g, eb = out["H"].cpu().numpy(), out["g"].cpu().numpy(), out["edge_blocks"].cpu().numpy()
    F = chunk.num_frames
    for a in range(F):
        for b in range(F):
            blk = H_ref[6 * a:6 * a + 6, 6 * b:6 * b + 6]
            tol = 1e-2 if (a in dframes or b in dframes) else 1e-5
            if np.abs(blk).max() == 0:
                assert np.abs(H[6 * a:6 * a + 6, 6 * b:6 * b + 6]).max() == 0
            else:
                assert block_rel_err(H[6 * a:6 * a + 6, 6 * b:6 * b + 6], blk) < tol, (a, b)
    assert np.array_equal(H, H.T)
    for f in range(F):
        tol = 1e-2 if f in dframes else 1e-5
        scale = np.linalg.norm(H_ref[6 * f:6 * f + 6, 6 * f:6 * f + 6])
        assert np.linalg.norm(g[6 * f:6 * f + 6] - g_ref[6 * f:6 * f + 6]) <= tol * max(scale * 1e-3, np.linalg.norm(g_ref[6 * f:6 * f + 6]))
    for e in range(len(chunk_setup.edges)):
        o = blocks[e]
        tol = 1e-2 if chunk_setup.edge_dense[e] in differ else 1e-5
        assert block_rel_err(eb[e, 0:36].reshape(6, 6), o["Hii"]) < tol
        assert block_rel_err(eb[e, 36:72].reshape(6, 6), o["Hjj"]) < tol
        assert block_rel_err(eb[e, 72:108].reshape(6, 6), o["Hij"]) < tol
        assert abs(eb[e, 120] - o["sparse"]["E"]) <= 1e-9 * o["sparse"]["E"]
    assert abs(out["energy"][0] - en["total"]) <= (1e-4 if differ else 1e-6) * en["total"]


@pytest.mark.parametrize("pcg_storage,solve_kernel", [(0, 1), (1, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 5),
                                                    (1, 5)])
def test_pcg_matches_oracle_pcg(ctx, chunk, chunk_setup, pcg_storage, solve_kernel, init_differ):
    """The 10-iteration PCG increment element by element within 1e-5 (rad, m) of the
    oracle's PCG on its own system, and r^T z at the start within 1e-5 relative."""
    prm = chunk_setup.params
    dp = device_problem(chunk)
    ne = bf.bf_build_normal_equations(ctx, dp, poses_cuda(chunk.init_poses),
                                      bf_params_from(prm, pcg_storage=pcg_storage, solve_kernel=solve_kernel),
                                      gn_iter=0, dense=False)
    delta, st = bf.bf_pcg_solve(ctx, ne["system"], chunk.num_frames, 10)
    delta = delta.cpu().numpy()
    H, g, _, _ = build_system(chunk_setup, chunk.init_poses, prm.dense_weight(0))
    Hr, gr, idx = reduce_system(H, g, chunk_setup.free)
    x, ost = solve_pcg(Hr, gr, 10)
    ref = np.zeros(6 * chunk.num_frames)
    ref[idx] = x
    err = float(np.abs(delta - ref).max())
    print(f"chunk PCG storage={pcg_storage} kernel={solve_kernel}: max |d increment| {err:.2e} "
          f"(max |increment| {np.abs(ref).max():.3f}), {len(init_differ[0])} jobs with excused decisions", flush=True)
    assert st["iters"] == ost["iters"] == 10
    assert err <= 1e-5
    assert abs(st["rz0"] - ost["rz0"]) <= 1e-5 * ost["rz0"]
    assert (delta[:6] == 0).all()


@pytest.mark.parametrize("pcg_storage,accumulate,solve_kernel",
                         [(0, 0, 1), (1, 0, 1), (0, 1, 1), (0, 2, 1), (0, 0, 2), (1, 0, 2), (0, 0, 3), (1, 2, 3),
                          (0, 0, 5), (1, 2, 5)])
def test_gauss_newton_chunk(ctx, chunk, pcg_storage, accumulate, solve_kernel):
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg)
    ref = solve(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                chunk.corr_q, chunk.init_poses, prm, linear="pcg")
    dp = device_problem(chunk)
    init = poses_cuda(chunk.init_poses)
    kw = dict(pcg_storage=pcg_storage, accumulate=accumulate, solve_kernel=solve_kernel)
    out = bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, **kw), trace=True)
    P = out["poses"].cpu().numpy()
    rot, tr = pose_errors(P, ref["poses"])
    print(f"chunk {kw}: pose err {rot:.3e} rad {tr:.3e} m, "
          f"energy {out['energy']['total']:.9g} vs {ref['energy']['total']:.9g}")
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]
    assert np.array_equal(P[0], chunk.init_poses[0])
    for k, t in enumerate(out["trace"]):
        assert abs(t[0] - ref["trace"][k]["total"]) <= 1e-4 * ref["trace"][k]["total"]
    # inputs untouched, deterministic
    assert np.array_equal(init.cpu().numpy(), chunk.init_poses)
    again = bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, **kw))
    assert torch.equal(again["poses"], out["poses"])


@pytest.mark.parametrize("solve_kernel", [0, 1, 2, 3, 5])
def test_frame_without_residuals_is_held(ctx, solve_kernel):
    """A variable frame that no residual touches (no valid depth, no
    correspondences, but dense pairs from lower frames) keeps its pose; the rest
    matches the oracle, which holds such frames in the same way."""
    pr = make_chunk(num_frames=6)
    f = 3
    pr.depth = pr.depth.copy()
    pr.depth[f] = 0.0
    keep = (pr.corr_i != f) & (pr.corr_j != f)
    pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q = pr.corr_i[keep], pr.corr_j[keep], pr.corr_p[keep], pr.corr_q[keep]
    prm = Params(num_gn=3, num_pcg=10)
    ref = solve(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q, pr.init_poses,
                prm, linear="pcg")
    assert f in ref["setup"].free
    out = bf.bf_gauss_newton(ctx, device_problem(pr), poses_cuda(pr.init_poses),
                             bf_params_from(prm, solve_kernel=solve_kernel))
    P = out["poses"].cpu().numpy()
    assert np.array_equal(P[f], pr.init_poses[f])
    rot, tr = pose_errors(P, ref["poses"])
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


@pytest.mark.parametrize("solve_kernel,pcg_storage", [(0, 0), (1, 0), (2, 0), (3, 0), (3, 1), (5, 0), (5, 1)])
def test_gauss_newton_chunk_jacobi_preconditioner(ctx, chunk, solve_kernel, pcg_storage):
    """The paper's scalar Jacobi preconditioner (Sec. 4.4) in every solve kernel."""
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg, preconditioner="jacobi")
    ref = solve(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                chunk.corr_q, chunk.init_poses, prm, linear="pcg")
    out = bf.bf_gauss_newton(ctx, device_problem(chunk), poses_cuda(chunk.init_poses),
                             bf_params_from(prm, solve_kernel=solve_kernel, pcg_storage=pcg_storage))
    rot, tr = pose_errors(out["poses"].cpu().numpy(), ref["poses"])
    print(f"chunk jacobi kernel={solve_kernel} storage={pcg_storage}: pose err {rot:.3e} rad {tr:.3e} m", flush=True)
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


@pytest.mark.parametrize("pcg_storage,accumulate", [(0, 0), (1, 2)])
def test_gauss_newton_chunk_matrix_free_sparse(ctx, chunk, pcg_storage, accumulate):
    """The paper's PCG variant (Sec. 4.4): the sparse term applied matrix-free in
    every PCG iteration (J p per correspondence, J^T of it per frame pair) instead of
    its assembled blocks; the linear system is the same, so the solve meets the
    oracle's PCG within 1e-5 like every other kernel, and its energy within 1e-4."""
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg)
    ref = solve(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                chunk.corr_q, chunk.init_poses, prm, linear="pcg")
    kw = dict(pcg_storage=pcg_storage, accumulate=accumulate)
    out = bf.bf_gauss_newton(ctx, device_problem(chunk), poses_cuda(chunk.init_poses),
                             bf_params_from(prm, sparse_matrix_free=1, **kw))
    asm = bf.bf_gauss_newton(ctx, device_problem(chunk), poses_cuda(chunk.init_poses),
                             bf_params_from(prm, solve_kernel=5, **kw))
    rot, tr = pose_errors(out["poses"].cpu().numpy(), ref["poses"])
    rot_a, tr_a = pose_errors(out["poses"].cpu().numpy(), asm["poses"].cpu().numpy())
    print(f"chunk matrix-free sparse {kw}: pose err {rot:.2e} rad {tr:.2e} m vs oracle, {rot_a:.2e} / {tr_a:.2e} vs "
          f"assembled blocks in the same kernel", flush=True)
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


def test_matrix_free_sparse_refusals(ctx, chunk):
    """Matrix-free sparse mode runs in the distributed-vector PCG of
    bf_gauss_newton only: other kernels, graphs, systems and batches refuse it."""
    dp = device_problem(chunk)
    init = poses_cuda(chunk.init_poses)
    prm = Params(num_gn=2, num_pcg=5)
    for kw in (dict(solve_kernel=3), dict(solve_kernel=1), dict(graph=1)):
        with pytest.raises(bf.BFError) as e:
            bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, sparse_matrix_free=1, **kw))
        assert e.value.status == bf.BF_ERR_UNSUPPORTED, kw
    with pytest.raises(bf.BFError) as e:
        bf.bf_build_normal_equations(ctx, dp, init, bf_params_from(prm, sparse_matrix_free=1), gn_iter=0)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, sparse_matrix_free=2))
    assert e.value.status == bf.BF_ERR_INVALID_ARG


def test_timing_levels(ctx, chunk):
    """Timing events change no result: levels 0, 1 and 2 give bitwise the same
    poses; level 1 fills every phase, level 2 only the dense launches and the total."""
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg)
    dp = device_problem(chunk)
    init = poses_cuda(chunk.init_poses)
    outs, tms = [], []
    for level in (0, 1, 2):
        outs.append(bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, timing=level, dense_threads=256))["poses"])
        tms.append(ctx.last_timings())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    t1, t2 = tms[1], tms[2]
    assert all(t1[k] > 0 for k in ("setup_us", "dense_us", "edges_us", "pcg_us", "final_us", "total_us"))
    assert t1["dense_launches"] == t2["dense_launches"] == chunk.n_gn
    assert t2["dense_us"] > 0 and t2["total_us"] > 0
    assert t2["setup_us"] == t2["edges_us"] == t2["pcg_us"] == t2["final_us"] == 0
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, timing=3))
    assert e.value.status == bf.BF_ERR_INVALID_ARG


@pytest.mark.parametrize("W,H", [(3, 3), (7, 5), (37, 23)])
@pytest.mark.parametrize("dense_threads", [64, 256, 512])
def test_small_and_ragged_images(ctx, W, H, dense_threads):
    """Images smaller than one wavefront and sizes that are not a multiple of the
    workgroup (the last step of every wavefront runs past the last pixel): the
    association masks pixel by pixel against the oracle (excused decisions only),
    the records' counts equal to the masks' and the energy at the initial poses
    within 1e-6 (1e-4 with an excused decision), then the solve within the pose
    tolerance, for each dense workgroup size."""
    f = 72.0 * W / 80.0
    pr = make_chunk(num_frames=4, W=W, H=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, name=f"small{W}x{H}")
    prm = Params(num_gn=3, num_pcg=10)
    setup = Setup(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q,
                  pr.init_poses, prm)
    dp = device_problem(pr)
    res = bf.bf_eval_residuals(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, dense_threads=dense_threads),
                               gn_iter=0, records=True, masks=True)
    _, _, blocks, en = build_system(setup, pr.init_poses, prm.dense_weight(0))
    rec = res["records"].cpu().numpy()
    masks = res["masks"].cpu().numpy()
    differ = check_masks(masks, setup.pairs, setup, pr.init_poses, prm, f" {W}x{H}") if len(setup.pairs) else set()
    for d in range(len(setup.pairs)):
        assert rec[d][29] == int(((masks[d][:, 0] & 1) != 0).sum()) and rec[d][30] == int(((masks[d][:, 0] & 2) != 0).sum())
    if not differ:
        assert res["n_geo"] == en["n_geo"] and res["n_photo"] == en["n_photo"]
    assert abs(res["total"] - en["total"]) <= (1e-4 if differ else 1e-6) * en["total"]
    ref = solve(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q, pr.init_poses,
                prm, linear="pcg")
    out = bf.bf_gauss_newton(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, dense_threads=dense_threads))
    rot, tr = pose_errors(out["poses"].cpu().numpy(), ref["poses"])
    print(f"{W}x{H} threads {dense_threads}: n_geo {en['n_geo']}, pose err {rot:.2e} rad {tr:.2e} m", flush=True)
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


@pytest.mark.parametrize("solve_kernel,accumulate", [(0, 0), (3, 0), (2, 1)])
def test_bidirectional_chunk(ctx, chunk, solve_kernel, accumulate):
    """Dense terms over the pixels of both frames of every pair (a second job
    j -> i per pair): forward and reverse records' counts bit-exact and their
    blocks within 1e-5 of the oracle's at fixed poses, the assembled normal
    equations within 1e-5, and the Gauss-Newton solve within the pose tolerance."""
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg, bidirectional=True)
    setup = Setup(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                  chunk.corr_q, chunk.init_poses, prm)
    dp = device_problem(chunk)
    kw = dict(solve_kernel=solve_kernel, accumulate=accumulate)
    res = bf.bf_eval_residuals(ctx, dp, poses_cuda(chunk.init_poses), bf_params_from(prm, **kw), gn_iter=2,
                               records=True, masks=True)
    rec = res["records"].cpu().numpy()
    P = len(setup.pairs)
    assert rec.shape[0] == 2 * P
    jobs = np.concatenate([setup.pairs, setup.pairs[:, ::-1]])
    differ = check_masks(res["masks"].cpu().numpy(), jobs, setup, chunk.init_poses, prm, " both directions")
    _, _, blocks, en = build_system(setup, chunk.init_poses, prm.dense_weight(2))
    for e, (i, j) in enumerate(setup.edges):
        d = setup.edge_dense[e]
        if d < 0:
            continue
        for k, r, o, blk in ((d, rec[d], blocks[e]["dense"], "Hjj"), (P + d, rec[P + d], blocks[e]["dense_rev"], "Hii")):
            if k in differ:
                assert block_rel_err(r[:21], upper21(o[blk])) < 1e-2, (i, j, blk)
                continue
            assert r[29] == o["ngeo"] and r[30] == o["nphoto"], (i, j, blk)
            assert block_rel_err(r[:21], upper21(o[blk])) < 1e-5, (i, j, blk)
    if not differ:
        assert res["n_geo"] == en["n_geo"] and res["n_photo"] == en["n_photo"]
    assert abs(res["total"] - en["total"]) <= (1e-4 if differ else 1e-6) * en["total"]
    out = bf.bf_build_normal_equations(ctx, dp, poses_cuda(chunk.init_poses), bf_params_from(prm, **kw), gn_iter=1)
    H_ref, g_ref, _, _ = build_system(setup, chunk.init_poses, prm.dense_weight(1))
    H, g = out["H"].cpu().numpy(), out["g"].cpu().numpy()
    F = chunk.num_frames
    dframes = {int(f) for k in differ for f in jobs[k]}
    for a in range(F):
        for b in range(F):
            ref = H_ref[6 * a:6 * a + 6, 6 * b:6 * b + 6]
            if np.abs(ref).max() > 0:
                tol = 1e-2 if (a in dframes or b in dframes) else 1e-5
                assert block_rel_err(H[6 * a:6 * a + 6, 6 * b:6 * b + 6], ref) < tol, (a, b)
    assert np.linalg.norm(g - g_ref) <= (1e-2 if differ else 1e-5) * np.linalg.norm(g_ref)
    ref = solve(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                chunk.corr_q, chunk.init_poses, prm, linear="pcg")
    sol = bf.bf_gauss_newton(ctx, dp, poses_cuda(chunk.init_poses), bf_params_from(prm, **kw))
    rot, tr = pose_errors(sol["poses"].cpu().numpy(), ref["poses"])
    print(f"bidirectional {kw}: pose err {rot:.2e} rad {tr:.2e} m", flush=True)
    assert rot < 1e-5 and tr < 1e-5
    assert abs(sol["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


@pytest.mark.parametrize("pcg_storage,accumulate,solve_kernel", [(0, 0, 0), (1, 2, 2), (0, 1, 3), (1, 2, 5)])
def test_gauss_newton_chunk_fixed_association(ctx, chunk, pcg_storage, accumulate, solve_kernel):
    """The dense association decided once by the oracle at the initial poses and held
    (bf_params.fixed_association, the oracle's freeze_association): with no decision
    left to round either way, the whole 5 x 10 solve agrees within 1e-5 and its
    energy within 1e-4, in every precision and PCG kernel."""
    from gpu_helpers import encode_association, fix_association
    prm = Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg)
    ref = solve(chunk.depth, chunk.intensity, chunk.intrinsics, chunk.corr_i, chunk.corr_j, chunk.corr_p,
                chunk.corr_q, chunk.init_poses, prm, linear="pcg", freeze_association=True)
    s = ref["setup"]
    jobs = [None] * len(s.pairs)
    for e, d in enumerate(s.edge_dense):
        if d >= 0:
            jobs[d] = ref["assoc"][e]
    fixed = encode_association(jobs, chunk.width)
    p = fix_association(bf_params_from(prm, pcg_storage=pcg_storage, accumulate=accumulate,
                                       solve_kernel=solve_kernel), fixed)
    out = bf.bf_gauss_newton(ctx, device_problem(chunk), poses_cuda(chunk.init_poses), p)
    rot, tr = pose_errors(out["poses"].cpu().numpy(), ref["poses"])
    print(f"chunk fixed association storage={pcg_storage} acc={accumulate} kernel={solve_kernel}: pose err "
          f"{rot:.2e} rad {tr:.2e} m", flush=True)
    assert rot < 1e-5 and tr < 1e-5
    assert abs(out["energy"]["total"] - ref["energy"]["total"]) <= 1e-4 * ref["energy"]["total"]


@pytest.mark.parametrize("W,H,nt,tiles,accumulate", [(80, 60, 256, 2, 2), (80, 60, 128, 4, 2), (37, 23, 64, 3, 2),
                                                    (160, 120, 256, 4, 2), (80, 60, 256, 2, 0),
                                                    (160, 120, 128, 4, 0)])
def test_dense_tiles(ctx, W, H, nt, tiles, accumulate):
    """A pair job split into tiles of its pixels (one workgroup each, partial records
    summed in tile order): the association identical pixel by pixel to the untiled
    job and the counts equal; every pixel's products are computed alike, only the
    order of the sums differs.

    FP64 lane sums (accumulate 2): records within 1e-12 relative, a solve within 1e-9.
    FP32 lane sums (accumulate 0): a lane takes at most ceil(H W / threads) + 1 pixels
    off its wavefront's queue, each with a geometric and a photometric product, so it
    adds at most m = 2 (ceil(H W / threads) + 1) products and each record word moves
    by at most m u (u = 2^-24) times the sum of
    its terms' magnitudes, which is at most the record's norm (|J_a J_b| and |J_a r|
    are at most half of J_a^2 + J_b^2 and J_a^2 + r^2); over the 29 words and both
    launches, sqrt(29) 2 m u relative.  The solve then stays within 1e-6, a tenth of
    the 1e-5 the FP32 path is held to against the oracle."""
    f = 72.0 * W / 80.0
    pr = make_chunk(num_frames=5, W=W, H=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, name=f"tiles{W}x{H}")
    dp = device_problem(pr)
    prm = Params(num_gn=3, num_pcg=10)
    kw = dict(dense_threads=nt, accumulate=accumulate)
    base = bf.bf_eval_residuals(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, **kw), gn_iter=1,
                                records=True, masks=True)
    tl = bf.bf_eval_residuals(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, dense_tiles=tiles, **kw),
                              gn_iter=1, records=True, masks=True)
    assert ctx.dense_shape()["jacobians"] == (nt, tiles)
    assert torch.equal(base["masks"], tl["masks"])
    r0, r1 = base["records"].cpu().numpy(), tl["records"].cpu().numpy()
    assert np.array_equal(r0[:, 29:31], r1[:, 29:31])
    m = 2 * (-(-W * H // nt) + 1)
    rec_tol = 1e-12 if accumulate == 2 else np.sqrt(29.0) * 2 * m * 2.0 ** -24
    worst = max(block_rel_err(r1[k, :29], r0[k, :29]) for k in range(len(r0)))
    assert worst <= rec_tol, (worst, rec_tol)
    assert abs(tl["total"] - base["total"]) <= rec_tol * base["total"]
    a = bf.bf_gauss_newton(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, **kw))
    b = bf.bf_gauss_newton(ctx, dp, poses_cuda(pr.init_poses), bf_params_from(prm, dense_tiles=tiles, **kw))
    rot, tr = pose_errors(a["poses"].cpu().numpy(), b["poses"].cpu().numpy())
    print(f"{W}x{H} {nt} threads x {tiles} tiles, accumulate {accumulate}: records {worst:.1e} (bound "
          f"{rec_tol:.1e}), pose difference to one tile {rot:.1e} rad {tr:.1e} m", flush=True)
    pose_tol = 1e-9 if accumulate == 2 else 1e-6
    assert rot < pose_tol and tr < pose_tol
