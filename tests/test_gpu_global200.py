"""Full-size parity on the 200-keyframe global workload, in the configuration the
benchmark times (8 GN x 20 PCG, FP32 PCG storage, automatic solve kernel).

* the dense pair set and the edge list, bit-exact against the oracle's run stored
  in tests/golden/global200_oracle.npz (written by tests/golden/make_golden.py,
  which calls only the oracle);
* per-pair dense records at the initial poses on a sample of 64 pair jobs,
  computed by the oracle one pair at a time: association counts bit-exact,
  6x6 blocks within 1e-5 of their Frobenius norm;
* one Gauss-Newton step at each of the oracle's 8 iterates (same poses, same
  pair set): the GPU increment matches the oracle's within 1e-5 (rad, m);
* the full 8-iteration solve: energy within 1e-4 relative of the oracle's.  The
  poses of two independently rounded runs drift apart along this
  non-converged, re-associating iteration (a 1e-8 difference flips a few of the
  3 million association decisions, and each step amplifies ~10x), so the
  end-to-end pose difference (about 1e-4) is reported and bounded by 2e-3 as a
  regression guard; the strict check is the one-step parity above."""
import os

import numpy as np
import pytest
import torch

from oracle import Params
from oracle.frames import prepare_frame
from oracle.system import dense_pair_blocks
from synth import make_problem

from gpu_helpers import bf_params_from, block_rel_err, device_problem, pose_errors, poses_cuda, upper21

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "global200_oracle.npz")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def prob():
    return make_problem(1)


@pytest.fixture(scope="module")
def golden(prob):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(os.path.dirname(GOLDEN), "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g = np.load(GOLDEN, allow_pickle=False)
    assert str(g["digest"]) == mg.input_digest(prob), "generator output changed: rerun tests/golden/make_golden.py"
    return g


def test_pairs_and_edges_bit_exact(ctx, prob, golden):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    dp = device_problem(prob)
    st = bf.bf_build_structure(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm))
    assert np.array_equal(st["pairs"].cpu().numpy(), golden["pairs"])
    assert np.array_equal(st["edges"].cpu().numpy(), golden["edges"])
    assert np.array_equal(st["free"].cpu().numpy(), golden["free"])


def test_sampled_pair_records(ctx, prob, golden):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    k = 3
    dp = device_problem(prob)
    res = bf.bf_eval_residuals(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm), gn_iter=k, records=True)
    rec = res["records"].cpu().numpy()
    pairs = golden["pairs"]
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(len(pairs), 64, replace=False))
    frames = {}
    for s in sample:
        i, j = pairs[s]
        for f in (i, j):
            if f not in frames:
                frames[f] = prepare_frame(prob.depth[f], prob.intensity[f], prob.intrinsics, prm)
        o = dense_pair_blocks(frames[i], frames[j], prob.init_poses[i], prob.init_poses[j], prob.intrinsics, prm,
                              prm.dense_weight(k))
        r = rec[s]
        assert r[29] == o["ngeo"] and r[30] == o["nphoto"], (i, j)
        if o["ngeo"] > 0:
            assert block_rel_err(r[:21], upper21(o["Hjj"])) < 1e-5, (i, j)
            assert abs(r[27] - o["Egeo"]) <= 1e-5 * o["Egeo"] + 1e-12


@pytest.mark.parametrize("accumulate,pcg_storage", [(0, 0), (2, 1)])
def test_one_step_parity_along_oracle_trajectory(ctx, prob, golden, accumulate, pcg_storage):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    dp = device_problem(prob, pairs=golden["pairs"])
    free = golden["free"]
    idx = (6 * free[:, None] + np.arange(6)[None, :]).ravel()
    worst = 0.0
    for k in range(prob.n_gn):
        X = golden["traj"][k]
        bf.bf_build_normal_equations(ctx, dp, poses_cuda(X),
                                     bf_params_from(prm, accumulate=accumulate, pcg_storage=pcg_storage),
                                     gn_iter=k, dense=False)
        delta, st = bf.bf_pcg_solve(ctx, prob.num_frames, prob.n_pcg)
        d = delta.cpu().numpy()[idx] - golden["steps"][k]
        err = float(np.abs(d).max())
        worst = max(worst, err)
        print(f"step {k}: max |d increment| {err:.2e} (|dx| {np.linalg.norm(golden['steps'][k]):.3f})", flush=True)
    assert worst < 1e-5


@pytest.mark.parametrize("pcg_storage,solve_kernel,accumulate", [(0, 0, 0), (1, 2, 0), (0, 3, 2)])
def test_gauss_newton_global200(ctx, prob, golden, pcg_storage, solve_kernel, accumulate):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    dp = device_problem(prob)
    out = bf.bf_gauss_newton(ctx, dp, poses_cuda(prob.init_poses),
                             bf_params_from(prm, pcg_storage=pcg_storage, solve_kernel=solve_kernel,
                                            accumulate=accumulate), trace=True)
    P = out["poses"].cpu().numpy()
    rot, tr = pose_errors(P, golden["poses"])
    e, er = out["energy"]["total"], float(golden["energy"][0])
    print(f"global200 storage={pcg_storage} kernel={solve_kernel} acc={accumulate}: pose err {rot:.3e} rad "
          f"{tr:.3e} m, energy rel err {abs(e - er) / er:.3e}", flush=True)
    assert abs(e - er) <= 1e-4 * er
    for k, t in enumerate(out["trace"]):
        assert abs(t[0] - golden["trace"][k][0]) <= 1e-4 * golden["trace"][k][0]
    assert rot < 2e-3 and tr < 2e-3


def test_one_step_jacobi_preconditioner(ctx, prob, golden):
    """One step at the initial poses with the scalar Jacobi preconditioner, against
    the oracle's (computed here: one assembly of the full system)."""
    from oracle.gn import Setup, build_system
    from oracle.system import inert_frames, reduce_system, solve_pcg
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg, preconditioner="jacobi")
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm, pairs=golden["pairs"])
    H, g, _, _ = build_system(s, prob.init_poses, prm.dense_weight(0))
    assert not inert_frames(H, s.free).any()
    Hr, gr, _ = reduce_system(H, g, s.free)
    ref, _ = solve_pcg(Hr, gr, prm.num_pcg, preconditioner="jacobi")
    dp = device_problem(prob, pairs=golden["pairs"])
    idx = (6 * s.free[:, None] + np.arange(6)[None, :]).ravel()
    for storage in (0, 1):
        bf.bf_build_normal_equations(ctx, dp, poses_cuda(prob.init_poses),
                                     bf_params_from(prm, pcg_storage=storage), gn_iter=0, dense=False)
        delta, st = bf.bf_pcg_solve(ctx, prob.num_frames, prob.n_pcg)
        err = float(np.abs(delta.cpu().numpy()[idx] - ref).max())
        print(f"global200 jacobi storage={storage}: max |d increment| {err:.2e}", flush=True)
        assert err < 1e-5
