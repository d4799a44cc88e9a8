"""Full-size parity on the 2000-keyframe floor workload (8 GN x 20 PCG, FP32 path,
automatic solve kernel; about 220k dense pair jobs, 10M correspondences, 11,994
unknowns), against the oracle's run stored in tests/golden/global2000_oracle.npz
(written by tests/golden/make_golden.py, which calls only the oracle):

* the dense pair set and the variables, bit-exact;
* energy and residual counts at the initial poses (energy within 1e-4 relative;
  the counts differ from the oracle's by at most the excused decisions, about
  one in a million here);
* the association masks of a sample of 2000 pair jobs at the initial poses,
  pixel by pixel against the oracle's FP64 decisions (mismatches only where the
  oracle flags a decision as within twice its binary32 rounding bound), and the
  records of 16 of them, computed by the oracle one pair at a time;
* one Gauss-Newton step at each of the oracle's 8 iterates: the increment within
  1e-5 (rad, m) of the oracle's in the mixed-precision configuration of this
  workload and with FP64 values, and on the all-FP32 path within the bound its
  arithmetic meets (printed; see the parameter list below);
* the full solve: the energies at the start of all 8 iterations within 1e-4
  relative of the oracle's.

The input is generated in a child process (parallel workers; this process holds a
GPU context and does not fork)."""
import os
import shutil
import tempfile

import numpy as np
import pytest
import torch

from oracle import Params
from oracle.frames import prepare_frame
from oracle.pairs import relative_pose64
from oracle.system import dense_pair_blocks
from oracle.terms import associate

from gpu_helpers import bf_params_from, block_rel_err, compare_masks, device_problem, poses_cuda, upper21

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "global2000_oracle.npz")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def prob():
    from synth.dump import generate_in_child
    d = tempfile.mkdtemp(prefix="global2000_")
    try:
        return generate_in_child(4, d)
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.fixture(scope="module")
def golden(prob):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(os.path.dirname(GOLDEN), "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g = np.load(GOLDEN, allow_pickle=False)
    assert str(g["digest"]) == mg.input_digest(prob), "generator output changed: rerun tests/golden/make_golden.py"
    return g


@pytest.fixture(scope="module")
def dp(prob):
    return device_problem(prob)


def test_pairs_and_variables_bit_exact(ctx, prob, golden, dp):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    st = bf.bf_build_structure(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm))
    assert np.array_equal(st["pairs"].cpu().numpy(), golden["pairs"])
    assert np.array_equal(st["free"].cpu().numpy(), golden["free"])


def test_energy_and_counts_at_init(ctx, prob, golden, dp):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    e = bf.bf_eval_residuals(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm), gn_iter=0)
    ref = golden["trace"][0]  # total, sparse, geo, photo, n_sparse, n_geo, n_photo
    print(f"global2000 energy at init {e['total']:.9g} vs {ref[0]:.9g}; counts geo {e['n_geo']} vs {int(ref[5])}, "
          f"photo {e['n_photo']} vs {int(ref[6])}", flush=True)
    assert e["n_sparse"] == int(ref[4])
    assert abs(e["n_geo"] - ref[5]) <= 1e-5 * ref[5] and abs(e["n_photo"] - ref[6]) <= 1e-5 * ref[6]
    for k, name in enumerate(("total", "sparse", "geo", "photo")):
        assert abs(e[name] - ref[k]) <= 1e-4 * ref[k], name


def test_sampled_masks_and_records(ctx, prob, golden, dp):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    res = bf.bf_eval_residuals(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm), gn_iter=0, records=True,
                               masks=True)
    pairs = golden["pairs"]
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(len(pairs), 2000, replace=False))
    masks = res["masks"][torch.as_tensor(sample).cuda()].cpu().numpy()
    rec = res["records"].cpu().numpy()
    del res
    frames = {}

    def fr(f):
        if f not in frames:
            frames[f] = prepare_frame(prob.depth[f], prob.intensity[f], prob.intrinsics, prm)
        return frames[f]

    tot = np.zeros(4, np.int64)
    differ = set()
    for n, s in enumerate(sample):
        i, j = pairs[s]
        R, t = relative_pose64(prob.init_poses[i], prob.init_poses[j])
        ug, up, eg, ep, same = compare_masks(masks[n], associate(fr(i), fr(j), R, t, prob.intrinsics, prm), prob.width)
        tot += (ug, up, eg, ep)
        if not same:
            differ.add(int(s))
    print(f"global2000 masks of {len(sample)} jobs: unexcused geo {tot[0]} photo {tot[1]}, excused geo {tot[2]} "
          f"photo {tot[3]} in {len(differ)} jobs", flush=True)
    assert tot[0] == 0 and tot[1] == 0
    for s in sample[::125]:
        i, j = pairs[s]
        o = dense_pair_blocks(fr(i), fr(j), prob.init_poses[i], prob.init_poses[j], prob.intrinsics, prm,
                              prm.dense_weight(0))
        r = rec[s]
        tol = 1e-2 if int(s) in differ else 1e-5
        if int(s) not in differ:
            assert r[29] == o["ngeo"] and r[30] == o["nphoto"], (i, j)
        if o["ngeo"] > 0:
            assert block_rel_err(r[:21], upper21(o["Hjj"])) < tol, (i, j)


# The FP32 path (FP32 values, lane sums, PCG matrix and vectors; FP64 dots and
# alpha/beta), the mixed-precision configuration of this workload (compensated FP32
# lane sums, FP64 PCG storage) and FP64 values.
SETTINGS = [(0, 0), (1, 1), (2, 1)]


@pytest.mark.parametrize("steps", [(0, 1), (2, 3), (4, 5), (6, 7)])
def test_one_step_parity_fixed_association(ctx, prob, golden, dp, steps):
    """At each of the oracle's 8 iterates (two per test), with the oracle's
    association of that iterate given to the kernels (all 220k jobs, computed in
    worker processes): the
    increment within 1e-5 (rad, m) of the oracle's in the mixed-precision setting
    and with FP64 values.  The all-FP32 path is held at the first two iterates to
    twice the error that binary32 storage of the PCG matrix and vectors alone
    causes on the oracle's own system (stored by make_golden.py: 5.8e-5 and 3.3e-6,
    this system is ill-conditioned), plus 1e-5; at the later iterates that storage
    error falls to 3e-7..1e-5, the same size as the FP32 lane sums' own error,
    which the storage model leaves out, so there the all-FP32 error is reported
    and not bounded."""
    from assoc_pool import oracle_association
    from gpu_helpers import fix_association
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    free = golden["free"]
    idx = (6 * free[:, None] + np.arange(6)[None, :]).ravel()
    dpp = device_problem(prob, pairs=golden["pairs"])
    for k in steps:
        fixed = oracle_association(prob, golden["pairs"], golden["traj"][k], prm)
        for accumulate, pcg_storage in SETTINGS:
            p = fix_association(bf_params_from(prm, accumulate=accumulate, pcg_storage=pcg_storage), fixed)
            ne = bf.bf_build_normal_equations(ctx, dpp, poses_cuda(golden["traj"][k]), p, gn_iter=k, dense=False)
            delta, st = bf.bf_pcg_solve(ctx, ne["system"], prob.num_frames, prob.n_pcg)
            ne["system"].close()
            err = float(np.abs(delta.cpu().numpy()[idx] - golden["steps"][k]).max())
            bound = 1e-5 if pcg_storage == 1 else 1e-5 + 2 * float(golden["fp32_storage_err"][k])
            print(f"global2000 step {k} accumulate={accumulate} storage={pcg_storage}, oracle's association: "
                  f"max |d increment| {err:.2e} (bound {bound:.1e}, max |increment| "
                  f"{np.abs(golden['steps'][k]).max():.3f})", flush=True)
            if pcg_storage == 1 or k < 2:
                assert err < bound
        del fixed
        torch.cuda.empty_cache()


def test_one_step_parity_decided(ctx, prob, golden, dp):
    """At each of the oracle's 8 iterates, the kernels deciding the association
    themselves: the increments of the three settings are reported beside the
    oracle's.  Decisions within binary32 rounding of a threshold (about one in 10^6)
    go either way, and this system carries one such pixel into the increment at up
    to ~2e-4 (the same in every value precision, so it is not arithmetic); the
    arithmetic is held to 1e-5 by the fixed-association test above.  Asserted here:
    frames without residuals are held by both, and every setting stays within 5e-4."""
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    free = golden["free"]
    idx = (6 * free[:, None] + np.arange(6)[None, :]).ravel()
    dpp = device_problem(prob, pairs=golden["pairs"])
    for accumulate, pcg_storage in SETTINGS:
        worst = 0.0
        for k in range(len(golden["steps"])):
            ne = bf.bf_build_normal_equations(ctx, dpp, poses_cuda(golden["traj"][k]),
                                              bf_params_from(prm, accumulate=accumulate, pcg_storage=pcg_storage),
                                              gn_iter=k, dense=False)
            delta, st = bf.bf_pcg_solve(ctx, ne["system"], prob.num_frames, prob.n_pcg)
            ne["system"].close()
            err = float(np.abs(delta.cpu().numpy()[idx] - golden["steps"][k]).max())
            print(f"global2000 accumulate={accumulate} storage={pcg_storage} step {k}: max |d increment| {err:.2e} "
                  f"(max |increment| {np.abs(golden['steps'][k]).max():.3f})", flush=True)
            worst = max(worst, err)
            held = free[golden["inert"][k]]
            assert not delta.cpu().numpy().reshape(-1, 6)[held].any()
        assert worst < 5e-4


def test_gauss_newton_trace(ctx, prob, golden, dp):
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    out = bf.bf_gauss_newton(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm), trace=True)
    for k in range(len(golden["trace"])):
        ref = golden["trace"][k][0]
        got = out["trace"][k][0]
        print(f"global2000 GN energy at iteration {k}: {got:.9g} vs oracle {ref:.9g}", flush=True)
        assert abs(got - ref) <= 1e-4 * ref
    assert np.isfinite(out["energy"]["total"]) and out["energy"]["total"] < out["trace"][0][0]
