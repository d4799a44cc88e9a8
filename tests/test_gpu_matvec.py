"""y = H x in the two representations of the sparse term (paper Sec. 4.4): the
assembled 6x6 blocks (from FP64 moments of the correspondences) and the paper's
matrix-free J^T (J x) over the correspondences.  Both against the oracle's dense H
(FP64), on the chunk and the 200-keyframe workloads; the timings are printed."""
import numpy as np
import pytest
import torch

from oracle import Params
from oracle.gn import Setup, build_system
from synth import make_problem

from gpu_helpers import bf_params_from, device_problem, poses_cuda

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.mark.parametrize("config", [0, 1])
def test_sparse_matvec_representations(ctx, config):
    prob = make_problem(config)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg, use_dense=False)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm)
    H, _, _, _ = build_system(s, prob.init_poses, prm.dense_weight(0))
    dp = device_problem(prob)
    y_sys = bf.bf_build_normal_equations(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm),
                                         dense=False)["system"]
    rng = np.random.default_rng(9)
    x = rng.normal(size=6 * prob.num_frames) * np.tile([0.01, 0.01, 0.01, 0.05, 0.05, 0.05], prob.num_frames)
    ref = H @ x
    xt = torch.as_tensor(x).cuda()
    y0, t0 = bf.bf_system_matvec(ctx, y_sys, dp, xt, 0)
    y1, t1 = bf.bf_system_matvec(ctx, y_sys, dp, xt, 1)
    y0, y1 = y0.cpu().numpy(), y1.cpu().numpy()
    e0 = np.abs(y0 - ref).max() / np.abs(ref).max()
    e1 = np.abs(y1 - ref).max() / np.abs(ref).max()
    print(f"config {config}: {len(prob.corr_i)} correspondences; blocks {t0:.1f} us (rel err {e0:.1e}), "
          f"matrix-free {t1:.1f} us (rel err {e1:.1e})", flush=True)
    assert e0 < 1e-10
    assert e1 < 1e-5


def test_matvec_with_dense_terms(ctx):
    prob = make_problem(0)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
              prob.init_poses, prm)
    H, _, _, _ = build_system(s, prob.init_poses, prm.dense_weight(2))
    dp = device_problem(prob)
    y_sys = bf.bf_build_normal_equations(ctx, dp, poses_cuda(prob.init_poses), bf_params_from(prm), gn_iter=2,
                                         dense=False)["system"]
    x = np.random.default_rng(10).normal(size=6 * prob.num_frames) * 0.01
    y0, _ = bf.bf_system_matvec(ctx, y_sys, dp, torch.as_tensor(x).cuda(), 0)
    ref = H @ x
    assert np.abs(y0.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    with pytest.raises(bf.BFError):
        bf.bf_system_matvec(ctx, y_sys, bf.DeviceProblem.from_numpy(prob.depth, prob.intensity, prob.intrinsics),
                            torch.as_tensor(x).cuda(), 1)
