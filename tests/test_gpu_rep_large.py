"""The replicated-vector PCG above the size where its block-Jacobi inverses fit in
LDS next to the vectors (they are then read from memory), and the
distributed-vector PCG: one Gauss-Newton step of a 400-keyframe and of an
800-keyframe problem of the serving workload's kind agrees with the cooperative
PCG kernel, which keeps nothing in LDS, within rounding (FP64 PCG storage: 400 keyframes, 528 B per frame do not fit in 128 KB;
FP32 storage: 800 keyframes, 264 B per frame do not)."""
import shutil
import tempfile

import numpy as np
import pytest
import torch

from oracle import Params

from gpu_helpers import bf_params_from, device_problem, pose_errors, poses_cuda

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


def _problem(n):
    from synth.dump import generate_in_child
    d = tempfile.mkdtemp(prefix=f"floor3_{n}_")
    try:
        return generate_in_child(f"floor3:{n}", d)
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("frames,pcg_storage,bound", [(400, 1, 1e-9), (800, 0, 1e-5)])
def test_one_step_replicated_vs_cooperative(ctx, frames, pcg_storage, bound):
    prob = _problem(frames)
    prm = Params(num_gn=1, num_pcg=20)
    dp = device_problem(prob)
    init = poses_cuda(prob.init_poses)
    out = {}
    for kernel in (3, 2, 5):
        out[kernel] = bf.bf_gauss_newton(ctx, dp, init, bf_params_from(prm, solve_kernel=kernel,
                                                                      pcg_storage=pcg_storage))
    step = pose_errors(out[2]["poses"].cpu().numpy(), prob.init_poses)
    for kernel, name in ((3, "replicated"), (5, "distributed")):
        rot, tr = pose_errors(out[kernel]["poses"].cpu().numpy(), out[2]["poses"].cpu().numpy())
        print(f"{frames} keyframes, storage {pcg_storage}: {name} vs cooperative {rot:.2e} rad {tr:.2e} m "
              f"(step {step[0]:.3f} rad {step[1]:.3f} m)", flush=True)
        assert rot < bound and tr < bound
        ek, e2 = out[kernel]["energy"]["total"], out[2]["energy"]["total"]
        assert abs(ek - e2) <= 1e-6 * e2
