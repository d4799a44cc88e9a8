"""Error paths and the normal-equation systems through the C ABI.

* A non-finite pose or correspondence point: BF_ERR_NONFINITE, outputs untouched.
* A frame whose only constraint is one correspondence (a rank-3 diagonal block):
  BF_ERR_NOT_PD from the solve, as the oracle's Cholesky fails on it.
* A PCG kernel whose wait for its other workgroups gives up: forced from the host
  with a spin limit of one poll on the kernels' own bounded waits (every kernel
  still exits normally), BF_ERR_DEVICE, outputs untouched; the next solve with
  the default limit is bitwise the solve of a fresh context.
* Systems: two systems of one context built at different poses and solved in the
  other order give bitwise the results of solving each right after its build (no
  "last system" state); a system is refused by another context and before it is
  built."""
import numpy as np
import pytest
import torch

from oracle import Params
from oracle.gn import solve
from oracle.system import NotPositiveDefinite
from oracle.se3 import exp_se3
from synth import make_problem
from synth.problems import window

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


@pytest.fixture(scope="module")
def chunk():
    return make_problem(0)


def _solve_expect(ctx, pr, poses, params, status):
    dp = device_problem(pr)
    out = torch.full((pr.num_frames, 4, 4), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton(ctx, dp, poses, params, out_poses=out)
    assert e.value.status == status, str(e.value)
    assert bool((out == -7.0).all())
    return str(e.value)


def test_nonfinite_pose(ctx, chunk):
    poses = chunk.init_poses.copy()
    poses[4, 1, 3] = np.nan
    msg = _solve_expect(ctx, chunk, poses_cuda(poses), bf.bf_params_default(num_gn=2), bf.BF_ERR_NONFINITE)
    print("nan pose:", msg, flush=True)


def test_nonfinite_point(ctx, chunk):
    pr = make_problem(0)
    pr.corr_p = pr.corr_p.copy()
    pr.corr_p[17, 2] = np.inf
    msg = _solve_expect(ctx, pr, poses_cuda(pr.init_poses), bf.bf_params_default(num_gn=2), bf.BF_ERR_NONFINITE)
    print("inf point:", msg, flush=True)


def test_singular_diagonal_block(ctx):
    """Sparse term only; frame 3 keeps a single correspondence, so its diagonal
    block A_p^T A_p has rank 3."""
    pr = make_problem(0)
    touch = (pr.corr_i == 3) | (pr.corr_j == 3)
    keep = ~touch
    keep[np.flatnonzero(touch)[0]] = True
    pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q = (pr.corr_i[keep], pr.corr_j[keep], pr.corr_p[keep],
                                                  pr.corr_q[keep])
    prm = Params(num_gn=2, num_pcg=10, use_dense=False)
    with pytest.raises(NotPositiveDefinite):
        solve(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q, pr.init_poses,
              prm, linear="cholesky")
    for kernel in (0, 2, 5):
        msg = _solve_expect(ctx, pr, poses_cuda(pr.init_poses), bf_params_from(prm, solve_kernel=kernel),
                            bf.BF_ERR_NOT_PD)
    print("singular block:", msg, flush=True)


@pytest.mark.parametrize("solve_kernel", [3, 2, 5])
def test_pcg_wait_gives_up(ctx, solve_kernel):
    """A 120-keyframe window (PCG in the replicated-vector kernel, the cooperative
    one or the distributed-vector one): one poll per wait, then BF_ERR_DEVICE; afterwards a solve with
    the default limit equals a fresh context's."""
    pr = window(make_problem(1), 40, 120)
    dp = device_problem(pr)
    init = poses_cuda(pr.init_poses)
    p_fail = bf.bf_params_default(num_gn=2, num_pcg=20, dense_threads=256, solve_kernel=solve_kernel,
                                  pcg_spin_limit=1)
    msg = _solve_expect(ctx, pr, init, p_fail, bf.BF_ERR_DEVICE)
    p_ok = bf.bf_params_default(num_gn=2, num_pcg=20, dense_threads=256, solve_kernel=solve_kernel)
    got = bf.bf_gauss_newton(ctx, dp, init, p_ok)
    fresh = bf.Context()
    try:
        ref = bf.bf_gauss_newton(fresh, dp, init, p_ok)
    finally:
        fresh.close()
    print(f"kernel {solve_kernel}: {msg}; energy after recovery {got['energy']['total']:.9g}", flush=True)
    assert torch.equal(got["poses"], ref["poses"]) and got["energy"] == ref["energy"]


def test_systems_have_no_shared_state(ctx, chunk):
    dp = device_problem(chunk)
    p = bf.bf_params_default(num_gn=5, num_pcg=10)
    X0 = chunk.init_poses.copy()
    X1 = chunk.init_poses.copy()
    for f in range(1, chunk.num_frames):
        X1[f] = X1[f] @ exp_se3([0.004, -0.003, 0.002, 0.01, 0.0, -0.01])
    F = chunk.num_frames
    a = bf.bf_build_normal_equations(ctx, dp, poses_cuda(X0), p, gn_iter=1, dense=False)
    da_first, _ = bf.bf_pcg_solve(ctx, a["system"], F, 10)
    b = bf.bf_build_normal_equations(ctx, dp, poses_cuda(X1), p, gn_iter=3, dense=False)
    db_first, _ = bf.bf_pcg_solve(ctx, b["system"], F, 10)
    # the other order, after both builds
    db, _ = bf.bf_pcg_solve(ctx, b["system"], F, 10)
    da, _ = bf.bf_pcg_solve(ctx, a["system"], F, 10)
    assert torch.equal(da, da_first) and torch.equal(db, db_first)
    assert not torch.equal(da, db)
    Ha, ga, _ = bf.bf_system_export(ctx, a["system"], F)
    a2 = bf.bf_build_normal_equations(ctx, dp, poses_cuda(X0), p, gn_iter=1, dense=True)
    assert torch.equal(Ha, a2["H"]) and torch.equal(ga, a2["g"])
    # a system belongs to its context, and must be built before use
    other = bf.Context()
    try:
        with pytest.raises(bf.BFError) as e:
            bf.bf_pcg_solve(other, a["system"], F, 10)
        assert e.value.status == bf.BF_ERR_INVALID_ARG
        empty = bf.System(other)
        with pytest.raises(bf.BFError) as e:
            bf.bf_pcg_solve(other, empty, F, 10)
        assert e.value.status == bf.BF_ERR_INVALID_ARG
    finally:
        other.close()
    for y in (a, b, a2):
        y["system"].close()
