"""The allocation-free entry point bf_gauss_newton_noalloc against bf_gauss_newton,
through the C ABI: poses, energies and energy traces bitwise equal on calls in a
row with shrinking inputs (a 120-keyframe window of the 200-keyframe workload,
whose PCG runs in the replicated-vector kernel with its exchange tags in the
scratch array, then the 11-frame chunk, then a 6-frame chunk); a problem whose
workspace exceeds the scratch array is refused with BF_ERR_OUT_OF_MEMORY, and the
entry point works as before afterwards."""
import numpy as np
import pytest
import torch

from synth import make_chunk, make_problem
from synth.problems import window

from gpu_helpers import device_problem, poses_cuda

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


def _same(ctx, pr, label):
    dp = device_problem(pr)
    init = poses_cuda(pr.init_poses)
    p = bf.bf_params_default(num_gn=pr.n_gn, num_pcg=pr.n_pcg, dense_threads=256)
    ref = bf.bf_gauss_newton(ctx, dp, init, p, trace=True)
    out = torch.full_like(init, float("nan"))
    got = bf.bf_gauss_newton_noalloc(ctx, dp, init, p, out_poses=out, trace=True)
    print(f"{label}: {pr.num_frames} frames, energy {got['energy']['total']:.9g} "
          f"(allocating entry point {ref['energy']['total']:.9g})", flush=True)
    assert torch.equal(out, ref["poses"])
    assert got["energy"] == ref["energy"]
    assert got["trace"] == ref["trace"]
    assert torch.equal(init, poses_cuda(pr.init_poses))


def test_noalloc_equals_allocating_entry_point(ctx):
    big = window(make_problem(1), 40, 120)
    _same(ctx, big, "120-keyframe window")
    _same(ctx, make_problem(0), "11-frame chunk")
    _same(ctx, make_chunk(num_frames=6, seed_offset=31), "6-frame chunk")


def test_noalloc_refuses_beyond_scratch(ctx):
    F, H, W = 1000, 60, 80      # 1000 frames of prepared images alone need 96 MB
    depth = torch.full((F, H, W), 2.0, dtype=torch.float32, device="cuda")
    inten = torch.full((F, H, W), 0.5, dtype=torch.float32, device="cuda")
    dp = bf.DeviceProblem(depth, inten, (72.0, 72.0, 40.0, 30.0, W, H))
    init = torch.eye(4, dtype=torch.float64, device="cuda").repeat(F, 1, 1).contiguous()
    p = bf.bf_params_default(num_gn=1, num_pcg=2, dense_threads=256)
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton_noalloc(ctx, dp, init, p, out_poses=torch.empty_like(init))
    assert e.value.status == bf.BF_ERR_OUT_OF_MEMORY and "MiB" in str(e.value)
    p0 = bf.bf_params_default(dense_threads=0)
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton_noalloc(ctx, dp, init, p0, out_poses=torch.empty_like(init))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    p1 = bf.bf_params_default(dense_threads=256, pcg_threads=-1)  # timing would create events
    with pytest.raises(bf.BFError) as e:
        bf.bf_gauss_newton_noalloc(ctx, dp, init, p1, out_poses=torch.empty_like(init))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    _same(ctx, make_chunk(num_frames=5, seed_offset=32), "5-frame chunk after a refusal")
