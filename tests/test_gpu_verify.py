"""Dense two-sided verification (paper Sec. 4.1.1) through bf_verify_pairs against
oracle/verify.py, whose association decisions are FP64: per direction the
association count equal to the oracle's up to the candidates the oracle flags as
within binary32 rounding of a threshold (``near``), the error sum within 1e-5
relative when none is near and otherwise within near * tau_dist (each such
candidate moves the sum by less than tau_dist), validity identical unless a near
candidate can move a pair across its count or mean-error threshold; on every
pair of the 11-frame chunk at the initial and at misaligned poses, and on a
sample of 200-keyframe pairs."""
import numpy as np
import pytest
import torch

from oracle import Params
from oracle.verify import verify_pairs
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


def _check(ctx, prob, pairs, poses):
    prm = Params()
    ref_st, ref_ok, near = verify_pairs(prob.depth, prob.intensity, prob.intrinsics, pairs, poses, prm)
    st, ok = bf.bf_verify_pairs(ctx, device_problem(prob), torch.as_tensor(np.asarray(pairs, np.int32)).cuda(),
                                poses_cuda(poses), bf_params_from(prm))
    st, ok = st.cpu().numpy(), ok.cpu().numpy()
    n_got, n_ref = st[:, [1, 3]], ref_st[:, [1, 3]]
    e_got, e_ref = st[:, [0, 2]], ref_st[:, [0, 2]]
    assert np.all(np.abs(n_got - n_ref) <= near)
    assert np.all(np.abs(e_got - e_ref) <= 1e-5 * np.maximum(e_ref, 1e-3) + near * prm.tau_dist)
    # validity: equal wherever no near candidate can move the pair across a threshold
    min_count = 0.02 * prob.width * prob.height
    with np.errstate(divide="ignore", invalid="ignore"):
        lo_n, hi_n = n_ref - near, n_ref + near
        undecided = ((near > 0) & ((lo_n < min_count) & (hi_n >= min_count)
                                   | (np.abs(e_ref / np.maximum(n_ref, 1) - 0.075) <=
                                      near * prm.tau_dist / np.maximum(lo_n, 1)))).any(axis=1)
    assert np.array_equal(ok[~undecided], ref_ok[~undecided])
    print(f"verify: {int(near.sum())} near candidates over {len(pairs)} pairs, count differences "
          f"{int(np.abs(n_got - n_ref).sum())}, {int(undecided.sum())} pairs undecided", flush=True)
    return ref_ok


def test_verify_chunk(ctx):
    prob = make_problem(0)
    F = prob.num_frames
    pairs = [(i, j) for i in range(F) for j in range(i + 1, F)]
    ok0 = _check(ctx, prob, pairs, prob.gt_poses)
    bad = prob.gt_poses.copy()
    bad[5, :3, 3] += np.array([0.25, 0.0, 0.25])
    ok1 = _check(ctx, prob, pairs + [(5, 2)], bad)
    print(f"chunk: {ok0.sum()}/{len(pairs)} valid at ground truth, {ok1.sum()} with frame 5 moved 35 cm", flush=True)
    assert ok0.sum() > ok1[:len(pairs)].sum()


def test_verify_global200_sample(ctx):
    prob = make_problem(1)
    rng = np.random.default_rng(3)
    i = rng.integers(0, prob.num_frames - 1, 40)
    j = np.minimum(i + rng.integers(1, 6, 40), prob.num_frames - 1)
    pairs = [(int(a), int(b)) for a, b in zip(i, j) if a != b]
    _check(ctx, prob, pairs, prob.init_poses)
