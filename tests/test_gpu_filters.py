"""Key-point and surface-area filters (paper Sec. 4.1.1) through
bf_filter_correspondences against oracle/filters.py: the kept correspondences
bit-exact (same FP64 decisions; the two sides use different 3x3 eigen/SVD
routines, so only a decision within rounding of a threshold could differ), on
the 11-frame chunk (10 % outliers), on constructed pairs with gross outliers,
collinear and small-area sets, and on a sample of 200-keyframe pairs."""
import numpy as np
import pytest
import torch

from oracle.filters import filter_pairs
from oracle.se3 import exp_se3
from synth import make_problem

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


def _run(ctx, F, ci, cj, p, q, cond_mode=0):
    depth = np.zeros((F, 4, 4), np.float32)
    dp = bf.DeviceProblem.from_numpy(depth, depth, (2.0, 2.0, 2.0, 2.0, 4, 4), ci, cj, p, q)
    keep, kept = bf.bf_filter_correspondences(ctx, dp, cond_mode=cond_mode)
    keep = keep.cpu().numpy()
    assert kept == int(keep.sum())
    return keep


def test_filters_chunk(ctx):
    pr = make_problem(0)
    ref = filter_pairs(pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q)
    keep = _run(ctx, pr.num_frames, pr.corr_i, pr.corr_j, pr.corr_p, pr.corr_q)
    print(f"chunk: kept {keep.sum()} of {len(keep)} (oracle {ref.sum()}); outliers kept {(keep & pr.outlier).sum()}",
          flush=True)
    assert np.array_equal(keep, ref)


@pytest.mark.parametrize("cond_mode", [0, 1])
def test_filters_constructed(ctx, cond_mode):
    rng = np.random.default_rng(7)
    T = exp_se3(np.array([0.2, -0.1, 0.3, 0.4, 0.1, -0.2]))
    R, t = T[:3, :3], T[:3, 3]
    ci, cj, p, q = [], [], [], []

    def add(a, b, P, Q):
        ci.extend([a] * len(P)); cj.extend([b] * len(P)); p.extend(P); q.extend(Q)

    P = rng.uniform(-1, 1, (60, 3)); Q = P @ R.T + t + rng.normal(scale=0.003, size=P.shape)
    Q[[3, 20, 41, 59]] += rng.normal(scale=0.4, size=(4, 3))
    add(0, 1, P, Q)                                            # gross outliers among inliers
    L = np.outer(np.linspace(-1, 1, 20), [0.3, -0.5, 0.8]) + 0.2
    add(1, 2, L, L @ R.T + t)                                  # collinear: discarded
    S = rng.uniform(-0.05, 0.05, (30, 3))
    add(3, 2, S @ R.T + t, S)                                  # small area, given as (3, 2)
    Pl = np.stack([rng.uniform(-1, 1, 40), rng.uniform(-1, 1, 40), np.zeros(40)], 1)
    add(0, 3, Pl, Pl @ R.T + t)                                # planar: kept
    ci, cj = np.array(ci, np.int32), np.array(cj, np.int32)
    p, q = np.array(p, np.float32), np.array(q, np.float32)
    ref = filter_pairs(ci, cj, p, q, cond_mode=cond_mode)
    keep = _run(ctx, 4, ci, cj, p, q, cond_mode)
    assert np.array_equal(keep, ref)
    if cond_mode == 0:
        assert not keep[[3, 20, 41, 59]].any() and keep[:60].sum() >= 50
        assert not keep[60:110].any() and keep[110:].all()
    else:
        assert not keep.any()   # the plain reading discards every set (its checks start at three points)


@pytest.mark.parametrize("cond_mode", [0, 1])
def test_filters_global200_sample(ctx, cond_mode):
    pr = make_problem(1)
    lo, hi = np.minimum(pr.corr_i, pr.corr_j), np.maximum(pr.corr_i, pr.corr_j)
    keys = lo.astype(np.int64) * pr.num_frames + hi
    uk = np.unique(keys)
    pick = np.random.default_rng(1).choice(uk, 40, replace=False)
    m = np.isin(keys, pick)
    ci, cj, p, q = pr.corr_i[m], pr.corr_j[m], pr.corr_p[m], pr.corr_q[m]
    ref = filter_pairs(ci, cj, p, q, cond_mode=cond_mode)
    keep = _run(ctx, pr.num_frames, ci, cj, p, q, cond_mode)
    print(f"global200 sample, condition mode {cond_mode}: kept {keep.sum()} of {len(keep)}, outliers kept "
          f"{(keep & pr.outlier[m]).sum()} of {pr.outlier[m].sum()}", flush=True)
    assert np.array_equal(keep, ref)
