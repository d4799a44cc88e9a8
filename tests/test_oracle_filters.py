"""Pins of the key-point and surface-area filter references (oracle/filters.py)."""
import numpy as np

from oracle.filters import condition_numbers, filter_pairs, kabsch, keypoint_filter, principal_area
from oracle.se3 import exp_se3


def _rigid(seed):
    rng = np.random.default_rng(seed)
    T = exp_se3(np.concatenate([rng.normal(size=3) * 0.4, rng.normal(size=3) * 0.5]))
    return T[:3, :3], T[:3, 3], rng


def test_kabsch_recovers_a_rigid_motion():
    R, t, rng = _rigid(1)
    P = rng.uniform(-1, 1, size=(20, 3))
    R2, t2 = kabsch(P, P @ R.T + t)
    assert np.abs(R2 - R).max() < 1e-12 and np.abs(t2 - t).max() < 1e-12
    assert abs(np.linalg.det(R2) - 1.0) < 1e-12


def test_condition_numbers_closed_forms():
    # axis-aligned box of points with extents 1, 0.5, 0.1 along x, y, z: covariance
    # eigenvalues in ratio 1 : 0.25 : 0.01 -> ratio of the two largest = 4
    g = np.array([[x, y, z] for x in (-1, 1) for y in (-0.5, 0.5) for z in (-0.1, 0.1)], float)
    cp, cq, cx = condition_numbers(g, g)
    assert abs(cp - 4.0) < 1e-12 and abs(cq - 4.0) < 1e-12 and abs(cx - 4.0) < 1e-12
    line = np.outer(np.linspace(-1, 1, 9), [0.3, 0.4, 0.5])
    assert max(condition_numbers(line, line)) > 1e12
    # the plain definition (largest / smallest): 1 / 0.01 = 100 for the box (the
    # eigenvalues of the covariance of a centred +-a box are a^2), a rotated copy alike
    cp, cq, cx = condition_numbers(g, g, mode=1)
    assert abs(cp - 100.0) < 1e-9 and abs(cq - 100.0) < 1e-9 and abs(cx - 100.0) < 1e-9
    R, t, _ = _rigid(9)
    assert abs(max(condition_numbers(g @ R.T + t, g, mode=1)) - 100.0) < 1e-8
    plane = g.copy()
    plane[:, 2] = 0.0
    assert condition_numbers(plane, plane, mode=0)[0] == 4.0 and condition_numbers(plane, plane, mode=1)[0] == np.inf


def test_plain_condition_rejects_every_set():
    """With the largest / smallest ratio the incremental filter, whose checks start
    at three members, can never pass: three points are always coplanar, so the
    smallest covariance eigenvalue is 0 and the third member is removed again --
    a planar set and a well spread set alike are discarded, while the second-largest
    reading keeps both."""
    R, t, rng = _rigid(6)
    plane = np.stack([rng.uniform(-1, 1, 30), rng.uniform(-1, 1, 30), np.zeros(30)], axis=1)
    P = rng.uniform(-1, 1, size=(30, 3))
    for X in (plane, P):
        assert len(keypoint_filter(X, X @ R.T + t, cond_mode=1)) == 0
        assert len(keypoint_filter(X, X @ R.T + t, cond_mode=0)) >= 25   # a nearly collinear start may lose one
    assert max(condition_numbers(P[:3], P[:3] @ R.T + t, mode=1)) > 1e12


def test_clean_correspondences_all_kept_and_outliers_removed():
    R, t, rng = _rigid(2)
    P = rng.uniform(-1.5, 1.5, size=(40, 3))
    Q = P @ R.T + t + rng.normal(scale=0.002, size=P.shape)
    assert np.array_equal(keypoint_filter(P, Q), np.arange(40))
    bad = [5, 17, 30]
    Q2 = Q.copy()
    Q2[bad] += rng.normal(scale=0.5, size=(3, 3))
    assert np.array_equal(keypoint_filter(P, Q2), np.setdiff1d(np.arange(40), bad))


def test_degenerate_sets_discarded_planar_kept():
    R, t, rng = _rigid(3)
    s = np.linspace(-1, 1, 12)
    line = np.outer(s, [0.2, 0.7, -0.3]) + 0.5
    assert len(keypoint_filter(line, line @ R.T + t)) == 0
    plane = np.stack([rng.uniform(-1, 1, 30), rng.uniform(-1, 1, 30), np.zeros(30)], axis=1)
    assert len(keypoint_filter(plane, plane @ R.T + t)) == 30
    assert len(keypoint_filter(plane[:4], plane[:4] @ R.T + t)) == 0   # fewer than 5


def test_principal_area_closed_form():
    R, t, rng = _rigid(4)
    sq = np.array([[x, y, 0.0] for x in np.linspace(0, 0.8, 5) for y in np.linspace(0, 0.3, 4)])
    assert abs(principal_area(sq @ R.T + t) - 0.8 * 0.3) < 1e-12
    assert principal_area(np.outer(np.linspace(0, 1, 5), [1, 2, 3])) < 1e-12   # collinear: no area


def test_filter_pairs_area_and_grouping():
    R, t, rng = _rigid(5)
    big = rng.uniform(-1, 1, size=(30, 3))
    small = rng.uniform(-0.05, 0.05, size=(30, 3))   # area ~0.01 m^2 < 0.032
    ci = np.r_[np.zeros(30, int), np.full(30, 2)]
    cj = np.r_[np.ones(30, int), np.full(30, 1)]      # second pair given as (2, 1): points swapped
    p = np.r_[big, small @ R.T + t]
    q = np.r_[big @ R.T + t, small]
    keep = filter_pairs(ci, cj, p, q)
    assert keep[:30].all() and not keep[30:].any()
