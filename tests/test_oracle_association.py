"""Pins of the dense association rule (paper Sec. 4.3: projections that leave the
frame are ignored, ICP-like distance and normal pruning; the readings of the
nearest-pixel lookup, the thresholds and the photometric footprint).

Hand-built frames with dyadic intrinsics and poses, so that every projection below
is exact in FP64, put each decision of the rule exactly on, or just on either side
of, its threshold:

* nearest pixel floor(u + 1/2): ties go up, at u = x + 1/2 and at u = x - 1/2
  (a floor, a round-half-even or a ties-down rule each fail one of the two), and
  the geometric residual shows which target pixel was read;
* the nearest pixel must lie in [0, W-1] x [0, H-1] (u = -1/2 is in, u = W - 1/2 out);
* the bilinear footprint floor(u) must lie in [0, W-2] x [0, H-2] (u = W - 7/8 in,
  u = W - 1 + 1/8 out), with every tap valid here so only the bound decides;
* in front of the camera: c_z > 0 (c_z = 0 and c_z < 0 rejected);
* |c - q| < tau_dist and m . N_j > tau_normal, both strict, each tested below, at
  and above its threshold;
* decisions on a threshold are flagged as near (within binary32 rounding), decisions
  far from every threshold are not.
"""
import numpy as np
import pytest

from oracle import Params
from oracle.frames import FrameData
from oracle.terms import associate, dense_terms, near_decisions

FX, CX, CY, W, H = 64.0, 8.0, 6.0, 16, 12
INTR = (FX, FX, CX, CY, W, H)


def frame(depth, normal=(0.0, 0.0, -1.0), grad=0.25):
    """A hand-built frame: positions back-projected from `depth` (scalar or [H,W]),
    one normal everywhere, every pixel valid (the border too, so that only the
    association rule decides)."""
    D = np.broadcast_to(np.asarray(depth, np.float64), (H, W))
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    P = np.stack([D * (xs - CX) / FX, D * (ys - CY) / FX, D], -1)
    N = np.broadcast_to(np.asarray(normal, np.float64), (H, W, 3)).copy()
    ones = np.ones((H, W), bool)
    return FrameData(P=P, N=N, G=np.full((H, W), grad), depth_ok=ones, normal_ok=ones.copy(), grad_ok=ones,
                     N_sigma=np.zeros((H, W)), flip_margin=np.full((H, W), np.inf))


def grid():
    ys, xs = np.mgrid[0:H, 0:W]
    return xs.ravel(), ys.ravel()


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("sign", [1, -1])
def test_nearest_pixel_ties_go_up(axis, sign):
    """A shift of half a pixel along x (or y): u = x + sign/2 exactly.  The nearest
    pixel is floor(u + 1/2): x + 1 for +1/2 and x for -1/2.  The target depth grows
    by 1/1024 per column (row), so the geometric residual m.(c - q) = D_j(xh, yh) - 2
    tells which pixel was read."""
    src = frame(2.0)
    xs, ys = grid()
    ramp = (np.arange(W)[None, :] if axis == 0 else np.arange(H)[:, None]) / 1024.0
    dst = frame(2.0 + ramp * np.ones((H, W)))
    t = np.zeros(3)
    t[axis] = sign * 2.0 / (2 * FX)          # c = d + t moves the projection by sign/2 px
    a = associate(src, dst, np.eye(3), t, INTR, Params())
    coord = xs if axis == 0 else ys
    lim = W if axis == 0 else H
    expect = coord + (1 if sign > 0 else 0)
    inside = expect <= lim - 1
    got = a["xh"] if axis == 0 else a["yh"]
    assert np.array_equal(a["geo"], inside)
    assert np.array_equal(got[inside], expect[inside])
    other = a["yh"] if axis == 0 else a["xh"]
    assert np.array_equal(other[inside], (ys if axis == 0 else xs)[inside])
    # u = -1/2 (pixel 0 shifted down) is inside: its nearest pixel is 0
    if sign < 0:
        assert a["geo"][coord == 0].all() and (got[coord == 0] == 0).all()
    # the residual reads the chosen target pixel
    terms = dense_terms(src, dst, np.eye(4), _pose(t), INTR, Params())
    assert np.allclose(terms["rg"], expect[inside] / 1024.0, rtol=0, atol=1e-13)
    # every one of these decisions sits on a tie: all flagged as within rounding
    near_geo, _ = near_decisions(a)
    assert near_geo[a["src_ok"]].all()


def _pose(t, R=np.eye(3)):
    """Pose T_j with T_j^-1 T_i = (R, t) when T_i = I."""
    T = np.eye(4)
    T[:3, :3] = R.T
    T[:3, 3] = -R.T @ t
    return T


@pytest.mark.parametrize("axis", [0, 1])
def test_bilinear_footprint_bound(axis):
    """u = x + 1/8: the nearest pixel is x (inside up to the last column) and the
    footprint floor(u) = x must be at most W - 2: the last column associates
    geometrically but not photometrically; every other pixel does both (all taps
    valid).  A shift of -1/8 puts floor(u) = x - 1 below 0 in the first column.
    Along the other axis the projection is integral, v = y, so its last row is out
    of the footprint in both cases."""
    src, dst = frame(2.0), frame(2.0)
    xs, ys = grid()
    coord, other = (xs, ys) if axis == 0 else (ys, xs)
    lim, olim = (W, H) if axis == 0 else (H, W)
    for sign in (1, -1):
        t = np.zeros(3)
        t[axis] = sign * 2.0 / (8 * FX)
        a = associate(src, dst, np.eye(3), t, INTR, Params())
        assert a["geo"].all()
        expect_photo = ((coord <= lim - 2) if sign > 0 else (coord >= 1)) & (other <= olim - 2)
        assert np.array_equal(a["photo"], expect_photo)
        # nearest-pixel choices are 1/8 px from a tie: not near; the footprint of the
        # integral coordinate sits on an integer, so those are near
        near_geo, near_ph = near_decisions(a)
        assert not near_geo.any() and near_ph.all()


def test_front_of_camera():
    """A half turn about the y axis puts the source points behind camera j (c_z = -2)
    while their projections land inside the image; with a distance threshold that
    cannot reject them and target normals facing the rotated source normals, only
    c_z > 0 decides: rejected at c_z = -2 and at c_z = 0, accepted at c_z = +2."""
    R = np.diag([-1.0, 1.0, -1.0])
    src = frame(2.0)
    dst = frame(2.0, normal=(0.0, 0.0, 1.0))
    prm = Params(tau_dist=100.0)
    xs, ys = grid()
    for tz, expect in ((0.0, False), (2.0, False), (4.0, True)):
        a = associate(src, dst, R, np.array([0.0, 0.0, tz]), INTR, prm)
        assert (a["m_front"] == tz - 2.0).all()
        if expect:
            # u = 2 cx - x: column 0 lands on u = W, outside
            assert np.array_equal(a["geo"], xs >= 1)
            assert np.array_equal(a["xh"][xs >= 1], 2 * int(CX) - xs[xs >= 1])
        else:
            assert not a["geo"].any()


def test_distance_threshold_is_strict():
    """Fronto-parallel planes at depth 2 (source) and D (target), identity pose: at the
    principal point |c - q| = D - 2 exactly, elsewhere it is larger.  With
    tau_dist = 1/8: D - 2 just below 1/8 associates, exactly 1/8 and just above do
    not; the decision at equality is flagged as near."""
    src = frame(2.0)
    pp = (np.arange(H * W) == int(CY) * W + int(CX))
    prm = Params(tau_dist=0.125)
    for D, expect in ((2.125 - 2.0 ** -30, True), (2.125, False), (2.125 + 2.0 ** -30, False)):
        a = associate(src, frame(D), np.eye(3), np.zeros(3), INTR, prm)
        assert a["geo"][pp][0] == expect
        assert not a["geo"][~pp].any()
        near_geo, _ = near_decisions(a)
        assert near_geo[pp][0]
    # well inside the threshold: every pixel associates and none is near
    a = associate(src, frame(2.0 + 2.0 ** -10), np.eye(3), np.zeros(3), INTR, prm)
    assert a["geo"].all() and not near_decisions(a)[0].any()


def test_normal_threshold_is_strict():
    """Source normals (0, 0, -1), target normals tilted so that m . N_j = 7/8 exactly:
    tau_normal = 7/8 rejects (strict), just below accepts, just above rejects."""
    c = 0.875
    src = frame(2.0)
    dst = frame(2.0, normal=(0.0, -np.sqrt(1.0 - c * c), -c))
    for tau, expect in ((c - 1e-12, True), (c, False), (c + 1e-12, False)):
        a = associate(src, dst, np.eye(3), np.zeros(3), INTR, Params(tau_normal=tau))
        assert (a["geo"] == expect).all()
        assert near_decisions(a)[0].all()
    a = associate(src, dst, np.eye(3), np.zeros(3), INTR, Params(tau_normal=0.8))
    assert a["geo"].all() and not near_decisions(a)[0].any()
