"""Pins of the oracle's pose exponential and per-frame preparation against
closed forms and library routines (not against the oracle itself)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import Params
from oracle.frames import prepare_frame
from oracle.se3 import adjoint, exp_se3, hat, inv, rotation_angle


def _twist_matrix(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = hat(xi[:3])
    M[:3, 3] = xi[3:]
    return M


def test_exp_matches_expm():
    rng = np.random.default_rng(1)
    for _ in range(200):
        w = rng.normal(size=3)
        w *= rng.uniform(0, np.pi - 0.1) / np.linalg.norm(w)
        xi = np.concatenate([w, rng.normal(size=3)])
        assert np.abs(exp_se3(xi) - scipy.linalg.expm(_twist_matrix(xi))).max() < 5e-14


@pytest.mark.parametrize("theta", [0.0, 1e-12, 1e-9, 1e-4, 9.99e-3, 1e-2, 1.001e-2, 0.1])
def test_exp_small_angle_continuous(theta):
    rng = np.random.default_rng(2)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    xi = np.concatenate([theta * a, [0.3, -0.2, 0.5]])
    assert np.abs(exp_se3(xi) - scipy.linalg.expm(_twist_matrix(xi))).max() < 2e-15


def test_exp_inverse_and_adjoint():
    rng = np.random.default_rng(3)
    for _ in range(50):
        xi = rng.normal(size=6)
        assert np.abs(exp_se3(xi) @ exp_se3(-xi) - np.eye(4)).max() < 1e-13
        T = exp_se3(rng.normal(size=6))
        # Exp(Ad(T) xi) = T Exp(xi) T^-1
        assert np.abs(exp_se3(adjoint(T) @ xi) - T @ exp_se3(xi) @ inv(T)).max() < 1e-12


def test_rotation_angle():
    for th in [1e-9, 1e-5, 0.3, 3.0]:
        assert abs(rotation_angle(exp_se3([0, 0, th, 0, 0, 0])[:3, :3]) - th) < 1e-15 + 1e-13 * th


# ----------------------------------------------------------------------------- frames

INTR = (72.0, 72.0, 40.0, 30.0, 80, 60)


def _plane_depth(n, d, intr):
    fx, fy, cx, cy, W, H = intr
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    ray = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], -1)
    return (d / (ray @ n)).astype(np.float32)


def test_planar_normals():
    """Normals of a tilted plane equal the analytic plane normal, oriented to the camera.
    Tolerance: FP32 depth quantisation moves points off the plane by <= 2^-24 z,
    which tilts a normal built from 2-pixel differences by < 1e-5."""
    n = np.array([0.2, -0.3, -1.0])
    n /= np.linalg.norm(n)
    D = _plane_depth(n, -2.0, INTR)
    fd = prepare_frame(D, np.zeros_like(D), INTR, Params())
    ok = fd.normal_ok
    assert ok[1:-1, 1:-1].all() and not ok[0].any() and not ok[-1].any() and not ok[:, 0].any()
    assert np.abs(fd.N[ok] - n).max() < 1e-5
    # the binary32 rounding bound of a normal covers the tilt that the FP32
    # quantisation of the depth itself causes (the same first-order effect)
    assert (np.linalg.norm(fd.N[ok] - n, axis=1) <= fd.N_sigma[ok]).all()
    assert fd.N_sigma[ok].max() < 1e-4 and (fd.flip_margin[ok] > 0.5).all()
    assert (np.einsum("ka,ka->k", fd.N[ok], fd.P[ok]) < 0).all()
    # P is the back-projection
    fx, fy, cx, cy, W, H = INTR
    assert np.allclose(fd.P[10, 20], D[10, 20] * np.array([(20 - cx) / fx, (10 - cy) / fy, 1.0]), rtol=0, atol=1e-15)


def test_gradient_of_linear_ramp():
    fx, fy, cx, cy, W, H = INTR
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    L = (xs / 64.0 + ys / 128.0 + 0.25).astype(np.float32)   # dyadic, exact in FP32
    fd = prepare_frame(np.full((H, W), 2.0, np.float32), L, INTR, Params())
    g = fd.G[fd.grad_ok]
    assert fd.grad_ok[1:-1, 1:-1].all() and not fd.grad_ok[0].any()
    assert np.abs(g - np.hypot(1 / 64.0, 1 / 128.0)).max() < 1e-15


def test_validity_masks_small_image():
    intr = (4.0, 4.0, 2.0, 2.0, 5, 5)
    D = np.full((5, 5), 2.0, np.float32)
    D[2, 3] = 0.0           # invalid depth
    D[1, 1] = 20.0          # beyond depth_max
    L = np.full((5, 5), 0.5, np.float32)
    L[3, 2] = np.nan
    fd = prepare_frame(D, L, intr, Params())
    dok = np.ones((5, 5), bool)
    dok[2, 3] = dok[1, 1] = False
    assert (fd.depth_ok == dok).all()
    exp_n = np.zeros((5, 5), bool)
    for y in range(1, 4):
        for x in range(1, 4):
            exp_n[y, x] = dok[y, x] and dok[y, x - 1] and dok[y, x + 1] and dok[y - 1, x] and dok[y + 1, x]
    assert (fd.normal_ok == exp_n).all()
    lok = np.isfinite(L)
    exp_g = np.zeros((5, 5), bool)
    for y in range(1, 4):
        for x in range(1, 4):
            exp_g[y, x] = lok[y, x] and lok[y, x - 1] and lok[y, x + 1] and lok[y - 1, x] and lok[y + 1, x]
    assert (fd.grad_ok == exp_g).all()
    assert np.isnan(fd.N[~exp_n]).all() and np.isnan(fd.G[~exp_g]).all()
