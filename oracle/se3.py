"""Rigid transforms and the SE(3) exponential (paper Sec. 4.3: each 4x4 pose is
parameterised by matrix exponentials of skew-symmetric generators, 3 rotation
and 3 translation parameters).

A twist is xi = (omega, v) and Exp(xi) is the matrix exponential of
[[omega]_x, v; 0, 0], written in closed form (Rodrigues' formula for the
rotation and the matching left-Jacobian V for the translation).  Poses are
updated by right multiplication, T <- T Exp(xi).
"""
import numpy as np


def hat(w):
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_se3(xi):
    xi = np.asarray(xi, np.float64)
    w, v = xi[:3], xi[3:]
    th2 = float(w @ w)
    th = np.sqrt(th2)
    W = hat(w)
    W2 = W @ W
    if th < 1e-2:
        # Taylor series through th^6; the first omitted terms are below 1e-21.
        t4 = th2 * th2
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t4 * th2 / 5040.0
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t4 * th2 / 40320.0
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t4 * th2 / 362880.0
    else:
        A = np.sin(th) / th
        B = (1.0 - np.cos(th)) / th2
        C = (th - np.sin(th)) / (th2 * th)
    R = np.eye(3) + A * W + B * W2
    V = np.eye(3) + B * W + C * W2
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ v
    return T


def inv(T):
    R, t = T[:3, :3], T[:3, 3]
    Ti = np.eye(4)
    Ti[:3, :3] = R.T
    Ti[:3, 3] = -R.T @ t
    return Ti


def adjoint(T):
    """Ad(T) for twists ordered (omega, v): Exp(Ad(T) xi) = T Exp(xi) T^-1."""
    R, t = T[:3, :3], T[:3, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[3:, :3] = hat(t) @ R
    A[3:, 3:] = R
    return A


def rotation_angle(R):
    """Angle of rotation R, accurate also for small angles (atan2 of sin and cos)."""
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    c = 0.5 * (np.trace(R) - 1.0)
    return float(np.arctan2(s, c))
