"""Camera trajectories and rigid-motion helpers for the synthetic generator.

Poses are 4x4 camera-to-world matrices.  Camera axes: z forward, x right,
y down; world: z up.  Rotations here are built from unit quaternions (an
input-synthesis convention of this module, independent of the solver's own
pose parameterisation).
"""
from __future__ import annotations

import numpy as np

UP = np.array([0.0, 0.0, 1.0])


def quat_rot(axis, angle):
    """Rotation matrix of `angle` radians about `axis`, via the unit quaternion."""
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    w = np.cos(0.5 * angle)
    x, y, z = np.sin(0.5 * angle) * axis
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def look_rotation(yaw, pitch):
    """Camera-to-world rotation for a camera looking along (yaw, pitch), no roll."""
    fwd = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
    right = np.cross(fwd, UP)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd], axis=1)


def make_pose(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def rigid_inv(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def perturbation(rng, rot_deg, trans_m):
    """Rigid motion rotating by exactly `rot_deg` about a uniform axis and translating
    by exactly `trans_m` in a uniform direction."""
    return make_pose(quat_rot(random_unit(rng), np.deg2rad(rot_deg)), trans_m * random_unit(rng))


def random_walk(rng, n, box, step_m=0.02, step_deg=1.0, wall_margin=0.5):
    """Smooth random walk inside box=(x0,x1,y0,y1): `step_m` translation and
    `step_deg` rotation per frame, view kept roughly horizontal."""
    x0, x1, y0, y1 = box
    pos = np.array([rng.uniform(x0 + 1.0, x1 - 1.0), rng.uniform(y0 + 1.0, y1 - 1.0), rng.uniform(1.2, 1.7)])
    R = look_rotation(rng.uniform(0, 2 * np.pi), np.deg2rad(rng.uniform(-15, -5)))
    d = random_unit(rng)
    d[2] *= 0.2
    d /= np.linalg.norm(d)
    spin = 1.0 if rng.uniform() < 0.5 else -1.0
    poses = []
    for _ in range(n):
        poses.append(make_pose(R.copy(), pos.copy()))
        d = d + 0.3 * rng.normal(size=3)
        d[2] *= 0.2
        d /= np.linalg.norm(d)
        nxt = pos + step_m * d
        if not (x0 + wall_margin <= nxt[0] <= x1 - wall_margin and y0 + wall_margin <= nxt[1] <= y1 - wall_margin
                and 0.8 <= nxt[2] <= 2.2):
            d = -d
            nxt = pos + step_m * d
        pos = nxt
        axis = UP + 0.25 * rng.normal(size=3)
        if rng.uniform() < 0.1:
            spin = -spin
        R = quat_rot(axis, spin * np.deg2rad(step_deg)) @ R
    return np.array(poses)


def _catmull_rom_closed(pts, samples_per_seg=200):
    pts = np.asarray(pts, np.float64)
    n = len(pts)
    out = []
    for i in range(n):
        p0, p1, p2, p3 = pts[(i - 1) % n], pts[i], pts[(i + 1) % n], pts[(i + 2) % n]
        t = np.linspace(0, 1, samples_per_seg, endpoint=False)[:, None]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3))
    return np.concatenate(out)


def resample_closed(curve, n):
    """n points equally spaced in arc length along a closed polyline; also the length."""
    seg = np.linalg.norm(np.diff(np.vstack([curve, curve[:1]]), axis=0), axis=1)
    s = np.concatenate([[0], np.cumsum(seg)])
    total = s[-1]
    targets = np.arange(n) * total / n
    ext = np.vstack([curve, curve[:1]])
    out = np.empty((n, curve.shape[1]))
    for k in range(curve.shape[1]):
        out[:, k] = np.interp(targets, s, ext[:, k])
    return out, total


def path_poses(points, height=1.5, pitch_deg=-8.0, yaw_wobble_deg=25.0, wobble_period=12):
    """Poses along a horizontal path, looking along the tangent with a slow yaw
    oscillation of +-yaw_wobble_deg."""
    n = len(points)
    poses = []
    for k in range(n):
        tang = points[(k + 1) % n] - points[(k - 1) % n]
        yaw = np.arctan2(tang[1], tang[0]) + np.deg2rad(yaw_wobble_deg) * np.sin(2 * np.pi * k / wobble_period)
        R = look_rotation(yaw, np.deg2rad(pitch_deg))
        poses.append(make_pose(R, np.array([points[k][0], points[k][1], height])))
    return np.array(poses)


def apartment_loop(n, scale=1.0):
    """Closed loop through a row of three 4x4 m rooms (doors centred at y=2 in the
    walls x=4 and x=8): out along y~1.8 with a bulge in the middle room, an outer
    and an inner loop in the far room, back along y~2.2 with a bulge, and an outer
    and an inner loop in the first room (about 39 m).  Returns (points [n,2], length)."""
    wp = [(2.6, 1.8), (4.0, 1.8), (5.0, 1.5), (5.6, 0.8), (6.6, 0.75), (7.4, 1.5), (8.0, 1.8),
          (9.0, 1.0), (10.0, 0.65), (11.2, 0.9), (11.4, 2.0), (11.2, 3.1), (10.0, 3.35), (9.0, 2.9),
          (9.1, 1.9), (10.0, 1.4), (10.8, 2.0), (10.2, 2.7), (9.0, 2.5), (8.0, 2.2),
          (7.3, 2.6), (6.6, 3.25), (5.4, 3.25), (4.6, 2.6), (4.0, 2.2),
          (3.0, 2.8), (2.0, 3.35), (0.9, 3.1), (0.65, 2.0), (0.9, 0.9), (2.0, 0.65), (3.0, 1.1),
          (2.9, 2.1), (2.0, 2.6), (1.3, 2.0), (1.8, 1.3)]
    curve = _catmull_rom_closed(wp)
    return resample_closed(curve, n)


def floor_lawnmower(n, nx=5, ny=5, size=4.0, passes=2):
    """Lawnmower sweeps over an nx-by-ny grid of rooms through the centred doors:
    rows along x, then columns along y, repeated `passes` times.  Returns
    (points [n,2], length)."""
    wp = []
    for _ in range(passes):
        for r in range(ny):
            y = (r + 0.5) * size
            lo, hi = 0.5 * size, (nx - 0.5) * size
            xs = [lo, hi] if r % 2 == 0 else [hi, lo]
            wp += [(xs[0], y), (0.5 * (xs[0] + xs[1]), y), (xs[1], y)]
        for c in range(nx - 1, -1, -1):
            x = (c + 0.5) * size
            lo, hi = 0.5 * size, (ny - 0.5) * size
            ys = [hi, lo] if (nx - 1 - c) % 2 == 0 else [lo, hi]
            wp += [(x, ys[0]), (x, 0.5 * (ys[0] + ys[1])), (x, ys[1])]
    curve = _catmull_rom_closed(wp, samples_per_seg=120)
    return resample_closed(curve, n)
