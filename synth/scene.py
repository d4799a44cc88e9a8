"""Procedural indoor scenes and an analytic ray caster for synthetic RGB-D scans.

This module only produces inputs: geometry, texture and rendered depth /
intensity images.  It holds none of the pose-alignment arithmetic (no
normals, gradients, residuals, Jacobians or solver steps).

Scenes are built from axis-aligned rectangles (walls, floor, ceiling, with
door openings cut out of shared walls) and spheres, in a world frame with z
up.  Texture is gradient noise written from Perlin's published lattice
gradient method (random gradients at integer lattice points, a quintic fade
curve, trilinear blending of the corner contributions).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROOM_HEIGHT = 3.0
DOOR_WIDTH = 1.0
DOOR_HEIGHT = 2.1

# Gradient directions: the 12 edge midpoints of a cube.
_GRADS = np.array(
    [[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0],
     [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
     [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], dtype=np.float64)


class GradientNoise:
    """3D lattice gradient noise with a seeded permutation table."""

    def __init__(self, rng: np.random.Generator):
        perm = rng.permutation(256)
        self.perm = np.concatenate([perm, perm]).astype(np.int64)

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def _corner(self, xi, yi, zi, fx, fy, fz):
        p = self.perm
        h = p[p[p[xi & 255] + (yi & 255)] + (zi & 255)] % 12
        g = _GRADS[h]
        return g[..., 0] * fx + g[..., 1] * fy + g[..., 2] * fz

    def __call__(self, x, y, z):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        z = np.asarray(z, np.float64)
        x0 = np.floor(x)
        y0 = np.floor(y)
        z0 = np.floor(z)
        fx, fy, fz = x - x0, y - y0, z - z0
        xi, yi, zi = x0.astype(np.int64), y0.astype(np.int64), z0.astype(np.int64)
        u, v, w = self._fade(fx), self._fade(fy), self._fade(fz)
        out = 0.0
        for dx in (0, 1):
            wx = u if dx else 1.0 - u
            for dy in (0, 1):
                wy = v if dy else 1.0 - v
                for dz in (0, 1):
                    wz = w if dz else 1.0 - w
                    c = self._corner(xi + dx, yi + dy, zi + dz, fx - dx, fy - dy, fz - dz)
                    out = out + wx * wy * wz * c
        return out


@dataclass
class Scene:
    """Axis-aligned rectangles plus spheres, with a noise texture."""
    # quads: rows of (axis, plane_value, lo_a, hi_a, lo_b, hi_b, tex_offset)
    # where (a, b) are the two remaining axes in increasing order.
    quads: np.ndarray
    sphere_c: np.ndarray          # [S,3]
    sphere_r: np.ndarray          # [S]
    sphere_tex: np.ndarray        # [S] texture offsets
    noise: GradientNoise
    rooms: list = field(default_factory=list)   # (x0, x1, y0, y1)

    def texture(self, pts, offs):
        """Intensity in [0,1] at world points `pts` [N,3]; `offs` [N] decorrelates surfaces."""
        n1 = self.noise(3.1 * pts[:, 0] + offs, 3.1 * pts[:, 1] + 0.37 * offs, 3.1 * pts[:, 2] - offs)
        n2 = self.noise(7.3 * pts[:, 0] - offs, 7.3 * pts[:, 1] + 11.0, 7.3 * pts[:, 2] + 0.5 * offs)
        val = 0.5 + 0.55 * (0.75 * n1 + 0.25 * n2)
        return np.clip(val, 0.0, 1.0)

    def _bounds(self):
        """Per primitive: axis-aligned box (lo [3], hi [3]) and texture offset, quads first."""
        if getattr(self, "_bounds_cache", None) is None:
            lo, hi, off = [], [], []
            for q in self.quads:
                ax = int(q[0])
                oa = [k for k in range(3) if k != ax]
                a = np.zeros(3)
                b = np.zeros(3)
                a[ax] = b[ax] = q[1]
                a[oa[0]], b[oa[0]] = q[2], q[3]
                a[oa[1]], b[oa[1]] = q[4], q[5]
                lo.append(a)
                hi.append(b)
                off.append(q[6])
            for c, r, o in zip(self.sphere_c, self.sphere_r, self.sphere_tex):
                lo.append(np.asarray(c, np.float64) - r)
                hi.append(np.asarray(c, np.float64) + r)
                off.append(o)
            self._bounds_cache = (np.array(lo).reshape(-1, 3), np.array(hi).reshape(-1, 3), np.array(off))
        return self._bounds_cache

    def raycast(self, origin, dirs, tmin=1e-6):
        """Nearest hit along rays origin + t*dirs from one origin [3] (dirs [N,3], not
        necessarily unit).  Returns (t [N] with inf for a miss, intensity [N], hit
        points [N,3]).

        Primitives are visited nearest first and each is tested only on the rays
        whose current hit is farther than the primitive's bounding box (with a
        relative margin far above rounding), so skipped tests could never have won.
        Among hits at exactly the same t the primitive listed first wins, so the
        result is bit for bit that of testing every primitive in list order
        (raycast_all)."""
        dirs = np.asarray(dirs, np.float64)
        n = dirs.shape[0]
        origin = np.asarray(origin, np.float64)
        if origin.ndim != 1 or n == 0:
            return self.raycast_all(origin, dirs, tmin)
        lo, hi, offs = self._bounds()
        nq = len(self.quads)
        gap = np.maximum(np.maximum(lo - origin, origin - hi), 0.0)
        dmin = np.sqrt((gap * gap).sum(axis=1))
        sc = np.asarray(self.sphere_c, np.float64).reshape(-1, 3)
        if len(sc):
            ds = np.sqrt(((sc - origin) ** 2).sum(axis=1)) - np.asarray(self.sphere_r, np.float64)
            dmin[nq:] = np.maximum(np.maximum(ds, 0.0), dmin[nq:])
        dlen = np.sqrt((dirs * dirs).sum(axis=1))
        o = np.broadcast_to(origin, (n, 3))
        best_t = np.full(n, np.inf)
        best_p = np.full(n, len(offs), np.int64)
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            reach = np.inf
            for i, p in enumerate(np.argsort(dmin, kind="stable")):
                if i % 16 == 0:
                    reach = float((best_t * dlen).max()) * (1.0 + 1e-9)
                if dmin[p] > reach:
                    break  # every later primitive is farther than every current hit
                act = np.nonzero(best_t * dlen * (1.0 + 1e-9) >= dmin[p])[0]
                if act.size == 0:
                    continue
                d = dirs[act]
                oo = o[act]
                bt = best_t[act]
                if p < nq:
                    q = self.quads[p]
                    ax = int(q[0])
                    oa = [k for k in range(3) if k != ax]
                    t = (q[1] - oo[:, ax]) / d[:, ax]
                    pa = oo[:, oa[0]] + t * d[:, oa[0]]
                    pb = oo[:, oa[1]] + t * d[:, oa[1]]
                    geo = (t > tmin) & (pa >= q[2]) & (pa <= q[3]) & (pb >= q[4]) & (pb <= q[5])
                else:
                    k = p - nq
                    c, r = self.sphere_c[k], self.sphere_r[k]
                    a = np.einsum("ij,ij->i", d, d)
                    oc = oo - c
                    b = 2.0 * np.einsum("ij,ij->i", d, oc)
                    cc = np.einsum("ij,ij->i", oc, oc) - r * r
                    disc = b * b - 4.0 * a * cc
                    sq = np.sqrt(np.maximum(disc, 0.0))
                    t1 = (-b - sq) / (2.0 * a)
                    t2 = (-b + sq) / (2.0 * a)
                    t = np.where(t1 > tmin, t1, t2)
                    geo = (disc >= 0) & (t > tmin)
                ok = geo & ((t < bt) | ((t == bt) & (p < best_p[act])))
                sel = act[ok]
                best_t[sel] = t[ok]
                best_p[sel] = p
        best_off = np.where(best_p < len(offs), offs[np.minimum(best_p, len(offs) - 1)], 0.0)
        hit = o + best_t[:, None] * dirs
        hit = np.where(np.isfinite(best_t)[:, None], hit, 0.0)
        inten = np.where(np.isfinite(best_t), self.texture(hit, best_off), 0.0)
        return best_t, inten, hit

    def raycast_all(self, origin, dirs, tmin=1e-6):
        """Nearest hit along rays origin + t*dirs, testing every primitive on every ray.

        origin: [3] or [N,3]; dirs: [N,3] (not necessarily unit).
        Returns (t [N] with inf for a miss, intensity [N], hit points [N,3]).
        """
        dirs = np.asarray(dirs, np.float64)
        n = dirs.shape[0]
        o = np.broadcast_to(np.asarray(origin, np.float64), (n, 3))
        best_t = np.full(n, np.inf)
        best_off = np.zeros(n)
        with np.errstate(divide="ignore", invalid="ignore"):
            for q in self.quads:
                ax = int(q[0])
                oa = [k for k in range(3) if k != ax]
                t = (q[1] - o[:, ax]) / dirs[:, ax]
                pa = o[:, oa[0]] + t * dirs[:, oa[0]]
                pb = o[:, oa[1]] + t * dirs[:, oa[1]]
                ok = (t > tmin) & (t < best_t) & (pa >= q[2]) & (pa <= q[3]) & (pb >= q[4]) & (pb <= q[5])
                best_t = np.where(ok, t, best_t)
                best_off = np.where(ok, q[6], best_off)
            a = np.einsum("ij,ij->i", dirs, dirs)
            for c, r, off in zip(self.sphere_c, self.sphere_r, self.sphere_tex):
                oc = o - c
                b = 2.0 * np.einsum("ij,ij->i", dirs, oc)
                cc = np.einsum("ij,ij->i", oc, oc) - r * r
                disc = b * b - 4.0 * a * cc
                sq = np.sqrt(np.maximum(disc, 0.0))
                t1 = (-b - sq) / (2.0 * a)
                t2 = (-b + sq) / (2.0 * a)
                t = np.where(t1 > tmin, t1, t2)
                ok = (disc >= 0) & (t > tmin) & (t < best_t)
                best_t = np.where(ok, t, best_t)
                best_off = np.where(ok, off, best_off)
        hit = o + best_t[:, None] * dirs
        hit = np.where(np.isfinite(best_t)[:, None], hit, 0.0)
        inten = np.where(np.isfinite(best_t), self.texture(hit, best_off), 0.0)
        return best_t, inten, hit


def _wall_segments(fixed_axis, value, span_lo, span_hi, door, tex):
    """Quads of a vertical wall on plane `axis=value`, spanning [span_lo, span_hi]
    horizontally and [0, ROOM_HEIGHT] vertically, optionally with a centred door."""
    # remaining axes in increasing order: for axis 0 -> (1, 2); axis 1 -> (0, 2)
    out = []
    if not door:
        out.append((fixed_axis, value, span_lo, span_hi, 0.0, ROOM_HEIGHT, tex))
        return out
    mid = 0.5 * (span_lo + span_hi)
    d0, d1 = mid - 0.5 * DOOR_WIDTH, mid + 0.5 * DOOR_WIDTH
    out.append((fixed_axis, value, span_lo, d0, 0.0, ROOM_HEIGHT, tex))
    out.append((fixed_axis, value, d1, span_hi, 0.0, ROOM_HEIGHT, tex + 0.5))
    out.append((fixed_axis, value, d0, d1, DOOR_HEIGHT, ROOM_HEIGHT, tex + 0.25))
    return out


def grid_rooms(nx, ny, size, rng, doors=True):
    """Quads for an nx-by-ny grid of square rooms of side `size`, with centred doors
    in every internal wall when `doors` is set."""
    quads = []
    tex = 10.0
    X, Y = nx * size, ny * size
    quads.append((2, 0.0, 0.0, X, 0.0, Y, tex)); tex += 17.0          # floor
    quads.append((2, ROOM_HEIGHT, 0.0, X, 0.0, Y, tex)); tex += 17.0  # ceiling
    for k in range(nx + 1):            # walls x = const, segments along y
        for c in range(ny):
            internal = 0 < k < nx
            quads += _wall_segments(0, k * size, c * size, (c + 1) * size, doors and internal, tex)
            tex += 17.0 + rng.uniform(0, 5)
    for k in range(ny + 1):            # walls y = const, segments along x
        for c in range(nx):
            internal = 0 < k < ny
            quads += _wall_segments(1, k * size, c * size, (c + 1) * size, doors and internal, tex)
            tex += 17.0 + rng.uniform(0, 5)
    rooms = [(i * size, (i + 1) * size, j * size, (j + 1) * size) for j in range(ny) for i in range(nx)]
    return np.array(quads, np.float64), rooms


def place_spheres(rng, rooms, cam_pos, per_room=6, rmin=0.2, rmax=0.6, clearance=0.45):
    """Seeded spheres fully inside each room, kept away from every camera centre."""
    cs, rs = [], []
    for (x0, x1, y0, y1) in rooms:
        placed = 0
        tries = 0
        while placed < per_room and tries < 2000:
            tries += 1
            r = rng.uniform(rmin, rmax)
            c = np.array([rng.uniform(x0 + r, x1 - r), rng.uniform(y0 + r, y1 - r),
                          rng.uniform(r, ROOM_HEIGHT - r)])
            if len(cam_pos) and np.min(np.linalg.norm(cam_pos - c, axis=1)) < r + clearance:
                continue
            if any(np.linalg.norm(c - c2) < r + r2 + 0.05 for c2, r2 in zip(cs, rs)):
                continue
            cs.append(c)
            rs.append(r)
            placed += 1
    cs = np.array(cs, np.float64).reshape(-1, 3)
    rs = np.array(rs, np.float64)
    return cs, rs


def make_scene(rng_scene, nx, ny, cam_pos, size=4.0, doors=True, spheres=True):
    quads, rooms = grid_rooms(nx, ny, size, rng_scene, doors=doors)
    noise = GradientNoise(rng_scene)
    if spheres:
        sc, sr = place_spheres(rng_scene, rooms, cam_pos)
    else:
        sc, sr = np.zeros((0, 3)), np.zeros(0)
    stex = 1000.0 + 37.0 * np.arange(len(sr))
    return Scene(quads=quads, sphere_c=sc, sphere_r=sr, sphere_tex=stex, noise=noise, rooms=rooms)
