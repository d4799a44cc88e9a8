"""Seeded synthetic pose-alignment problems shaped like the paper's workloads.

The paper's captured indoor sequences are not available; these renders stand
in for them.  Every problem is a set of RGB-D frames (depth in metres,
intensity in [0,1]), sparse 3D point correspondences between frame pairs,
ground-truth poses and initial poses.  Frame 0 defines the world frame.

Workloads (frame counts, resolutions, correspondence counts, noise, outlier
rates and iteration budgets follow the five configurations this library is
measured on):

* ``chunk``   -- 11 frames, 80x60, one 4x4x3 m room with 6 spheres, random walk
  of 2 cm / 1 deg per frame, 150 correspondences on every one of the 55 pairs,
  10% outliers, init = GT perturbed by 3 cm / 2 deg, 5 GN x 10 PCG.
* ``global200`` -- 200 keyframes on a closed loop through three rooms, 80x60,
  100-300 correspondences per co-visible pair, 5% outliers, init with
  accumulated 1 cm / 0.5 deg per-frame drift, 8 GN x 20 PCG.
* ``batch_chunk`` -- one chunk of a batch: 4-11 frames at 160x120 (fx=fy=144),
  sparse term as ``chunk``.
* ``global2000`` -- 2000 keyframes over a 5x5-room floor (400 m^2), 80x60,
  200 correspondences per co-visible pair, 10% outliers, drift init, 8 GN x 20 PCG.

Noise model: depth += N(0, (0.0012 z^2)^2), 1% of pixels dropped to 0; sparse
observations get 1 px of Gaussian pixel noise at 640x480 sensor resolution
(1/8 px at 80x60) and the same depth noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .scene import make_scene
from .trajectory import (apartment_loop, floor_lawnmower, make_pose, path_poses, perturbation,
                         random_walk, rigid_inv)

SENSOR_W, SENSOR_H = 640, 480


@dataclass
class Problem:
    name: str
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    depth: np.ndarray          # f32 [F,H,W]
    intensity: np.ndarray      # f32 [F,H,W]
    corr_i: np.ndarray         # i32 [M]
    corr_j: np.ndarray         # i32 [M]
    corr_p: np.ndarray         # f32 [M,3] point in camera corr_i
    corr_q: np.ndarray         # f32 [M,3] point in camera corr_j
    gt_poses: np.ndarray       # f64 [F,4,4] camera-to-world, frame 0 = identity
    init_poses: np.ndarray     # f64 [F,4,4]
    n_gn: int
    n_pcg: int
    outlier: np.ndarray = None  # bool [M]
    info: dict = field(default_factory=dict)

    @property
    def num_frames(self):
        return self.depth.shape[0]

    @property
    def intrinsics(self):
        return (self.fx, self.fy, self.cx, self.cy, self.width, self.height)


_SHARED = {}


def _workers(n_items, workers=None):
    """Worker processes for n_items independent tasks: $BF_SYNTH_WORKERS if set,
    else min(16, cpu count); 1 (no fork) when torch already holds a GPU context in
    this process.  Set BF_SYNTH_WORKERS=1 when a tool attached to the process may
    hold one (a profiler)."""
    import os
    import sys
    if workers is None:
        env = os.environ.get("BF_SYNTH_WORKERS")
        workers = int(env) if env else min(16, os.cpu_count() or 1)
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        workers = 1
    import multiprocessing as mp
    if mp.current_process().daemon:
        workers = 1  # already inside a pool worker
    return workers if n_items >= 2 * workers else 1


def _pmap(fn, items, shared, workers=None):
    """map(fn, items) over forked worker processes; `shared` (read-only, e.g. the
    scene) is inherited by the workers through a module global instead of being
    pickled per task.  Results are returned in item order."""
    items = list(items)
    _SHARED.clear()
    _SHARED.update(shared)
    w = _workers(len(items), workers)
    try:
        if w <= 1:
            return [fn(x) for x in items]
        import multiprocessing as mp
        with mp.get_context("fork").Pool(w) as pool:
            return pool.map(fn, items, chunksize=max(1, len(items) // (8 * w)))
    finally:
        _SHARED.clear()


def _pixel_rays(W, H, fx, fy, cx, cy):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    return np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], axis=-1).reshape(-1, 3)


def _render_one(T):
    scene, rays = _SHARED["scene"], _SHARED["rays"]
    t, val, _ = scene.raycast(T[:3, 3], rays @ T[:3, :3].T)
    return t, val


def render_frames(scene, abs_poses, W, H, fx, fy, cx, cy, rng_noise, noise=True, dropout=0.01):
    """Noise-free renders in parallel (deterministic), then depth noise and dropout
    drawn frame by frame in order from rng_noise."""
    rays = _pixel_rays(W, H, fx, fy, cx, cy)
    F = len(abs_poses)
    depth = np.zeros((F, H, W), np.float32)
    inten = np.zeros((F, H, W), np.float32)
    clean = _pmap(_render_one, list(abs_poses), {"scene": scene, "rays": rays})
    for f, (t, val) in enumerate(clean):
        z = np.where(np.isfinite(t), t, 0.0)
        if noise:
            z = np.where(z > 0, z + rng_noise.normal(size=z.shape) * 0.0012 * z * z, 0.0)
            drop = rng_noise.uniform(size=z.shape) < dropout
            z = np.where(drop, 0.0, z)
        depth[f] = z.reshape(H, W).astype(np.float32)
        inten[f] = val.reshape(H, W).astype(np.float32)
    return depth, inten


class _Sensor:
    """Full-resolution pinhole model used to place sparse feature observations."""

    def __init__(self, W, fx, fy, cx, cy):
        s = SENSOR_W / W
        self.fx, self.fy = fx * s, fy * s
        self.cx, self.cy = cx * s, cy * s

    def rays(self, u, v):
        return np.stack([(u - self.cx) / self.fx, (v - self.cy) / self.fy, np.ones_like(u)], axis=-1)

    def project(self, Xc):
        return self.fx * Xc[:, 0] / Xc[:, 2] + self.cx, self.fy * Xc[:, 1] / Xc[:, 2] + self.cy

    def in_image(self, u, v):
        return (u >= 0) & (u < SENSOR_W) & (v >= 0) & (v < SENSOR_H)


def _visible_from(scene, T, X, tol=0.01):
    """Points X [N,3] (world) that are in front of camera T and not occluded."""
    o = T[:3, 3]
    d = X - o
    t, _, _ = scene.raycast(o, d)
    dist = np.linalg.norm(d, axis=1)
    return t >= 1.0 - tol / np.maximum(dist, 1e-9)


def _cam_coords(T, X):
    return (X - T[:3, 3]) @ T[:3, :3]


def _surface_samples(scene, T, sensor, n, rng):
    u = rng.uniform(0, SENSOR_W, n)
    v = rng.uniform(0, SENSOR_H, n)
    t, _, X = scene.raycast(T[:3, 3], sensor.rays(u, v) @ T[:3, :3].T)
    ok = np.isfinite(t)
    return u[ok], v[ok], X[ok]


def _observe(rng, sensor, Xc, u, v, noise=True):
    """Back-project a noisy observation of camera-space points Xc seen at pixels (u,v)."""
    z = Xc[:, 2].copy()
    if noise:
        u = u + rng.normal(size=u.shape)
        v = v + rng.normal(size=v.shape)
        z = z + rng.normal(size=z.shape) * 0.0012 * z * z
    return sensor.rays(u, v) * z[:, None]


def pair_correspondences(rng, scene, Ti, Tj, sensor, k, outlier_rate, noise=True, max_rounds=6):
    """k sparse correspondences between frames i and j at surface points visible in both."""
    got_u, got_v, got_X = [], [], []
    need = k
    for _ in range(max_rounds):
        u, v, X = _surface_samples(scene, Ti, sensor, max(4 * need, 64), rng)
        Xj = _cam_coords(Tj, X)
        front = Xj[:, 2] > 0.1
        uj, vj = np.full(len(X), -1.0), np.full(len(X), -1.0)
        uj[front], vj[front] = sensor.project(Xj[front])
        ok = front & sensor.in_image(uj, vj)
        idx = np.nonzero(ok)[0]
        if len(idx):
            vis = _visible_from(scene, Tj, X[idx])
            idx = idx[vis]
        idx = idx[:need]
        got_u.append(u[idx]); got_v.append(v[idx]); got_X.append(X[idx])
        need -= len(idx)
        if need <= 0:
            break
    u = np.concatenate(got_u); v = np.concatenate(got_v); X = np.concatenate(got_X).reshape(-1, 3)
    if len(X) == 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, bool)
    Xi = _cam_coords(Ti, X)
    Xj = _cam_coords(Tj, X)
    p = _observe(rng, sensor, Xi, u, v, noise)
    uj, vj = sensor.project(Xj)
    q = _observe(rng, sensor, Xj, uj, vj, noise)
    outl = rng.uniform(size=len(X)) < outlier_rate
    n_out = int(outl.sum())
    if n_out:
        ou, ov, oX = _surface_samples(scene, Tj, sensor, 4 * n_out + 16, rng)
        oXc = _cam_coords(Tj, oX)[:n_out]
        if len(oXc) == n_out:
            q[outl] = sensor.rays(ou[:n_out], ov[:n_out]) * oXc[:, 2:3]
        else:
            outl[:] = False
    return p, q, outl


def _covisible_row(i):
    sh = _SHARED
    scene, abs_poses, sensor, samp = sh["scene"], sh["poses"], sh["sensor"], sh["samp"]
    max_dist, cos_max, need = sh["max_dist"], sh["cos_max"], sh["need"]
    F = len(abs_poses)
    pos = abs_poses[:, :3, 3]
    fwd = abs_poses[:, :3, 2]
    pairs = []
    js = np.arange(i + 1, F)
    js = js[(np.linalg.norm(pos[js] - pos[i], axis=1) <= max_dist) & (fwd[js] @ fwd[i] >= cos_max)]
    if len(js) == 0:
        return pairs
    X = samp[i]
    Xj = np.einsum("nk,jkl->jnl", X, abs_poses[js, :3, :3]) - np.einsum("jk,jkl->jl", pos[js], abs_poses[js, :3, :3])[:, None, :]
    z = Xj[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = sensor.fx * Xj[..., 0] / z + sensor.cx
        v = sensor.fy * Xj[..., 1] / z + sensor.cy
    ok = (z > 0.1) & sensor.in_image(u, v)
    maps = sh.get("maps")
    for jj in np.nonzero(ok.sum(axis=1) >= need)[0]:
        if maps is None:
            vis = _visible_from(scene, abs_poses[js[jj]], X[ok[jj]])
        else:
            vis = _map_visible(maps[js[jj]][1], u[jj][ok[jj]], v[jj][ok[jj]], z[jj][ok[jj]])
        if vis.sum() >= need:
            pairs.append((i, int(js[jj])))
    return pairs


def _map_visible(zmap, u, v, z):
    """Depth-map visibility at sensor pixels (u, v) of points at camera depth z: the
    nearest grid point of the frame's surface map is not more than 2 cm (or 1 % of
    the depth) in front of the point."""
    gw, gh = SENSOR_W // _MAP_STEP, SENSOR_H // _MAP_STEP
    gx = np.clip(np.floor(u / _MAP_STEP), 0, gw - 1).astype(np.int64)
    gy = np.clip(np.floor(v / _MAP_STEP), 0, gh - 1).astype(np.int64)
    zb = zmap[gy * gw + gx]
    return (zb > 0) & (zb >= z - np.maximum(0.02, 0.01 * z))


def covisible_pairs(rng, scene, abs_poses, sensor, max_dist=8.0, max_angle_deg=75.0,
                    samples=48, min_frac=0.25, maps=None):
    """Frame pairs i<j that see a common part of the scene (ground truth): at least
    `min_frac` of `samples` surface points seen by i are in j's view and unoccluded.
    The samples are drawn in frame order; the rows are tested in parallel."""
    F = len(abs_poses)
    samp = [_surface_samples(scene, T, sensor, samples, rng)[2] for T in abs_poses]
    shared = {"scene": scene, "poses": abs_poses, "sensor": sensor, "samp": samp, "max_dist": max_dist,
              "cos_max": np.cos(np.deg2rad(max_angle_deg)), "need": min_frac * samples, "maps": maps}
    rows = _pmap(_covisible_row, range(F - 1), shared)
    return [p for row in rows for p in row]


# Sample grid of the per-frame surface maps used by the parallel correspondence
# generator: every 4th sensor pixel in each direction (160x120 of 640x480).
_MAP_STEP = 4


def _surface_map_one(T):
    """Surface points (world, float32) and camera depths (0 = no hit) of the sample
    grid of one frame."""
    scene, rays = _SHARED["scene"], _SHARED["grid_rays"]
    t, _, X = scene.raycast(T[:3, 3], rays @ T[:3, :3].T)
    ok = np.isfinite(t)
    return X.astype(np.float32), np.where(ok, t, 0.0).astype(np.float32)


def surface_maps(scene, abs_poses, sensor):
    """Per frame: surface points and depths of the sample grid (in parallel)."""
    gw, gh = SENSOR_W // _MAP_STEP, SENSOR_H // _MAP_STEP
    gy, gx = np.mgrid[0:gh, 0:gw].astype(np.float64)
    grid_rays = sensor.rays((gx * _MAP_STEP + 0.5 * (_MAP_STEP - 1)).ravel(),
                            (gy * _MAP_STEP + 0.5 * (_MAP_STEP - 1)).ravel())
    return _pmap(_surface_map_one, list(abs_poses), {"scene": scene, "grid_rays": grid_rays})


def _pair_job(args):
    """Correspondences of pair n from its own random stream, using the frames'
    surface maps: samples are grid points of frame i, visibility in frame j is a
    depth-map test at the nearest grid point (2 cm or 1 % of the depth)."""
    n, i, j, k = args
    sh = _SHARED
    rng = np.random.Generator(np.random.PCG64([sh["seed"], n]))
    sensor, Ti, Tj = sh["sensor"], sh["poses"][i], sh["poses"][j]
    Xi_map, zi = sh["maps"][i]
    _, zj = sh["maps"][j]
    gw, gh = SENSOR_W // _MAP_STEP, SENSOR_H // _MAP_STEP
    valid_i = np.nonzero(zi > 0)[0]
    got, need = [], k
    for _ in range(6):
        if need <= 0 or len(valid_i) == 0:
            break
        idx = valid_i[rng.integers(0, len(valid_i), max(4 * need, 64))]
        X = Xi_map[idx].astype(np.float64)
        Xj = _cam_coords(Tj, X)
        front = Xj[:, 2] > 0.1
        uj, vj = np.full(len(X), -1.0), np.full(len(X), -1.0)
        uj[front], vj[front] = sensor.project(Xj[front])
        ok = front & sensor.in_image(uj, vj)
        ok &= _map_visible(zj, uj, vj, Xj[:, 2])
        sel = idx[np.nonzero(ok)[0][:need]]
        got.append(sel)
        need -= len(sel)
    sel = np.concatenate(got) if got else np.zeros(0, np.int64)
    if len(sel) == 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, bool)
    X = Xi_map[sel].astype(np.float64)
    u = (sel % gw) * _MAP_STEP + 0.5 * (_MAP_STEP - 1)
    v = (sel // gw) * _MAP_STEP + 0.5 * (_MAP_STEP - 1)
    Xi = _cam_coords(Ti, X)
    Xj = _cam_coords(Tj, X)
    p = _observe(rng, sensor, Xi, u, v, sh["noise"])
    uj, vj = sensor.project(Xj)
    q = _observe(rng, sensor, Xj, uj, vj, sh["noise"])
    outl = rng.uniform(size=len(X)) < sh["outlier_rate"]
    n_out = int(outl.sum())
    Xj_map, _ = sh["maps"][j]
    valid_j = np.nonzero(zj > 0)[0]
    if n_out and len(valid_j):
        oi = valid_j[rng.integers(0, len(valid_j), n_out)]
        q[outl] = _cam_coords(Tj, Xj_map[oi].astype(np.float64))
    elif n_out:
        outl[:] = False
    return p, q, outl


def _assemble(name, scene, abs_poses, W, H, fx, fy, cx, cy, seeds, sparse_pairs, k_of_pair,
              outlier_rate, init_mode, n_gn, n_pcg, noise=True, init_rot=2.0, init_trans=0.03,
              drift_rot=0.5, drift_trans=0.01, per_pair_streams=False, maps=None):
    """per_pair_streams: pair n draws its correspondences from its own stream
    PCG64([corr seed, n]) against per-frame surface maps (pairs run in parallel);
    otherwise one stream in pair order with exact ray casts."""
    rng_noise = np.random.Generator(np.random.PCG64(seeds["noise"]))
    rng_corr = np.random.Generator(np.random.PCG64(seeds["corr"]))
    depth, inten = render_frames(scene, abs_poses, W, H, fx, fy, cx, cy, rng_noise, noise=noise,
                                 dropout=0.01 if noise else 0.0)
    sensor = _Sensor(W, fx, fy, cx, cy)
    ci, cj, cp, cq, co = [], [], [], [], []
    if per_pair_streams:
        jobs = [(n, i, j, k_of_pair(rng_corr)) for n, (i, j) in enumerate(sparse_pairs)]
        if maps is None:
            maps = surface_maps(scene, abs_poses, sensor)
        shared = {"seed": seeds["corr"], "poses": abs_poses, "sensor": sensor, "maps": maps,
                  "outlier_rate": outlier_rate, "noise": noise}
        results = _pmap(_pair_job, jobs, shared)
    else:
        results = []
        for (i, j) in sparse_pairs:
            k = k_of_pair(rng_corr)
            results.append(pair_correspondences(rng_corr, scene, abs_poses[i], abs_poses[j], sensor, k,
                                                outlier_rate, noise=noise))
    for (i, j), (p, q, outl) in zip(sparse_pairs, results):
        ci.append(np.full(len(p), i, np.int32)); cj.append(np.full(len(p), j, np.int32))
        cp.append(p); cq.append(q); co.append(outl)
    base_inv = rigid_inv(abs_poses[0])
    gt = np.array([base_inv @ T for T in abs_poses])
    gt[0] = np.eye(4)
    rng_init = np.random.Generator(np.random.PCG64(seeds["traj"] + 7))
    init = np.empty_like(gt)
    init[0] = np.eye(4)
    for f in range(1, len(gt)):
        if init_mode == "perturb":
            init[f] = gt[f] @ perturbation(rng_init, init_rot, init_trans)
        elif init_mode == "drift":
            init[f] = init[f - 1] @ (rigid_inv(gt[f - 1]) @ gt[f]) @ perturbation(rng_init, drift_rot, drift_trans)
        elif init_mode == "identity":
            init[f] = np.eye(4)
        else:
            init[f] = gt[f]
    cat = lambda xs, dt, shape: (np.concatenate(xs).astype(dt) if xs else np.zeros(shape, dt))
    return Problem(name=name, width=W, height=H, fx=fx, fy=fy, cx=cx, cy=cy, depth=depth, intensity=inten,
                   corr_i=cat(ci, np.int32, (0,)), corr_j=cat(cj, np.int32, (0,)),
                   corr_p=cat(cp, np.float32, (0, 3)).reshape(-1, 3), corr_q=cat(cq, np.float32, (0, 3)).reshape(-1, 3),
                   gt_poses=gt, init_poses=init, n_gn=n_gn, n_pcg=n_pcg,
                   outlier=cat(co, bool, (0,)),
                   info={"seeds": seeds, "sparse_pairs": len(sparse_pairs), "rooms": len(scene.rooms),
                         "spheres": int(len(scene.sphere_r))})


def _seeds(config, offset=0):
    return {"scene": 100 + config + offset, "traj": 200 + config + offset,
            "noise": 300 + config + offset, "corr": 400 + config + offset}


def make_chunk(num_frames=11, W=80, H=60, fx=72.0, fy=72.0, cx=40.0, cy=30.0, seed_offset=0, config=0,
               noise=True, outlier_rate=0.10, corr_per_pair=150, spheres=True, init_mode="perturb",
               n_gn=5, n_pcg=10, name="chunk"):
    """A single intra-chunk problem in one 4x4x3 m room (all frame pairs get sparse terms)."""
    seeds = _seeds(config, seed_offset)
    rng_traj = np.random.Generator(np.random.PCG64(seeds["traj"]))
    rng_scene = np.random.Generator(np.random.PCG64(seeds["scene"]))
    abs_poses = random_walk(rng_traj, num_frames, (0.0, 4.0, 0.0, 4.0))
    scene = make_scene(rng_scene, 1, 1, abs_poses[:, :3, 3], doors=False, spheres=spheres)
    pairs = [(i, j) for i in range(num_frames) for j in range(i + 1, num_frames)]
    return _assemble(name, scene, abs_poses, W, H, fx, fy, cx, cy, seeds, pairs,
                     lambda r: corr_per_pair, outlier_rate if noise else 0.0, init_mode, n_gn, n_pcg,
                     noise=noise)


def make_global(num_frames=200, layout="apartment", seed_offset=0, config=1, outlier_rate=0.05,
                corr_range=(100, 300), n_gn=8, n_pcg=20, noise=True, name="global200", per_pair_streams=False):
    """A global keyframe problem along a closed path through a multi-room floor."""
    seeds = _seeds(config, seed_offset)
    rng_scene = np.random.Generator(np.random.PCG64(seeds["scene"]))
    rng_pairs = np.random.Generator(np.random.PCG64(seeds["corr"] + 99))
    if layout == "apartment":
        pts, length = apartment_loop(num_frames)
        nx, ny = 3, 1
    elif layout == "floor3":
        pts, length = floor_lawnmower(num_frames, nx=3, ny=3)
        nx, ny = 3, 3
    else:
        pts, length = floor_lawnmower(num_frames)
        nx, ny = 5, 5
    abs_poses = path_poses(pts)
    scene = make_scene(rng_scene, nx, ny, abs_poses[:, :3, 3], doors=True, spheres=True)
    sensor = _Sensor(80, 72.0, 72.0, 40.0, 30.0)
    maps = surface_maps(scene, abs_poses, sensor) if per_pair_streams else None
    pairs = covisible_pairs(rng_pairs, scene, abs_poses, sensor, maps=maps)
    lo, hi = corr_range
    prob = _assemble(name, scene, abs_poses, 80, 60, 72.0, 72.0, 40.0, 30.0, seeds, pairs,
                     lambda r: int(r.integers(lo, hi + 1)), outlier_rate, "drift", n_gn, n_pcg, noise=noise,
                     per_pair_streams=per_pair_streams, maps=maps)
    prob.info["path_length_m"] = float(length)
    return prob


def make_problem(config, seed_offset=0):
    """Problem for one of the measured workload shapes (see module docstring)."""
    if config in (0, "chunk"):
        return make_chunk(config=0, seed_offset=seed_offset)
    if config in (1, "global200"):
        return make_global(200, "apartment", config=1, seed_offset=seed_offset)
    if config in (4, "global2000"):
        return make_global(2000, "floor", config=4, seed_offset=seed_offset, outlier_rate=0.10,
                           corr_range=(200, 200), name="global2000", per_pair_streams=True)
    if isinstance(config, str) and config.startswith("floor3:"):
        # a global problem of the serving workload's kind with the given keyframe count
        n = int(config.split(":")[1])
        return make_global(n, "floor3", config=3, seed_offset=seed_offset, outlier_rate=0.10,
                           corr_range=(200, 200), name=f"floor3_{n}", per_pair_streams=True)
    raise ValueError(f"unknown config {config!r}")


def _batch_member(args):
    k, n, config = args
    return make_chunk(num_frames=int(n), W=160, H=120, fx=144.0, fy=144.0, cx=80.0, cy=60.0,
                      seed_offset=1000 * k, config=config, name=f"batch_chunk{k}")


def batch_sizes(count=256, config=2, min_frames=4, max_frames=11):
    """Frame counts U{min..max} of the members of a chunk batch."""
    rng = np.random.Generator(np.random.PCG64(500 + config))
    return rng.integers(min_frames, max_frames + 1, size=count)


def make_batch_chunks(count=256, config=2, min_frames=4, max_frames=11, workers=None):
    """`count` independent chunk problems at 160x120 with frame counts U{min..max}.
    Members depend only on their index, so they are generated in parallel
    (`workers` processes, see _workers; 1 = in this process)."""
    sizes = batch_sizes(count, config, min_frames, max_frames)
    jobs = [(k, int(n), config) for k, n in enumerate(sizes)]
    workers = _workers(count, workers)
    if workers <= 1 or count < 8:
        return [_batch_member(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_member, jobs, chunksize=max(1, count // (4 * workers)))


def window(prob, start, count, name=None):
    """The sub-problem of frames [start, start+count) of a global problem: its
    frames, the correspondences between two of them (indices re-based), and its
    poses (frame `start` becomes the window's fixed first frame)."""
    end = start + count
    keep = (prob.corr_i >= start) & (prob.corr_i < end) & (prob.corr_j >= start) & (prob.corr_j < end)
    return Problem(name=name or f"{prob.name}[{start}:{end}]", width=prob.width, height=prob.height,
                   fx=prob.fx, fy=prob.fy, cx=prob.cx, cy=prob.cy,
                   depth=np.ascontiguousarray(prob.depth[start:end]),
                   intensity=np.ascontiguousarray(prob.intensity[start:end]),
                   corr_i=(prob.corr_i[keep] - start).astype(np.int32),
                   corr_j=(prob.corr_j[keep] - start).astype(np.int32),
                   corr_p=np.ascontiguousarray(prob.corr_p[keep]), corr_q=np.ascontiguousarray(prob.corr_q[keep]),
                   gt_poses=np.ascontiguousarray(prob.gt_poses[start:end]),
                   init_poses=np.ascontiguousarray(prob.init_poses[start:end]),
                   n_gn=prob.n_gn, n_pcg=prob.n_pcg,
                   outlier=None if prob.outlier is None else prob.outlier[keep],
                   info={"window_of": prob.name, "start": start, "count": count})


def make_serving_pool(num_chunks=64, global_frames=800, global_windows=6, seed=7):
    """Request pool of the serving workload: `num_chunks` chunk problems (160x120,
    4-11 frames) and `global_windows` keyframe windows of 50..global_frames frames
    (geometrically spaced sizes, seeded start frames) cut from one `global_frames`-keyframe problem on a 3x3-room floor at 80x60 (the
    keyframe spacing of the 2000-keyframe floor)."""
    chunks = make_batch_chunks(count=num_chunks, config=3)
    g = make_global(global_frames, "floor3", config=3, outlier_rate=0.10, corr_range=(200, 200),
                    name=f"global{global_frames}", per_pair_streams=True)
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.unique(np.round(np.geomspace(50, global_frames, global_windows)).astype(int))
    wins = []
    for n in sizes:
        s = int(rng.integers(0, global_frames - n + 1))
        wins.append(window(g, s, int(n)))
    return chunks, wins
