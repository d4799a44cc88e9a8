"""Frame-pair structure of the energy.

Dense pair set E (paper Sec. 4.3): a pair (i, j) is included when the two
camera viewing directions are within 60 degrees and the frames overlap.  The
paper does not say how overlap is measured; the reading used here is a
frustum test on the initial poses: at least one pixel of a fixed 8x6 grid of
frame i (x = 5+10a, y = 5+10b at 80x60, doubled at 160x120) with valid depth
lands, under T_j^-1 T_i, in front of camera j and inside [0,W-1]x[0,H-1].
One dense pair job per unordered pair, with the lower index as the source
(the dense sums of Sec. 4.3 run over the pixels of frame i only).

The test is a decision taken in FP64 with this fixed operation order and no
fused multiply-add (identical on the GPU):
  R_ji[a][b] = (Rj[0][a]*Ri[0][b] + Rj[1][a]*Ri[1][b]) + Rj[2][a]*Ri[2][b]
  d = t_i - t_j;  t_ji[a] = (Rj[0][a]*d[0] + Rj[1][a]*d[1]) + Rj[2][a]*d[2]
  angle:  (Ri[0][2]*Rj[0][2] + Ri[1][2]*Rj[1][2]) + Ri[2][2]*Rj[2][2] > cos(60 deg)
  point:  p = (((x-cx)/fx)*D, ((y-cy)/fy)*D, D) with D the FP32 depth widened,
          c[a] = ((R_ji[a][0]*p0 + R_ji[a][1]*p1) + R_ji[a][2]*p2) + t_ji[a],
          c2 > 0,  u = ((fx*c0)/c2) + cx in [0, W-1],  v likewise in [0, H-1].

Sparse correspondences (Sec. 4.3, E_sparse) are grouped by unordered frame
pair; a correspondence given as (j, i) with j > i has its two points swapped.
"""
import numpy as np


def relative_pose64(Ti, Tj):
    """T_ji = T_j^-1 T_i (maps camera i into camera j), fixed FP64 operation order."""
    Ri, Rj = Ti[:3, :3], Tj[:3, :3]
    R = np.empty((3, 3))
    for a in range(3):
        for b in range(3):
            R[a, b] = (Rj[0, a] * Ri[0, b] + Rj[1, a] * Ri[1, b]) + Rj[2, a] * Ri[2, b]
    d = Ti[:3, 3] - Tj[:3, 3]
    t = np.empty(3)
    for a in range(3):
        t[a] = (Rj[0, a] * d[0] + Rj[1, a] * d[1]) + Rj[2, a] * d[2]
    return R, t


def grid_points(W, H):
    """The 8x6 overlap-test grid: pixels 5, 15, ..., 75 by 5, 15, ..., 55 at 80x60,
    scaled with the image (x = (5 + 10a) W / 80, y = (5 + 10b) H / 60, integer
    division), so every grid pixel lies inside the image at any size."""
    xs = np.array([(5 + 10 * a) * W // 80 for a in range(8)])
    ys = np.array([(5 + 10 * b) * H // 60 for b in range(6)])
    return xs, ys


def dense_pairs(depth, poses, intr, params):
    """Sorted list of (i, j), i < j, passing the angle and overlap test."""
    fx, fy, cx, cy, W, H = intr
    F = depth.shape[0]
    xs, ys = grid_points(W, H)
    X, Y = np.meshgrid(xs, ys)
    X, Y = X.ravel(), Y.ravel()
    cos_lim = np.cos(np.deg2rad(params.max_angle_deg))
    out = []
    for i in range(F):
        D32 = depth[i][Y, X].astype(np.float32)
        with np.errstate(invalid="ignore"):
            ok = np.isfinite(D32) & (D32.astype(np.float64) >= params.depth_min) & (D32.astype(np.float64) <= params.depth_max)
        D = D32[ok].astype(np.float64)
        p0 = ((X[ok] - cx) / fx) * D
        p1 = ((Y[ok] - cy) / fy) * D
        p2 = D
        Ri = poses[i][:3, :3]
        for j in range(i + 1, F):
            Rj = poses[j][:3, :3]
            dot = (Ri[0, 2] * Rj[0, 2] + Ri[1, 2] * Rj[1, 2]) + Ri[2, 2] * Rj[2, 2]
            if not dot > cos_lim or len(D) == 0:
                continue
            R, t = relative_pose64(poses[i], poses[j])
            c0 = ((R[0, 0] * p0 + R[0, 1] * p1) + R[0, 2] * p2) + t[0]
            c1 = ((R[1, 0] * p0 + R[1, 1] * p1) + R[1, 2] * p2) + t[1]
            c2 = ((R[2, 0] * p0 + R[2, 1] * p1) + R[2, 2] * p2) + t[2]
            with np.errstate(divide="ignore", invalid="ignore"):
                u = ((fx * c0) / c2) + cx
                v = ((fy * c1) / c2) + cy
                hit = (c2 > 0) & (u >= 0) & (u <= W - 1) & (v >= 0) & (v <= H - 1)
            if hit.any():
                out.append((i, j))
    return np.array(out, np.int32).reshape(-1, 2)


def group_correspondences(corr_i, corr_j, p, q, num_frames):
    """Canonical (a<b) grouping: returns (keys [K,2], ptr [K+1], perm, pa, qb) where
    perm is the stable sort of correspondences by (a, b), and pa/qb are the points in
    frames a and b in sorted order."""
    ci = np.asarray(corr_i, np.int64)
    cj = np.asarray(corr_j, np.int64)
    a = np.minimum(ci, cj)
    b = np.maximum(ci, cj)
    swap = ci > cj
    pa = np.where(swap[:, None], q, p)
    qb = np.where(swap[:, None], p, q)
    key = a * num_frames + b
    perm = np.argsort(key, kind="stable")
    ks = key[perm]
    uniq, start = np.unique(ks, return_index=True)
    ptr = np.append(start, len(ks)).astype(np.int64)
    keys = np.stack([uniq // num_frames, uniq % num_frames], axis=1).astype(np.int32)
    return keys, ptr, perm, pa[perm].astype(np.float64), qb[perm].astype(np.float64)


def edge_list(dense, sparse_keys):
    """Sorted union of dense pairs and sparse pair keys, with per-edge flags."""
    allp = {}
    for k, (i, j) in enumerate(dense):
        allp.setdefault((int(i), int(j)), [-1, -1])[0] = k
    for k, (i, j) in enumerate(sparse_keys):
        allp.setdefault((int(i), int(j)), [-1, -1])[1] = k
    keys = sorted(allp)
    edges = np.array(keys, np.int32).reshape(-1, 2)
    dense_idx = np.array([allp[k][0] for k in keys], np.int64)
    sparse_idx = np.array([allp[k][1] for k in keys], np.int64)
    return edges, dense_idx, sparse_idx
