"""Per-frame data for the dense terms (paper Sec. 4.1.1: camera-space positions
P and normals N of the downsampled depth are computed and cached per frame;
Sec. 4.3: the photometric term works on the gradient of the luminance).

For each frame this module computes, in FP64:

* P(x,y) = D(x,y) * ((x-cx)/fx, (y-cy)/fy, 1), pixel centres at integer (x,y);
  a depth is valid when finite and within [depth_min, depth_max].
* N(x,y) = normalised cross product of the central differences
  (P(x+1,y)-P(x-1,y)) x (P(x,y+1)-P(x,y-1)), oriented towards the camera
  (N.P < 0).  Invalid on the image border, where the centre or any of the four
  neighbours has invalid depth, or where the cross product vanishes.
* G(x,y) = |grad L| with central differences ((L(x+1)-L(x-1))/2, same in y),
  the intensity taken as luminance.  Invalid on the border or next to a
  non-finite intensity.

Validity is a decision taken in FP32 (the precision of the GPU kernels), with
this fixed operation sequence and no fused multiply-add:
  kx = fl32((x - cx) / fx)  [FP64 then rounded],  P32 = (kx*D, ky*D, D);
  d1 = P32(x+1,y) - P32(x-1,y),  d2 = P32(x,y+1) - P32(x,y-1);
  c = (d1.y*d2.z - d1.z*d2.y, d1.z*d2.x - d1.x*d2.z, d1.x*d2.y - d1.y*d2.x);
  l2 = (c.x*c.x + c.y*c.y) + c.z*c.z,  valid iff l2 > 0;
  N32 = c / sqrt(l2) (three divisions),  flip iff (N.x*P.x + N.y*P.y) + N.z*P.z > 0.
P32 and N32 also enter the per-pixel association decisions of the dense terms.
"""
from dataclasses import dataclass

import numpy as np

f32 = np.float32


@dataclass
class FrameData:
    P: np.ndarray        # f64 [H,W,3]
    N: np.ndarray        # f64 [H,W,3]   (NaN where invalid)
    G: np.ndarray        # f64 [H,W]     (NaN where invalid)
    P32: np.ndarray      # f32 [H,W,3]
    N32: np.ndarray      # f32 [H,W,3]
    depth_ok: np.ndarray  # bool [H,W]
    normal_ok: np.ndarray  # bool [H,W]  (implies depth_ok)
    grad_ok: np.ndarray   # bool [H,W]


def ray_coeffs32(W, H, fx, fy, cx, cy):
    kx = ((np.arange(W, dtype=np.float64) - cx) / fx).astype(f32)
    ky = ((np.arange(H, dtype=np.float64) - cy) / fy).astype(f32)
    return kx, ky


def prepare_frame(depth, intensity, intr, params):
    fx, fy, cx, cy, W, H = intr
    D32 = np.asarray(depth, f32)
    L = np.asarray(intensity, np.float64)
    D = D32.astype(np.float64)
    with np.errstate(invalid="ignore"):
        dok = np.isfinite(D32) & (D32 >= f32(params.depth_min)) & (D32 <= f32(params.depth_max))

    # FP64 positions
    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    Dz = np.where(dok, D, 0.0)
    P = np.stack([Dz * ((xs[None, :] - cx) / fx), Dz * ((ys[:, None] - cy) / fy), Dz], axis=-1)

    # FP32 decision positions
    kx, ky = ray_coeffs32(W, H, fx, fy, cx, cy)
    D32z = np.where(dok, D32, f32(0))
    P32 = np.stack([kx[None, :] * D32z, ky[:, None] * D32z, D32z], axis=-1).astype(f32)

    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = True
    nb = np.zeros((H, W), bool)
    nb[1:-1, 1:-1] = dok[1:-1, 1:-1] & dok[1:-1, 2:] & dok[1:-1, :-2] & dok[2:, 1:-1] & dok[:-2, 1:-1]

    # FP32 normal decision, fixed operation order
    d1 = np.zeros((H, W, 3), f32)
    d2 = np.zeros((H, W, 3), f32)
    d1[1:-1, 1:-1] = P32[1:-1, 2:] - P32[1:-1, :-2]
    d2[1:-1, 1:-1] = P32[2:, 1:-1] - P32[:-2, 1:-1]
    c32 = np.stack([d1[..., 1] * d2[..., 2] - d1[..., 2] * d2[..., 1],
                    d1[..., 2] * d2[..., 0] - d1[..., 0] * d2[..., 2],
                    d1[..., 0] * d2[..., 1] - d1[..., 1] * d2[..., 0]], axis=-1).astype(f32)
    l2 = (c32[..., 0] * c32[..., 0] + c32[..., 1] * c32[..., 1]) + c32[..., 2] * c32[..., 2]
    nok = nb & (l2 > f32(0))
    with np.errstate(invalid="ignore", divide="ignore"):
        nrm = np.sqrt(l2)
        N32 = np.stack([c32[..., 0] / nrm, c32[..., 1] / nrm, c32[..., 2] / nrm], axis=-1).astype(f32)
        s32 = (N32[..., 0] * P32[..., 0] + N32[..., 1] * P32[..., 1]) + N32[..., 2] * P32[..., 2]
    flip = s32 > f32(0)
    N32 = np.where(flip[..., None], -N32, N32).astype(f32)
    N32 = np.where(nok[..., None], N32, f32(np.nan)).astype(f32)

    # FP64 normal values, same orientation decision
    e1 = np.zeros((H, W, 3))
    e2 = np.zeros((H, W, 3))
    e1[1:-1, 1:-1] = P[1:-1, 2:] - P[1:-1, :-2]
    e2[1:-1, 1:-1] = P[2:, 1:-1] - P[:-2, 1:-1]
    c = np.cross(e1, e2)
    with np.errstate(invalid="ignore", divide="ignore"):
        N = c / np.linalg.norm(c, axis=-1, keepdims=True)
    N = np.where(flip[..., None], -N, N)
    N = np.where(nok[..., None], N, np.nan)

    # luminance gradient magnitude
    lok = np.isfinite(L)
    gok = np.zeros((H, W), bool)
    gok[1:-1, 1:-1] = (lok[1:-1, 1:-1] & lok[1:-1, 2:] & lok[1:-1, :-2] & lok[2:, 1:-1] & lok[:-2, 1:-1])
    G = np.full((H, W), np.nan)
    gx = 0.5 * (L[1:-1, 2:] - L[1:-1, :-2])
    gy = 0.5 * (L[2:, 1:-1] - L[:-2, 1:-1])
    G[1:-1, 1:-1] = np.sqrt(gx * gx + gy * gy)
    G = np.where(gok, G, np.nan)
    return FrameData(P=P, N=N, G=G, P32=P32, N32=N32, depth_ok=dok, normal_ok=nok & inner, grad_ok=gok)


def prepare_frames(depth, intensity, intr, params):
    return [prepare_frame(depth[f], intensity[f], intr, params) for f in range(depth.shape[0])]
