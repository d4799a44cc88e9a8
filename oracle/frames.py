"""Per-frame data for the dense terms (paper Sec. 4.1.1: camera-space positions
P and normals N of the downsampled depth are computed and cached per frame;
Sec. 4.3: the photometric term works on the gradient of the luminance).

For each frame this module computes, in FP64, by the plain definitions:

* P(x,y) = D(x,y) * ((x-cx)/fx, (y-cy)/fy, 1), pixel centres at integer (x,y);
  a depth is valid when finite and within [depth_min, depth_max] (the depth as
  given, compared exactly).
* N(x,y) = normalised cross product of the central differences
  (P(x+1,y)-P(x-1,y)) x (P(x,y+1)-P(x,y-1)), oriented towards the camera
  (N.P < 0).  Invalid on the image border, where the centre or any of the four
  neighbours has invalid depth, or where the cross product vanishes.
* G(x,y) = |grad L| with central differences ((L(x+1)-L(x-1))/2, same in y),
  the intensity taken as luminance.  Invalid on the border or next to a
  non-finite intensity.

Beside the values it exports, per pixel, two numbers that say how far a
computation of the normal in binary32 (the precision of the GPU kernels) can be
from the FP64 one, so that a test can tell a decision within rounding from a
wrong one:

* ``N_sigma`` -- a first-order bound on the error of a binary32 normal (any
  evaluation order): the positions carry a relative error of about 2u (u =
  2^-24, the ray coefficient and the product are rounded), so a central
  difference d of two positions P carries about 4u|P| + u|d| absolutely; the
  cross product's direction then moves by the sum of the two relative errors
  divided by the sine of the angle between d1 and d2; normalising adds a few u.
* ``flip_margin`` -- |N.P| / |P|, how far the orientation decision N.P < 0 is
  from its threshold.
"""
from dataclasses import dataclass

import numpy as np

U32 = 2.0 ** -24   # unit roundoff of binary32


@dataclass
class FrameData:
    P: np.ndarray           # f64 [H,W,3]
    N: np.ndarray           # f64 [H,W,3]   (NaN where invalid)
    G: np.ndarray           # f64 [H,W]     (NaN where invalid)
    depth_ok: np.ndarray    # bool [H,W]
    normal_ok: np.ndarray   # bool [H,W]  (implies depth_ok)
    grad_ok: np.ndarray     # bool [H,W]
    N_sigma: np.ndarray     # f64 [H,W]  binary32 rounding bound of N (0 where invalid)
    flip_margin: np.ndarray  # f64 [H,W] |N.P|/|P| (inf where invalid)


def prepare_frame(depth, intensity, intr, params):
    fx, fy, cx, cy, W, H = intr
    D = np.asarray(depth, np.float32).astype(np.float64)
    L = np.asarray(intensity, np.float32).astype(np.float64)
    with np.errstate(invalid="ignore"):
        dok = np.isfinite(D) & (D >= params.depth_min) & (D <= params.depth_max)

    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    Dz = np.where(dok, D, 0.0)
    P = np.stack([Dz * ((xs[None, :] - cx) / fx), Dz * ((ys[:, None] - cy) / fy), Dz], axis=-1)

    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = True
    nb = np.zeros((H, W), bool)
    nb[1:-1, 1:-1] = dok[1:-1, 1:-1] & dok[1:-1, 2:] & dok[1:-1, :-2] & dok[2:, 1:-1] & dok[:-2, 1:-1]

    e1 = np.zeros((H, W, 3))
    e2 = np.zeros((H, W, 3))
    e1[1:-1, 1:-1] = P[1:-1, 2:] - P[1:-1, :-2]
    e2[1:-1, 1:-1] = P[2:, 1:-1] - P[:-2, 1:-1]
    c = np.cross(e1, e2)
    cl = np.linalg.norm(c, axis=-1)
    nok = nb & (cl > 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        N = c / cl[..., None]
        s = np.einsum("hwa,hwa->hw", N, P)
    flip = s > 0
    N = np.where(flip[..., None], -N, N)
    N = np.where(nok[..., None], N, np.nan)

    with np.errstate(invalid="ignore", divide="ignore"):
        l1 = np.linalg.norm(e1, axis=-1)
        l2 = np.linalg.norm(e2, axis=-1)
        Pn = np.linalg.norm(P, axis=-1)
        sin = cl / (l1 * l2)
        rel1 = (4.0 * Pn + l1) / l1
        rel2 = (4.0 * Pn + l2) / l2
        sigma = U32 * ((rel1 + rel2 + 2.0) / sin + 6.0)
        flip_margin = np.abs(s) / Pn
    N_sigma = np.where(nok, sigma, 0.0)
    flip_margin = np.where(nok, flip_margin, np.inf)

    # luminance gradient magnitude
    lok = np.isfinite(L)
    gok = np.zeros((H, W), bool)
    gok[1:-1, 1:-1] = (lok[1:-1, 1:-1] & lok[1:-1, 2:] & lok[1:-1, :-2] & lok[2:, 1:-1] & lok[:-2, 1:-1])
    G = np.full((H, W), np.nan)
    with np.errstate(invalid="ignore"):
        gx = 0.5 * (L[1:-1, 2:] - L[1:-1, :-2])
        gy = 0.5 * (L[2:, 1:-1] - L[:-2, 1:-1])
        G[1:-1, 1:-1] = np.sqrt(gx * gx + gy * gy)
    G = np.where(gok, G, np.nan)
    return FrameData(P=P, N=N, G=G, depth_ok=dok, normal_ok=nok & inner, grad_ok=gok, N_sigma=N_sigma,
                     flip_margin=flip_margin)


def prepare_frames(depth, intensity, intr, params):
    return [prepare_frame(depth[f], intensity[f], intr, params) for f in range(depth.shape[0])]
