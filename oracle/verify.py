"""Dense two-sided verification of frame pairs (paper Sec. 4.1.1, "Dense
Verification").

Test infrastructure: the plain reference of the GPU path's verification.

For frames f_a, f_b and the relative transform T_ba = T_b^-1 T_a, each pixel of
f_a with a valid normal is associated with the nearest pixel of f_b under the
dense term's rules (oracle.terms.associate32: the same FP32 decisions, tau_dist,
tau_normal) and must also be photo-consistent: |C_a(x,y) - C_b(x',y')| < tau_c
(FP32).  The re-projection error of a valid association is |T_ba p - q| (FP64).
A pair is valid when, in both directions, at least min_frac * W * H associations
are valid and their mean error is at most max_err.
"""
import numpy as np

from .frames import prepare_frame
from .pairs import relative_pose64
from .terms import associate32, decision_constants

f32 = np.float32


def verify_direction(fa, fb, Ca, Cb, Ta, Tb, intr, params, tau_c):
    """(error sum, count) of the valid associations from frame a to frame b."""
    W, H = intr[4], intr[5]
    R, t = relative_pose64(Ta, Tb)
    intr32, consts32 = decision_constants(intr, params)
    geo, _, xh, yh, _, _ = associate32(fa, fb, R.astype(f32), t.astype(f32), intr32, consts32, W, H)
    ca = np.asarray(Ca, f32).reshape(-1)
    cb = np.asarray(Cb, f32)[yh, xh]
    with np.errstate(invalid="ignore"):
        ok = geo & (np.abs(ca - cb) < f32(tau_c))
    c = fa.P.reshape(-1, 3)[ok] @ R.T + t
    q = fb.P[yh[ok], xh[ok]]
    return float(np.linalg.norm(c - q, axis=1).sum()), int(ok.sum())


def verify_pairs(depth, intensity, intr, pairs, poses, params, tau_c=0.1, max_err=0.075, min_frac=0.02):
    """Per pair: stats (err_ab, n_ab, err_ba, n_ba) and validity."""
    frames = {}
    stats = np.zeros((len(pairs), 4))
    valid = np.zeros(len(pairs), bool)
    min_count = min_frac * intr[4] * intr[5]
    for k, (a, b) in enumerate(pairs):
        for f in (a, b):
            if f not in frames:
                frames[f] = prepare_frame(depth[f], intensity[f], intr, params)
        e0, n0 = verify_direction(frames[a], frames[b], intensity[a], intensity[b], poses[a], poses[b], intr, params,
                                  tau_c)
        e1, n1 = verify_direction(frames[b], frames[a], intensity[b], intensity[a], poses[b], poses[a], intr, params,
                                  tau_c)
        stats[k] = (e0, n0, e1, n1)
        valid[k] = all(n >= min_count and n > 0 and e / n <= max_err for e, n in ((e0, n0), (e1, n1)))
    return stats, valid
