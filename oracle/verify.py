"""Dense two-sided verification of frame pairs (paper Sec. 4.1.1, "Dense
Verification").

Test infrastructure: the plain reference of the GPU path's verification.

For frames f_a, f_b and the relative transform T_ba = T_b^-1 T_a, each pixel of
f_a with a valid normal is associated with the nearest pixel of f_b under the
dense term's rules (oracle.terms.associate: FP64, tau_dist, tau_normal) and must
also be photo-consistent: |C_a(x,y) - C_b(x',y')| < tau_c.  The re-projection
error of a valid association is |T_ba p - q|.  A pair is valid when, in both
directions, at least min_frac * W * H associations are valid and their mean
error is at most max_err.

Beside the counts and sums it reports, per direction, how many candidates lie
within the binary32 rounding bound of one of their tests
(``terms.near_decisions``, and |C_a - C_b| within that bound of tau_c): a
binary32 evaluation may decide those either way, or pick the neighbouring target
pixel, so a count can differ by at most that many and an error sum by at most
that many times tau_dist (the largest error a valid association can have).
"""
import numpy as np

from .frames import U32, prepare_frame
from .pairs import relative_pose64
from .terms import associate, near_decisions


def verify_direction(fa, fb, Ca, Cb, Ta, Tb, intr, params, tau_c, k_near=2.0):
    """(error sum, count, near count) of the valid associations from frame a to
    frame b."""
    R, t = relative_pose64(Ta, Tb)
    a = associate(fa, fb, R, t, intr, params)
    geo, xh, yh = a["geo"], a["xh"], a["yh"]
    ca = np.asarray(Ca, np.float32).astype(np.float64).reshape(-1)
    cb = np.asarray(Cb, np.float32).astype(np.float64)[yh, xh]
    with np.errstate(invalid="ignore"):
        dc = np.abs(ca - cb)
        ok = geo & (dc < tau_c)
        near_geo, _ = near_decisions(a, k_near)
        near = near_geo | (geo & (np.abs(dc - tau_c) <= k_near * 2.0 * U32 * (np.abs(ca) + np.abs(cb) + tau_c)))
    c = fa.P.reshape(-1, 3)[ok] @ R.T + t
    q = fb.P[yh[ok], xh[ok]]
    return float(np.linalg.norm(c - q, axis=1).sum()), int(ok.sum()), int(near.sum())


def verify_pairs(depth, intensity, intr, pairs, poses, params, tau_c=0.1, max_err=0.075, min_frac=0.02):
    """Per pair: stats (err_ab, n_ab, err_ba, n_ba), validity, and the near-decision
    counts of both directions (near [P,2])."""
    frames = {}
    stats = np.zeros((len(pairs), 4))
    valid = np.zeros(len(pairs), bool)
    near = np.zeros((len(pairs), 2), np.int64)
    min_count = min_frac * intr[4] * intr[5]
    for k, (a, b) in enumerate(pairs):
        for f in (a, b):
            if f not in frames:
                frames[f] = prepare_frame(depth[f], intensity[f], intr, params)
        e0, n0, k0 = verify_direction(frames[a], frames[b], intensity[a], intensity[b], poses[a], poses[b], intr,
                                          params, tau_c)
        e1, n1, k1 = verify_direction(frames[b], frames[a], intensity[b], intensity[a], poses[b], poses[a], intr,
                                          params, tau_c)
        stats[k] = (e0, n0, e1, n1)
        near[k] = (k0, k1)
        valid[k] = all(n >= min_count and n > 0 and e / n <= max_err for e, n in ((e0, n0), (e1, n1)))
    return stats, valid, near
