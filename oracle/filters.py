"""Key-point correspondence filter and surface-area filter (paper Sec. 4.1.1).

Test infrastructure: the plain FP64 reference of the GPU path's filters.

Key-point filter, per frame pair, with the candidates in their given order
(the paper's order of match distance): candidates are added one at a time; after
each addition, while the current set has at least three correspondences, the
rigid transform q = R p + t with the least RMSD over the set is computed by the
Kabsch/Umeyama method, and the set is checked: the largest residual |R p + t - q|
must be at most max_res, and the transform must be well determined -- the
condition numbers of the covariance of the p's, of the q's, and of the
cross-covariance must be at most max_cond.  While a check fails, the
correspondence with the largest residual is removed.  A pair keeps its final set
only if that set has at least min_count correspondences and passes both checks.

Condition number (reading of "condition analysis"), two modes: mode 0 (the
default) the ratio of the largest to the second largest eigenvalue of each 3x3
covariance, and of the largest to the second largest singular value of the
cross-covariance -- it detects point sets on a line, the ambiguity the filter
exists for, and keeps planar sets, which determine a rigid transform fine; mode 1
the plain definition, largest over smallest, which also rejects planar sets.

Surface-area filter: for the kept p's and q's separately, the points are
projected onto the plane of their two principal axes (covariance eigenvectors
of the two largest eigenvalues); the area is the product of the extents along
those two axes (the box aligned with the principal axes).  The pair is discarded
if either area is below min_area.
"""
import numpy as np


def kabsch(P, Q):
    """R, t minimising sum |R p + t - q|^2 (rows of P, Q)."""
    pm, qm = P.mean(axis=0), Q.mean(axis=0)
    H = (P - pm).T @ (Q - qm)
    U, _, Vt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ np.diag([1.0, 1.0, d]) @ U.T
    return R, qm - R @ pm


def condition_numbers(P, Q, mode=0):
    """Largest / second-largest (mode 0) or largest / smallest (mode 1) eigenvalue
    of cov(P) and cov(Q), and the same ratio of the singular values of the
    cross-covariance (inf if undefined)."""
    pm, qm = P.mean(axis=0), Q.mean(axis=0)
    n = len(P)
    ratio = lambda a, b: a / b if b > 0 else np.inf
    ep = np.linalg.eigvalsh((P - pm).T @ (P - pm) / n)[::-1]
    eq = np.linalg.eigvalsh((Q - qm).T @ (Q - qm) / n)[::-1]
    sv = np.linalg.svd((P - pm).T @ (Q - qm) / n, compute_uv=False)
    lo = 2 if mode else 1
    return ratio(ep[0], ep[lo]), ratio(eq[0], eq[lo]), ratio(sv[0], sv[lo])


def keypoint_filter(P, Q, max_res=0.02, max_cond=100.0, min_count=5, cond_mode=0):
    """Indices (into P, Q) of the correspondences the filter keeps, in order; an
    empty array when the pair is discarded."""
    P = np.asarray(P, np.float64)
    Q = np.asarray(Q, np.float64)
    cur = []
    ok = False
    for c in range(len(P)):
        cur.append(c)
        ok = False
        while len(cur) >= 3:
            R, t = kabsch(P[cur], Q[cur])
            res = np.linalg.norm(P[cur] @ R.T + t - Q[cur], axis=1)
            stable = max(condition_numbers(P[cur], Q[cur], cond_mode)) <= max_cond
            if res.max() <= max_res and stable:
                ok = True
                break
            del cur[int(np.argmax(res))]
    if len(cur) < max(min_count, 3) or not ok:
        return np.zeros(0, np.int64)
    return np.array(cur, np.int64)


def principal_area(X):
    """Area of the box spanned by X along its two principal axes."""
    X = np.asarray(X, np.float64)
    Xc = X - X.mean(axis=0)
    w, V = np.linalg.eigh(Xc.T @ Xc / len(X))
    A = Xc @ V[:, [2, 1]]   # the two largest eigenvalues' axes
    ext = A.max(axis=0) - A.min(axis=0)
    return float(ext[0] * ext[1])


def filter_pairs(ci, cj, p, q, max_res=0.02, max_cond=100.0, min_count=5, min_area=0.032, cond_mode=0):
    """Both filters over all correspondences, grouped by unordered frame pair in
    input order.  Returns a keep mask [M]."""
    ci = np.asarray(ci)
    cj = np.asarray(cj)
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    lo, hi = np.minimum(ci, cj), np.maximum(ci, cj)
    sw = ci > cj
    P = np.where(sw[:, None], q, p)    # the lower frame's point
    Q = np.where(sw[:, None], p, q)
    keep = np.zeros(len(ci), bool)
    keys = lo.astype(np.int64) * (int(max(hi.max(initial=0), 0)) + 1) + hi
    for key in np.unique(keys):
        idx = np.nonzero(keys == key)[0]   # input order
        kept = keypoint_filter(P[idx], Q[idx], max_res, max_cond, min_count, cond_mode)
        if len(kept) == 0:
            continue
        if principal_area(P[idx[kept]]) < min_area or principal_area(Q[idx[kept]]) < min_area:
            continue
        keep[idx[kept]] = True
    return keep
