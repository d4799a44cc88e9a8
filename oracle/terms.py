"""Residuals and Jacobians of the alignment energy (paper Sec. 4.3).

Poses T_f = (R_f, t_f) map camera f to world; a perturbation acts on the right,
T_f <- T_f Exp(xi_f) with xi_f = (omega_f, v_f).  Each function returns the
residuals and their Jacobians with respect to the perturbations of both frames
of a pair, all derived here directly from the energy definitions (no adjoint
shortcut), in FP64.

Sparse term:  r = T_i p - T_j q in R^3 (world), for a correspondence between
point p of frame i and point q of frame j.
  d r / d xi_i = R_i [-[p]_x | I],   d r / d xi_j = -R_j [-[q]_x | I].

Dense geometric term (point-to-plane):  with c = T_j^-1 T_i d, m = R_ji n and
q the back-projected depth of frame j at the nearest pixel to pi(c),
  r_g = n^T (d - T_i^-1 T_j q) = m^T (c - q);
  d r_g / d xi_j = [(m x q)^T, -m^T],   d r_g / d xi_i = [((T_ij q) x n)^T, n^T],
with the association (the pixel of q) held fixed.

Dense photometric term:  r_p = G_i(x,y) - G_j(pi(c)), G_j read by bilinear
interpolation; with a = Jpi(c)^T grad G_j(pi(c)),
  d r_p / d xi_j = [(c x a)^T, a^T],   d r_p / d xi_i = [(b x d)^T, -b^T],  b = R_ji^T a,
where grad G_j is the analytic derivative of the bilinear interpolant.

Dense association (Sec. 4.3: projections that leave the frame are ignored;
ICP-like distance and normal pruning), the plain rule in FP64: nearest pixel
(floor(u+1/2), floor(v+1/2)) inside the image with a valid normal,
|c - q| < tau_dist and m.N_j > tau_normal; the photometric residual is used only
where the geometric association holds, G_i(x,y) is valid and the four bilinear
taps (floor(u), floor(v)) .. +1 are inside the image and valid.  ``associate``
also exports the margin of every decision and a first-order bound on how far a
binary32 evaluation of the same quantity can be from the FP64 one (see there).
"""
import numpy as np

from .pairs import relative_pose64


def _cross(a, b):
    return np.cross(a, b)


# ----------------------------------------------------------------------------- sparse

def skew_rows(v):
    """[n,3,3] cross-product matrices of the rows of v."""
    z = np.zeros(len(v))
    return np.stack([np.stack([z, -v[:, 2], v[:, 1]], -1),
                     np.stack([v[:, 2], z, -v[:, 0]], -1),
                     np.stack([-v[:, 1], v[:, 0], z], -1)], axis=1)


def sparse_terms(Ti, Tj, p, q):
    """Residuals [n,3] and Jacobians Ji, Jj [n,3,6] for correspondences (p in i, q in j)."""
    Ri, ti = Ti[:3, :3], Ti[:3, 3]
    Rj, tj = Tj[:3, :3], Tj[:3, 3]
    p = np.asarray(p, np.float64).reshape(-1, 3)
    q = np.asarray(q, np.float64).reshape(-1, 3)
    r = p @ Ri.T + ti - (q @ Rj.T + tj)
    I3 = np.broadcast_to(np.eye(3), (len(p), 3, 3))
    Ap = np.concatenate([-skew_rows(p), I3], axis=2)
    Aq = np.concatenate([-skew_rows(q), I3], axis=2)
    Ji = np.einsum("ab,nbk->nak", Ri, Ap)
    Jj = -np.einsum("ab,nbk->nak", Rj, Aq)
    return r, Ji, Jj


# ----------------------------------------------------------------------------- dense

U32 = 2.0 ** -24   # unit roundoff of binary32


def _half_margin(u):
    """Distance of u to the nearest k + 1/2: where floor(u + 1/2) changes."""
    with np.errstate(invalid="ignore"):
        return np.abs(u - np.floor(u) - 0.5)


def _int_margin(u):
    """Distance of u to the nearest integer: where floor(u) changes."""
    with np.errstate(invalid="ignore"):
        return np.abs(u - np.round(u))


def associate(fi, fj, R, t, intr, params):
    """Association decisions of pair job i -> j (source pixels of frame i) at the
    relative pose T_ji = (R, t), FP64, plain rule:

      source pixel with a valid normal: d = P_i(x,y), n = N_i(x,y);
      c = R d + t, m = R n; in front: c_z > 0;
      u = fx c_x / c_z + cx, v = fy c_y / c_z + cy;
      nearest pixel (xh, yh) = (floor(u + 1/2), floor(v + 1/2)) in [0,W-1] x [0,H-1]
      with a valid normal; q = P_j(xh, yh);
      geometric: |c - q| < tau_dist and m . N_j(xh, yh) > tau_normal;
      photometric: geometric, G_i(x,y) valid, (x0, y0) = (floor(u), floor(v)) in
      [0,W-2] x [0,H-2] and the four taps of G_j at x0..x0+1, y0..y0+1 valid.

    Returns a dict of flat [H*W] arrays: masks 'geo', 'photo'; indices 'xh', 'yh',
    'x0', 'y0' (0 where unused); and for every decision its margin with the
    binary32 rounding bound of the quantity it tests ('m_*' and 's_*'):

      front    c_z                      s_c  = u (8 |d|_1 + 6 |t|_inf + 2 |c|_inf)
      half_u/v distance of u (v) to the nearest half-integer (nearest-pixel choice,
               in-image test)          s_u  = fx s_c (1 + |c_x/c_z|) / |c_z|
                                                 + u (4 |u - cx| + 3 |u| + |cx| + 1)
      int_u/v  distance of u (v) to the nearest integer (bilinear footprint)
      dist     | |c - q| - tau_dist |  s_dist = sqrt(3) (s_c + 3 u |q|_inf) + 4 u tau_dist
      normal   | m.N_j - tau_normal |  s_n  = N_sigma(i) + N_sigma(j) + u (10 + tau_normal)
      flip     orientation margins of the source and target normals (frames.py)

    s_c follows the rounding of d = (kx D, ky D, D) (kx itself rounded), of R and t,
    and of three fused multiply-adds per row; s_u that of 1/c_z, the product fx c_x,
    the final fused multiply-add and the addition of 1/2 before the floor.  A
    binary32 decision can differ from this one only where a margin is within its
    bound; ``near_decisions`` flags those pixels."""
    fx, fy, cx, cy, W, H = intr
    d = fi.P.reshape(-1, 3)
    n = fi.N.reshape(-1, 3)
    src_ok = fi.normal_ok.reshape(-1)
    with np.errstate(all="ignore"):
        c = d @ R.T + t
        m = n @ R.T
        front = c[:, 2] > 0
        u = fx * c[:, 0] / c[:, 2] + cx
        v = fy * c[:, 1] / c[:, 2] + cy
        xf = np.floor(u + 0.5)
        yf = np.floor(v + 0.5)
        inb = front & (xf >= 0) & (xf <= W - 1) & (yf >= 0) & (yf <= H - 1)
        ok = src_ok & inb
        xh = np.where(ok, xf, 0).astype(np.int64)
        yh = np.where(ok, yf, 0).astype(np.int64)
        ok &= fj.normal_ok[yh, xh]
        q = fj.P[yh, xh]
        Nj = fj.N[yh, xh]
        dist = np.linalg.norm(c - q, axis=1)
        dn = np.einsum("na,na->n", m, Nj)
        geo = ok & (dist < params.tau_dist) & (dn > params.tau_normal)
        x0f = np.floor(u)
        y0f = np.floor(v)
        inb2 = (x0f >= 0) & (x0f <= W - 2) & (y0f >= 0) & (y0f <= H - 2)
        ph = geo & inb2 & fi.grad_ok.reshape(-1)
        x0 = np.where(ph, x0f, 0).astype(np.int64)
        y0 = np.where(ph, y0f, 0).astype(np.int64)
        gj = fj.grad_ok
        ph &= gj[y0, x0] & gj[y0, x0 + 1] & gj[y0 + 1, x0] & gj[y0 + 1, x0 + 1]

        # margins and binary32 rounding bounds
        s_c = U32 * (8.0 * np.abs(d).sum(axis=1) + 6.0 * np.abs(t).max() + 2.0 * np.abs(c).max(axis=1))
        az = np.abs(c[:, 2])
        s_u = fx * s_c * (1.0 + np.abs(c[:, 0] / c[:, 2])) / az + U32 * (4 * np.abs(u - cx) + 3 * np.abs(u) + abs(cx) + 1)
        s_v = fy * s_c * (1.0 + np.abs(c[:, 1] / c[:, 2])) / az + U32 * (4 * np.abs(v - cy) + 3 * np.abs(v) + abs(cy) + 1)
        s_dist = np.sqrt(3.0) * (s_c + 3.0 * U32 * np.abs(q).max(axis=1)) + 4.0 * U32 * params.tau_dist
        s_n = fi.N_sigma.reshape(-1) + fj.N_sigma[yh, xh] + U32 * (10.0 + abs(params.tau_normal))
        m_flip = np.minimum(fi.flip_margin.reshape(-1), fj.flip_margin[yh, xh])
        s_flip = fi.N_sigma.reshape(-1) + fj.N_sigma[yh, xh] + 4.0 * U32
    return {"geo": geo, "photo": ph, "xh": xh, "yh": yh, "x0": x0, "y0": y0, "u": u, "v": v,
            "src_ok": src_ok, "target_ok": ok,
            "m_front": c[:, 2], "s_c": s_c,
            "m_half_u": _half_margin(u), "m_half_v": _half_margin(v), "s_u": s_u, "s_v": s_v,
            "m_int_u": _int_margin(u), "m_int_v": _int_margin(v),
            "m_dist": np.abs(dist - params.tau_dist), "s_dist": s_dist,
            "m_normal": np.abs(dn - params.tau_normal), "s_n": s_n,
            "m_flip": m_flip, "s_flip": s_flip}


def near_decisions(a, k=2.0):
    """Pixels whose geometric / photometric decision lies within k times the
    binary32 rounding bound of one of its tests (see ``associate``): there a
    binary32 evaluation may decide either way.  Returns (near_geo, near_photo)."""
    with np.errstate(invalid="ignore"):
        n_geo = a["src_ok"] & (
            (np.abs(a["m_front"]) <= k * a["s_c"])
            | (a["m_half_u"] <= k * a["s_u"]) | (a["m_half_v"] <= k * a["s_v"])
            | (a["target_ok"] & ((a["m_dist"] <= k * a["s_dist"]) | (a["m_normal"] <= k * a["s_n"])
                                 | (a["m_flip"] <= k * a["s_flip"]))))
        n_ph = n_geo | (a["geo"] & ((a["m_int_u"] <= k * a["s_u"]) | (a["m_int_v"] <= k * a["s_v"])))
    return n_geo, n_ph


def dense_terms(fi, fj, Ti, Tj, intr, params, assoc=None):
    """Geometric and photometric residuals/Jacobians of pair job i -> j.

    The association is decided at (Ti, Tj) unless `assoc` (a previous result of
    this function) is given, in which case its pixels are reused unchanged.
    Returns dict with 'rg' [ng], 'Jg_i', 'Jg_j' [ng,6], 'rp' [np], 'Jp_i', 'Jp_j' [np,6],
    and the decision masks/indices."""
    fx, fy, cx, cy, W, H = intr
    R, t = relative_pose64(Ti, Tj)
    asc = associate(fi, fj, R, t, intr, params) if assoc is None else assoc
    geo, ph, xh, yh, x0, y0 = (asc[k] for k in ("geo", "photo", "xh", "yh", "x0", "y0"))

    d_all = fi.P.reshape(-1, 3)
    n_all = fi.N.reshape(-1, 3)
    # geometric
    d = d_all[geo]
    n = n_all[geo]
    c = d @ R.T + t
    m = n @ R.T
    q = fj.P[yh[geo], xh[geo]]
    rg = np.einsum("na,na->n", m, c - q)
    Jg_j = np.concatenate([_cross(m, q), -m], axis=1)
    Tij_q = (q - t) @ R          # R^T (q - t)
    Jg_i = np.concatenate([_cross(Tij_q, n), n], axis=1)

    # photometric
    d = d_all[ph]
    c = d @ R.T + t
    X0 = x0[ph]
    Y0 = y0[ph]
    u = fx * c[:, 0] / c[:, 2] + cx
    v = fy * c[:, 1] / c[:, 2] + cy
    al = u - X0
    be = v - Y0
    G = fj.G
    g00, g10 = G[Y0, X0], G[Y0, X0 + 1]
    g01, g11 = G[Y0 + 1, X0], G[Y0 + 1, X0 + 1]
    Gj = (1 - al) * (1 - be) * g00 + al * (1 - be) * g10 + (1 - al) * be * g01 + al * be * g11
    gu = (1 - be) * (g10 - g00) + be * (g11 - g01)
    gv = (1 - al) * (g01 - g00) + al * (g11 - g10)
    Gi = fi.G.reshape(-1)[ph]
    rp = Gi - Gj
    iz = 1.0 / c[:, 2]
    a = np.stack([gu * fx * iz, gv * fy * iz, -(gu * fx * c[:, 0] + gv * fy * c[:, 1]) * iz * iz], axis=1)
    Jp_j = np.concatenate([_cross(c, a), a], axis=1)
    b = a @ R                    # R^T a
    Jp_i = np.concatenate([_cross(b, d), -b], axis=1)
    out = dict(asc)
    out.update({"rg": rg, "Jg_i": Jg_i, "Jg_j": Jg_j, "rp": rp, "Jp_i": Jp_i, "Jp_j": Jp_j,
                "u_photo": u, "v_photo": v})
    return out
