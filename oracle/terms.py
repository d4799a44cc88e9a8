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

Dense association (Sec. 4.3: out-of-frame projections are ignored; ICP-like
distance and normal pruning): nearest pixel (floor(u+1/2), floor(v+1/2)) inside
the image with valid depth and normal, |c - q| < tau_dist and m.N_j > tau_normal;
the photometric residual is used only where the geometric association holds,
G_i(x,y) is valid and all four bilinear taps are inside the image and valid.
These decisions are taken in FP32 with the fixed operation sequence of
``associate32``; see that function.
"""
import numpy as np

from .fp32 import fma32
from .pairs import relative_pose64

f32 = np.float32


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

def associate32(fi, fj, R32, t32, intr32, consts32, W, H):
    """FP32 association decisions for pair job i -> j, fixed operation sequence
    with fused multiply-adds (fma(a, b, c) = a*b + c rounded once, oracle.fp32):

      c_a = fma(R_a0, d.x, fma(R_a1, d.y, fma(R_a2, d.z, t_a)))   (row a of R_ji)
      m_a = fma(R_a0, n.x, fma(R_a1, n.y, R_a2*n.z))
      front: c.z > 0;  iz = 1/c.z;  u = fma(fx*c.x, iz, cx),  v = fma(fy*c.y, iz, cy)
      xh = floor(u + 0.5), yh = floor(v + 0.5) in [0,W-1] x [0,H-1]
      e = c - q, fma(e.x, e.x, fma(e.y, e.y, e.z*e.z)) < tau_d2,
      fma(m.x, N.x, fma(m.y, N.y, m.z*N.z)) > tau_n
      photometric: x0 = floor(u), y0 = floor(v) in [0,W-2] x [0,H-2], taps and G_i valid.
    Returns (geo_ok [H*W], photo_ok [H*W], xh, yh, x0, y0) as flat arrays."""
    fx, fy, cx, cy = intr32
    tau_d2, tau_n = consts32
    d = fi.P32.reshape(-1, 3)
    n = fi.N32.reshape(-1, 3)
    src_ok = fi.normal_ok.reshape(-1)
    with np.errstate(all="ignore"):
        c = np.stack([fma32(R32[a, 0], d[:, 0], fma32(R32[a, 1], d[:, 1], fma32(R32[a, 2], d[:, 2], t32[a])))
                      for a in range(3)], axis=1)
        m = np.stack([fma32(R32[a, 0], n[:, 0], fma32(R32[a, 1], n[:, 1], R32[a, 2] * n[:, 2]))
                      for a in range(3)], axis=1)
        front = c[:, 2] > f32(0)
        iz = f32(1) / c[:, 2]
        u = fma32(fx * c[:, 0], iz, cx)
        v = fma32(fy * c[:, 1], iz, cy)
        xf = np.floor(u + f32(0.5))
        yf = np.floor(v + f32(0.5))
        inb = front & (xf >= f32(0)) & (xf <= f32(W - 1)) & (yf >= f32(0)) & (yf <= f32(H - 1))
        ok = src_ok & inb
        xh = np.where(ok, xf, 0).astype(np.int64)
        yh = np.where(ok, yf, 0).astype(np.int64)
        ok &= fj.normal_ok[yh, xh]
        q = fj.P32[yh, xh]
        e = (c - q).astype(f32)
        dist2 = fma32(e[:, 0], e[:, 0], fma32(e[:, 1], e[:, 1], e[:, 2] * e[:, 2]))
        Nj = fj.N32[yh, xh]
        dn = fma32(m[:, 0], Nj[:, 0], fma32(m[:, 1], Nj[:, 1], m[:, 2] * Nj[:, 2]))
        geo = ok & (dist2 < tau_d2) & (dn > tau_n)
        x0f = np.floor(u)
        y0f = np.floor(v)
        inb2 = (x0f >= f32(0)) & (x0f <= f32(W - 2)) & (y0f >= f32(0)) & (y0f <= f32(H - 2))
        ph = geo & inb2 & fi.grad_ok.reshape(-1)
        x0 = np.where(ph, x0f, 0).astype(np.int64)
        y0 = np.where(ph, y0f, 0).astype(np.int64)
        gj = fj.grad_ok
        ph &= gj[y0, x0] & gj[y0, x0 + 1] & gj[y0 + 1, x0] & gj[y0 + 1, x0 + 1]
    return geo, ph, xh, yh, x0, y0


def decision_constants(intr, params):
    fx, fy, cx, cy, W, H = intr
    return (f32(fx), f32(fy), f32(cx), f32(cy)), (f32(params.tau_dist * params.tau_dist), f32(params.tau_normal))


def dense_terms(fi, fj, Ti, Tj, intr, params, assoc=None):
    """Geometric and photometric residuals/Jacobians of pair job i -> j.

    The association is decided at (Ti, Tj) unless `assoc` (a previous result of
    this function) is given, in which case its pixels are reused unchanged.
    Returns dict with 'rg' [ng], 'Jg_i', 'Jg_j' [ng,6], 'rp' [np], 'Jp_i', 'Jp_j' [np,6],
    and the decision masks/indices."""
    fx, fy, cx, cy, W, H = intr
    R, t = relative_pose64(Ti, Tj)
    if assoc is None:
        intr32, consts32 = decision_constants(intr, params)
        geo, ph, xh, yh, x0, y0 = associate32(fi, fj, R.astype(f32), t.astype(f32), intr32, consts32, W, H)
    else:
        geo, ph, xh, yh, x0, y0 = (assoc[k] for k in ("geo", "photo", "xh", "yh", "x0", "y0"))

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
    return {"rg": rg, "Jg_i": Jg_i, "Jg_j": Jg_j, "rp": rp, "Jp_i": Jp_i, "Jp_j": Jp_j,
            "geo": geo, "photo": ph, "xh": xh, "yh": yh, "x0": x0, "y0": y0,
            "u": u, "v": v}
