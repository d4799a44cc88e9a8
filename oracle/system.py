"""Gauss-Newton normal equations and their solution (paper Sec. 4.4).

The canonical least-squares form E = sum_k r_k^2 gives, after linearisation,
J^T J dX = -J^T F.  Here J^T J and J^T F are accumulated from the per-pair
residual Jacobians of ``terms`` (each residual touches the two frames of its
pair, so the contributions are 6x6 blocks), in FP64, into a dense 6F x 6F
matrix.  The reference frame T_0 is not a variable (Sec. 4.3) and frames with
no constraint at all are left out (Sec. 4.4.1), so their rows and columns are
deleted before solving.

Two linear solvers:
* ``solve_cholesky`` -- the exact solution by a dense Cholesky factorisation.
* ``solve_pcg``      -- preconditioned conjugate gradients (Sec. 4.4) with a
  6x6 block-Jacobi preconditioner, x0 = 0, a fixed iteration count and an early
  exit only when r^T z <= 1e-30.  (The paper names a Jacobi preconditioner;
  the per-frame block variant is the reading used here.)
"""
import numpy as np
import scipy.linalg

from .terms import dense_terms, sparse_terms


def _blocks(Ji, Jj, r, w):
    """Weighted J^T J blocks and J^T r for residual rows with Jacobians Ji, Jj [n,6].
    The diagonal blocks are symmetrised explicitly (a matrix library need not round
    the two triangles of J^T J identically)."""
    sym = lambda A: 0.5 * (A + A.T)
    return {"Hii": w * sym(Ji.T @ Ji), "Hij": w * (Ji.T @ Jj), "Hjj": w * sym(Jj.T @ Jj),
            "gi": w * (Ji.T @ r), "gj": w * (Jj.T @ r), "E": w * float(r @ r)}


def sparse_pair_blocks(Ti, Tj, p, q, w):
    r, Ji, Jj = sparse_terms(Ti, Tj, p, q)
    out = _blocks(Ji.reshape(-1, 6), Jj.reshape(-1, 6), r.reshape(-1), w)
    out["n"] = len(p)
    return out


def dense_pair_blocks(fi, fj, Ti, Tj, intr, params, wd, assoc=None):
    t = dense_terms(fi, fj, Ti, Tj, intr, params, assoc=assoc)
    wg = wd * params.w_geo
    wp = wd * params.w_photo
    bg = _blocks(t["Jg_i"], t["Jg_j"], t["rg"], wg)
    bp = _blocks(t["Jp_i"], t["Jp_j"], t["rp"], wp)
    out = {k: bg[k] + bp[k] for k in ("Hii", "Hij", "Hjj", "gi", "gj")}
    out["Egeo"] = bg["E"]
    out["Ephoto"] = bp["E"]
    out["ngeo"] = int(t["geo"].sum())
    out["nphoto"] = int(t["photo"].sum())
    out["terms"] = t
    return out


def assemble(F, edges, blocks):
    """Dense H [6F,6F] and g [6F] from per-edge block dicts (list aligned with edges)."""
    H = np.zeros((6 * F, 6 * F))
    g = np.zeros(6 * F)
    for (i, j), b in zip(edges, blocks):
        si, sj = slice(6 * i, 6 * i + 6), slice(6 * j, 6 * j + 6)
        H[si, si] += b["Hii"]
        H[sj, sj] += b["Hjj"]
        H[si, sj] += b["Hij"]
        H[sj, si] += b["Hij"].T
        g[si] += b["gi"]
        g[sj] += b["gj"]
    return H, g


def free_frames(F, edges):
    """Frames that are variables: not frame 0 and touched by at least one pair."""
    deg = np.zeros(F, np.int64)
    for i, j in edges:
        deg[i] += 1
        deg[j] += 1
    return np.array([f for f in range(1, F) if deg[f] > 0], np.int64)


def inert_frames(H, free):
    """Mask over `free`: frames whose 6x6 diagonal block of H is identically zero,
    i.e. no residual touches them at these poses (every pixel association of their
    pairs failed and they have no correspondence).  Like the unconstrained frames of
    Sec. 4.4.1 they carry no information in this iteration and are held fixed."""
    return np.array([not np.any(H[6 * f:6 * f + 6, 6 * f:6 * f + 6]) for f in free], bool)


def reduce_system(H, g, free):
    idx = (6 * free[:, None] + np.arange(6)[None, :]).ravel()
    return H[np.ix_(idx, idx)], g[idx], idx


class NotPositiveDefinite(RuntimeError):
    pass


def solve_cholesky(Hr, gr):
    """Solve Hr dx = -gr by Cholesky; raises NotPositiveDefinite."""
    try:
        L = np.linalg.cholesky(Hr)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e)) from e
    y = scipy.linalg.solve_triangular(L, -gr, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


def block_jacobi_inverse(Hr):
    n = Hr.shape[0] // 6
    Minv = np.zeros((n, 6, 6))
    for k in range(n):
        B = Hr[6 * k:6 * k + 6, 6 * k:6 * k + 6]
        try:
            L = np.linalg.cholesky(B)
        except np.linalg.LinAlgError as e:
            raise NotPositiveDefinite(f"diagonal block {k}: {e}") from e
        Li = scipy.linalg.solve_triangular(L, np.eye(6), lower=True)
        Minv[k] = Li.T @ Li
    return Minv


def jacobi_inverse(Hr):
    """The paper's Jacobi preconditioner (Sec. 4.4): the inverse of the diagonal of
    Hr, as 6x6 diagonal blocks."""
    d = np.diag(Hr).reshape(-1, 6)
    if np.any(~(d > 0)):
        raise NotPositiveDefinite("non-positive diagonal entry")
    return np.einsum("ka,ab->kab", 1.0 / d, np.eye(6))


def solve_pcg(Hr, gr, iters, eps=1e-30, preconditioner="block"):
    """PCG on Hr dx = -gr from dx = 0 with the 6x6 block-Jacobi ("block") or the
    scalar Jacobi ("jacobi") preconditioner; returns (dx, stats)."""
    Minv = block_jacobi_inverse(Hr) if preconditioner == "block" else jacobi_inverse(Hr)
    n = Hr.shape[0] // 6

    def prec(r):
        return np.einsum("kab,kb->ka", Minv, r.reshape(n, 6)).ravel()

    x = np.zeros_like(gr)
    r = -gr.copy()
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    rz0 = rz
    done = 0
    for _ in range(iters):
        if rz <= eps:
            break
        Ap = Hr @ p
        alpha = rz / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = prec(r)
        rz_new = float(r @ z)
        done += 1
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, {"rz0": rz0, "rz_final": rz, "iters": done}
