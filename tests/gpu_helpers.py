"""Shared helpers of the GPU parity tests: device problems, parameter mapping,
pose error measures."""
import numpy as np
import torch

from oracle import Params
from oracle.se3 import rotation_angle
from paper_1604_01093_amd import bf


def device_problem(prob, pairs=None):
    dp = bf.DeviceProblem.from_numpy(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j,
                                     prob.corr_p, prob.corr_q)
    if pairs is not None:
        dp.set_pairs(torch.as_tensor(np.asarray(pairs, np.int32).reshape(-1, 2)).cuda().contiguous())
    return dp


def bf_params_from(prm: Params, **kw):
    p = bf.bf_params_default(
        w_sparse=prm.w_sparse, w_dense=prm.w_dense, w_geo=prm.w_geo, w_photo=prm.w_photo,
        dense_ramp=int(prm.dense_ramp), use_sparse=int(prm.use_sparse), use_dense=int(prm.use_dense),
        num_gn=prm.num_gn, num_pcg=prm.num_pcg, tau_dist=prm.tau_dist, tau_normal=prm.tau_normal,
        max_angle_deg=prm.max_angle_deg, depth_min=prm.depth_min, depth_max=prm.depth_max,
        preconditioner={"block": 0, "jacobi": 1}[prm.preconditioner], bidirectional=int(prm.bidirectional))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def poses_cuda(poses):
    return torch.as_tensor(np.ascontiguousarray(poses, np.float64)).cuda()


def pose_errors(A, B):
    """Max rotation angle (rad) and translation distance (m) between pose stacks."""
    rot = max(rotation_angle(A[f][:3, :3].T @ B[f][:3, :3]) for f in range(len(A)))
    tr = max(float(np.linalg.norm(A[f][:3, 3] - B[f][:3, 3])) for f in range(len(A)))
    return rot, tr


def block_rel_err(A, B):
    """|A - B|_F / max(|B|_F, tiny)."""
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / max(nb, 1e-300))


def upper21(M):
    return np.array([M[a, b] for a in range(6) for b in range(a, 6)])


def compare_masks(gpu_words, assoc, W, k_near=2.0):
    """Compare a job's GPU association ([H*W, 2] words from bf_eval_residuals:
    target pixel << 2 | photometric << 1 | geometric, footprint pixel) with the
    oracle's FP64 decisions (``oracle.terms.associate``): the geometric and
    photometric decisions, the target pixel where both associate and the bilinear
    footprint where both use the photometric residual.

    A difference is excused only where the oracle flags the decision as within
    k_near times the binary32 rounding bound of one of its tests (a different
    target pixel or footprint arises only at a rounding tie of u or v); returns
    (unexcused geometric, unexcused photometric, excused geometric, excused
    photometric, identical)."""
    from oracle.terms import near_decisions
    g = np.asarray(gpu_words).reshape(-1, 2).astype(np.int64) & 0xffffffff
    w0, w1 = g[:, 0], g[:, 1]
    g_geo = (w0 & 1) != 0
    g_ph = (w0 & 2) != 0
    near_geo, near_ph = near_decisions(assoc, k_near)
    geo, ph = assoc["geo"], assoc["photo"]
    mg = (g_geo != geo) | (g_geo & geo & ((w0 >> 2) != assoc["yh"] * W + assoc["xh"]))
    mp = (g_ph != ph) | (g_ph & ph & (w1 != assoc["y0"] * W + assoc["x0"]))
    return (int((mg & ~near_geo).sum()), int((mp & ~near_ph).sum()), int((mg & near_geo).sum()),
            int((mp & near_ph).sum()), not mg.any() and not mp.any())


def encode_association(assocs, W):
    """The oracle's associations of a list of jobs as the fixed association the
    kernels take (bf_params.fixed_association): [jobs, H*W, 2] int32 on the GPU."""
    out = np.zeros((len(assocs), len(assocs[0]["geo"]) if assocs else 0, 2), np.int64)
    for k, a in enumerate(assocs):
        geo, ph = a["geo"], a["photo"]
        out[k, :, 0] = np.where(geo, ((a["yh"] * W + a["xh"]) << 2) | 1 | np.where(ph, 2, 0), 0)
        out[k, :, 1] = np.where(ph, a["y0"] * W + a["x0"], 0)
    return torch.as_tensor(out.astype(np.int32)).cuda().contiguous()


def fix_association(params, t):
    """Point params.fixed_association at the device tensor t (kept alive by the caller)."""
    params.fixed_association = t.data_ptr() if t is not None else None
    return params
