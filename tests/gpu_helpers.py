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


def compare_masks(gpu_masks, assoc, k_near=2.0):
    """Compare a job's GPU association masks ([H*W] uint8: bit 0 geometric, bit 1
    photometric) with the oracle's FP64 decisions (``oracle.terms.associate``).

    A mismatch is excused only where the oracle flags the decision as within
    k_near times the binary32 rounding bound of one of its tests; returns
    (unexcused geometric, unexcused photometric, excused geometric, excused
    photometric, identical) where `identical` says both masks agree everywhere."""
    from oracle.terms import near_decisions
    g = np.asarray(gpu_masks).reshape(-1)
    g_geo = (g & 1) != 0
    g_ph = (g & 2) != 0
    near_geo, near_ph = near_decisions(assoc, k_near)
    mg = g_geo != assoc["geo"]
    mp = g_ph != assoc["photo"]
    return (int((mg & ~near_geo).sum()), int((mp & ~near_ph).sum()), int((mg & near_geo).sum()),
            int((mp & near_ph).sum()), not mg.any() and not mp.any())
