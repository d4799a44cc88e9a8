"""Python binding of libbf.so (include/bf.h): argument marshalling only.

Every computation runs in the HIP kernels behind the C ABI; this module turns
torch tensors into device pointers and C structs, and C statuses into
exceptions.  It raises if the library has not been built -- there is no CPU
fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import sys
import weakref
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

import torch

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libbf.so")
HEADER = os.path.join(os.path.dirname(PKG_DIR), "include", "bf.h")

BF_OK, BF_ERR_INVALID_ARG, BF_ERR_OUT_OF_MEMORY, BF_ERR_DEVICE, BF_ERR_NOT_PD, BF_ERR_NONFINITE, \
    BF_ERR_UNSUPPORTED = range(7)


class BFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class bf_intrinsics(ctypes.Structure):
    _fields_ = [("fx", c_double), ("fy", c_double), ("cx", c_double), ("cy", c_double),
                ("width", c_int32), ("height", c_int32)]


class bf_frames(ctypes.Structure):
    _fields_ = [("num_frames", c_int32), ("depth", c_void_p), ("intensity", c_void_p)]


class bf_corrs(ctypes.Structure):
    _fields_ = [("count", c_int64), ("frame_i", c_void_p), ("frame_j", c_void_p), ("p_i", c_void_p),
                ("p_j", c_void_p)]


class bf_pairs(ctypes.Structure):
    _fields_ = [("count", c_int64), ("ij", c_void_p)]


class bf_params(ctypes.Structure):
    _fields_ = [("w_sparse", c_double), ("w_dense", c_double), ("w_geo", c_double), ("w_photo", c_double),
                ("dense_ramp", c_int32), ("use_sparse", c_int32), ("use_dense", c_int32), ("num_gn", c_int32),
                ("num_pcg", c_int32), ("accumulate", c_int32), ("pcg_storage", c_int32), ("timing", c_int32),
                ("solve_kernel", c_int32), ("dense_threads", c_int32),
                ("tau_dist", c_double), ("tau_normal", c_double), ("max_angle_deg", c_double),
                ("depth_min", c_double), ("depth_max", c_double), ("preconditioner", c_int32),
                ("graph", c_int32), ("bidirectional", c_int32), ("dense_tiles", c_int32),
                ("pcg_spin_limit", c_int32), ("fixed_association", c_void_p),
                ("sparse_matrix_free", c_int32), ("pcg_threads", c_int32)]


class bf_structure(ctypes.Structure):
    _fields_ = [("num_pairs", c_int64), ("num_sparse_pairs", c_int64), ("num_edges", c_int64),
                ("num_free", c_int64), ("pairs_ij", c_void_p), ("sparse_ij", c_void_p), ("sparse_ptr", c_void_p),
                ("corr_perm", c_void_p), ("edges_ij", c_void_p), ("free_frames", c_void_p)]


_SIGS = {
    "bf_params_default": (None, [POINTER(bf_params)]),
    "bf_create": (c_int, [POINTER(c_void_p), c_void_p]),
    "bf_destroy": (None, [c_void_p]),
    "bf_status_string": (c_char_p, [c_int]),
    "bf_last_error": (c_char_p, [c_void_p]),
    "bf_prepare_frames": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_params),
                                  c_void_p, c_void_p]),
    "bf_build_pairs": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), c_void_p,
                               POINTER(bf_params), c_void_p, c_int64, POINTER(c_int64)]),
    "bf_build_structure": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                   POINTER(bf_pairs), c_void_p, POINTER(bf_params), POINTER(bf_structure)]),
    "bf_eval_residuals": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                  POINTER(bf_pairs), c_void_p, POINTER(bf_params), c_int32, POINTER(c_double),
                                  POINTER(c_int64), c_void_p, c_void_p]),
    "bf_system_create": (c_int, [c_void_p, POINTER(c_void_p)]),
    "bf_system_destroy": (None, [c_void_p]),
    "bf_build_normal_equations": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                          POINTER(bf_pairs), c_void_p, POINTER(bf_params), c_int32, c_void_p,
                                          c_void_p, POINTER(c_double)]),
    "bf_system_export": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_int64)]),
    "bf_pcg_solve": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, POINTER(c_double)]),
    "bf_gauss_newton": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                POINTER(bf_pairs), c_void_p, POINTER(bf_params), c_void_p, POINTER(c_double),
                                POINTER(c_double)]),
    "bf_gauss_newton_noalloc": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                        POINTER(bf_pairs), c_void_p, POINTER(bf_params), c_void_p, POINTER(c_double),
                                        POINTER(c_double)]),
    "bf_gauss_newton_batch": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                      POINTER(bf_pairs), c_int32, POINTER(c_int32), c_void_p, POINTER(bf_params),
                                      c_void_p, POINTER(c_double), POINTER(c_double)]),
    "bf_gauss_newton_pruned": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_corrs),
                                       POINTER(bf_pairs), c_void_p, POINTER(bf_params), c_double, c_int32, c_void_p,
                                       POINTER(c_double), c_void_p, c_void_p, POINTER(c_int32), POINTER(c_double)]),
    "bf_filter_correspondences": (c_int, [c_void_p, POINTER(bf_corrs), c_int32, c_double, c_double, c_int32,
                                          c_int32, c_double, c_void_p, POINTER(c_int64)]),
    "bf_verify_pairs": (c_int, [c_void_p, POINTER(bf_frames), POINTER(bf_intrinsics), POINTER(bf_pairs), c_void_p,
                                POINTER(bf_params), c_double, c_double, c_double, c_void_p, c_void_p]),
    "bf_system_matvec": (c_int, [c_void_p, c_void_p, POINTER(bf_corrs), c_void_p, c_void_p, c_int32,
                                 POINTER(c_double)]),
    "bf_last_timings": (c_int, [c_void_p, POINTER(c_double)]),
    "bf_dense_shape": (c_int, [c_void_p, POINTER(c_int32)]),
    "bf_workspace_bytes": (c_int, [c_void_p, POINTER(c_int64)]),
    "bf_pcg_threads": (c_int, [c_void_p, POINTER(c_int32)]),
    "bf_graph_captures": (ctypes.c_int64, [c_void_p]),
}

_lib = None


def load():
    """Load libbf.so (raises if it is missing: build it with paper_1604_01093_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python -m paper_1604_01093_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def header_functions(path=HEADER):
    """Names of the functions declared in include/bf.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z_0-9]+)\s*\(", text)))


def bf_params_default(**overrides):
    p = bf_params()
    load().bf_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape=None, name="tensor"):
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {shape}, got {tuple(t.shape)}")


# Contexts still open.  They are closed by an exit hook registered here, after
# torch has registered its own (exit hooks run in reverse order), so bf_destroy's
# frees run while the HIP runtime is still up; a context reached by the garbage
# collector during interpreter shutdown makes no HIP call at all.
_live = weakref.WeakSet()


def _close_live_contexts():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


atexit.register(_close_live_contexts)


class Context:
    """A bf_context bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, stream=None):
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        self._check(self.lib.bf_create(ctypes.byref(h), c_void_p(stream.cuda_stream)), ctx=None)
        self.h = h
        self.systems = weakref.WeakSet()
        _live.add(self)

    def _check(self, st, ctx="self"):
        if st != BF_OK:
            msg = self.lib.bf_last_error(self.h if ctx == "self" else None)
            raise BFError(st, (msg or b"").decode() or self.lib.bf_status_string(st).decode())

    def close(self):
        for y in list(getattr(self, "systems", ())):
            y.close()
        if getattr(self, "h", None):
            self.lib.bf_destroy(self.h)
            self.h = None
        _live.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: at interpreter exit the module's globals may be gone
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def last_timings(self):
        out = (c_double * 8)()
        self._check(self.lib.bf_last_timings(self.h, out))
        keys = ["setup_us", "dense_us", "edges_us", "assemble_us", "pcg_us", "final_us", "total_us",
                "dense_launches"]
        return dict(zip(keys, list(out)))

    def dense_shape(self):
        """(threads, tiles) of the last dense launch with Jacobians and of the last
        energy-only one."""
        out = (c_int32 * 4)()
        self._check(self.lib.bf_dense_shape(self.h, out))
        return {"jacobians": (out[0], out[1]), "energy": (out[2], out[3])}

    def pcg_threads(self):
        """Workgroup size of the last per-problem PCG launch (0 before any)."""
        out = c_int32(0)
        self._check(self.lib.bf_pcg_threads(self.h, ctypes.byref(out)))
        return int(out.value)

    def workspace_bytes(self):
        """Device bytes held by this context's workspace buffers."""
        out = c_int64(0)
        self._check(self.lib.bf_workspace_bytes(self.h, ctypes.byref(out)))
        return int(out.value)

    def graph_captures(self):
        """How often this context has captured the Gauss-Newton loop into a graph."""
        return int(self.lib.bf_graph_captures(self.h))


class System:
    """A bf_system: normal equations built by bf_build_normal_equations, owned here
    and freed by close() (or when its context is closed)."""

    def __init__(self, ctx):
        self.ctx = ctx
        h = c_void_p()
        ctx._check(ctx.lib.bf_system_create(ctx.h, ctypes.byref(h)))
        self.h = h
        ctx.systems.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.bf_system_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: at interpreter exit the module's globals may be gone
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class DeviceProblem:
    """Device tensors of one problem, marshalled into the C structs."""

    def __init__(self, depth, intensity, intr, corr_i=None, corr_j=None, p_i=None, p_j=None, pairs=None):
        F, H, W = depth.shape
        _need(depth, torch.float32, name="depth")
        _need(intensity, torch.float32, (F, H, W), "intensity")
        self.depth, self.intensity = depth, intensity
        fx, fy, cx, cy, w, h = intr
        if (w, h) != (W, H):
            raise ValueError("intrinsics size does not match the frames")
        self.intr = bf_intrinsics(fx, fy, cx, cy, W, H)
        self.frames = bf_frames(F, _ptr(depth), _ptr(intensity))
        self.num_frames = F
        if corr_i is not None and len(corr_i):
            M = corr_i.shape[0]
            _need(corr_i, torch.int32, (M,), "corr_i")
            _need(corr_j, torch.int32, (M,), "corr_j")
            _need(p_i, torch.float32, (M, 3), "p_i")
            _need(p_j, torch.float32, (M, 3), "p_j")
            self.keep = (corr_i, corr_j, p_i, p_j)
            self.corrs = bf_corrs(M, _ptr(corr_i), _ptr(corr_j), _ptr(p_i), _ptr(p_j))
        else:
            self.corrs = bf_corrs(0, None, None, None, None)
        self.num_corrs = self.corrs.count
        self.set_pairs(pairs)

    def set_pairs(self, pairs):
        self.pairs_t = pairs
        if pairs is None:
            self.pairs = None
        else:
            _need(pairs, torch.int32, name="pairs")
            self.pairs = bf_pairs(pairs.shape[0], _ptr(pairs) if pairs.numel() else None)

    @classmethod
    def from_numpy(cls, depth, intensity, intr, corr_i=None, corr_j=None, p_i=None, p_j=None, device="cuda"):
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        if corr_i is None:
            return cls(t(depth, torch.float32), t(intensity, torch.float32), intr)
        return cls(t(depth, torch.float32), t(intensity, torch.float32), intr, t(corr_i, torch.int32),
                   t(corr_j, torch.int32), t(p_i, torch.float32).reshape(-1, 3).contiguous(),
                   t(p_j, torch.float32).reshape(-1, 3).contiguous())

    def _pairs_ref(self):
        return ctypes.byref(self.pairs) if self.pairs is not None else None


def _poses_check(poses, F):
    _need(poses, torch.float64, (F, 4, 4), "poses")


def bf_prepare_frames(ctx, prob, params):
    F, H, W = prob.depth.shape
    nd = torch.empty((F, H, W, 4), dtype=torch.float32, device=prob.depth.device)
    g = torch.empty((F, H, W), dtype=torch.float32, device=prob.depth.device)
    ctx._check(ctx.lib.bf_prepare_frames(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                         ctypes.byref(params), _ptr(nd), _ptr(g)))
    return nd, g


def bf_build_pairs(ctx, prob, poses, params):
    _poses_check(poses, prob.num_frames)
    F = prob.num_frames
    cap = max(F * (F - 1) // 2, 1)
    out = torch.empty((cap, 2), dtype=torch.int32, device=poses.device)
    n = c_int64()
    ctx._check(ctx.lib.bf_build_pairs(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr), _ptr(poses),
                                      ctypes.byref(params), _ptr(out), cap, ctypes.byref(n)))
    return out[:n.value].clone()


def bf_build_structure(ctx, prob, poses, params):
    _poses_check(poses, prob.num_frames)
    s = bf_structure()
    args = (ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr), ctypes.byref(prob.corrs),
            prob._pairs_ref(), _ptr(poses), ctypes.byref(params))
    ctx._check(ctx.lib.bf_build_structure(*args, ctypes.byref(s)))
    dev = poses.device
    out = {
        "pairs": torch.empty((s.num_pairs, 2), dtype=torch.int32, device=dev),
        "sparse_ij": torch.empty((s.num_sparse_pairs, 2), dtype=torch.int32, device=dev),
        "sparse_ptr": torch.empty((s.num_sparse_pairs + 1,), dtype=torch.int64, device=dev),
        "corr_perm": torch.empty((prob.num_corrs if params.use_sparse else 0,), dtype=torch.int64, device=dev),
        "edges": torch.empty((s.num_edges, 2), dtype=torch.int32, device=dev),
        "free": torch.empty((s.num_free,), dtype=torch.int32, device=dev),
    }
    s2 = bf_structure(0, 0, 0, 0, _ptr(out["pairs"]), _ptr(out["sparse_ij"]), _ptr(out["sparse_ptr"]),
                      _ptr(out["corr_perm"]), _ptr(out["edges"]), _ptr(out["free"]))
    ctx._check(ctx.lib.bf_build_structure(*args, ctypes.byref(s2)))
    return out


def bf_eval_residuals(ctx, prob, poses, params, gn_iter=0, records=False, masks=False):
    """Energies and counts at fixed poses; optionally the per-job records [jobs, 32]
    and (masks=True) the per-pixel association [jobs, H*W, 2] int32: word 0 = target
    pixel << 2 | photometric << 1 | geometric (0 without a geometric residual), word 1
    = first pixel of the bilinear footprint."""
    _poses_check(poses, prob.num_frames)
    e = (c_double * 4)()
    n = (c_int64 * 3)()
    rec = msk = None
    if records or masks:
        st = bf_build_structure(ctx, prob, poses, params)
        jobs = st["pairs"].shape[0] * (2 if params.bidirectional else 1)
        if records:
            rec = torch.empty((jobs, 32), dtype=torch.float64, device=poses.device)
        if masks:
            Hh, Ww = prob.depth.shape[1], prob.depth.shape[2]
            msk = torch.empty((jobs, Hh * Ww, 2), dtype=torch.int32, device=poses.device)
    ctx._check(ctx.lib.bf_eval_residuals(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                         ctypes.byref(prob.corrs), prob._pairs_ref(), _ptr(poses),
                                         ctypes.byref(params), gn_iter, e, n,
                                         _ptr(rec) if rec is not None and rec.numel() else None,
                                         _ptr(msk) if msk is not None and msk.numel() else None))
    out = {"total": e[0], "sparse": e[1], "geo": e[2], "photo": e[3],
           "n_sparse": n[0], "n_geo": n[1], "n_photo": n[2]}
    if records:
        out["records"] = rec
    if masks:
        out["masks"] = msk
    return out


def bf_build_normal_equations(ctx, prob, poses, params, gn_iter=0, dense=True, edge_blocks=False, system=None):
    """Build the normal equations at `poses` into `system` (a new System when None);
    returns the system, the energies and, with dense=True, H [6F,6F] and g [6F]
    exported from it, with edge_blocks=True the per-edge blocks [E,128]."""
    _poses_check(poses, prob.num_frames)
    F = prob.num_frames
    dev = poses.device
    y = System(ctx) if system is None else system
    eb = None
    if edge_blocks:
        st = bf_build_structure(ctx, prob, poses, params)
        eb = torch.empty((st["edges"].shape[0], 128), dtype=torch.float64, device=dev)
    e = (c_double * 4)()
    ctx._check(ctx.lib.bf_build_normal_equations(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                                 ctypes.byref(prob.corrs), prob._pairs_ref(), _ptr(poses),
                                                 ctypes.byref(params), gn_iter, y.h,
                                                 _ptr(eb) if eb is not None and eb.numel() else None, e))
    out = {"system": y, "edge_blocks": eb, "energy": list(e), "H": None, "g": None}
    if dense:
        out["H"], out["g"], out["num_free"] = bf_system_export(ctx, y, F)
    return out


def bf_system_export(ctx, system, num_frames, device="cuda"):
    """Dense H [6F,6F], g [6F] and the number of free frames of a system."""
    H = torch.empty((6 * num_frames, 6 * num_frames), dtype=torch.float64, device=device)
    g = torch.empty((6 * num_frames,), dtype=torch.float64, device=device)
    nf = c_int64()
    ctx._check(ctx.lib.bf_system_export(ctx.h, system.h, _ptr(H), _ptr(g), ctypes.byref(nf)))
    return H, g, nf.value


def bf_pcg_solve(ctx, system, num_frames, iters, device="cuda"):
    delta = torch.empty((6 * num_frames,), dtype=torch.float64, device=device)
    st = (c_double * 3)()
    ctx._check(ctx.lib.bf_pcg_solve(ctx.h, system.h, iters, _ptr(delta), st))
    return delta, {"rz0": st[0], "rz_final": st[1], "iters": int(st[2])}


def bf_gauss_newton(ctx, prob, init_poses, params, out_poses=None, trace=False):
    _poses_check(init_poses, prob.num_frames)
    if out_poses is None:
        out_poses = torch.empty_like(init_poses)
    e = (c_double * 4)()
    tr = (c_double * (4 * max(params.num_gn, 1)))() if trace else None
    ctx._check(ctx.lib.bf_gauss_newton(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                       ctypes.byref(prob.corrs), prob._pairs_ref(), _ptr(init_poses),
                                       ctypes.byref(params), _ptr(out_poses), e, tr))
    res = {"poses": out_poses, "energy": {"total": e[0], "sparse": e[1], "geo": e[2], "photo": e[3]}}
    if trace:
        res["trace"] = [list(tr[4 * k:4 * k + 4]) for k in range(params.num_gn)]
    return res


def bf_gauss_newton_noalloc(ctx, prob, init_poses, params, out_poses=None, trace=False):
    """bf_gauss_newton with its workspace in the library's static scratch array
    (no allocation inside the call).  out_poses must be given by callers that
    cannot allocate; it is allocated here only for convenience when omitted."""
    _poses_check(init_poses, prob.num_frames)
    if out_poses is None:
        out_poses = torch.empty_like(init_poses)
    e = (c_double * 4)()
    tr = (c_double * (4 * max(params.num_gn, 1)))() if trace else None
    ctx._check(ctx.lib.bf_gauss_newton_noalloc(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                               ctypes.byref(prob.corrs), prob._pairs_ref(), _ptr(init_poses),
                                               ctypes.byref(params), _ptr(out_poses), e, tr))
    res = {"poses": out_poses, "energy": {"total": e[0], "sparse": e[1], "geo": e[2], "photo": e[3]}}
    if trace:
        res["trace"] = [list(tr[4 * k:4 * k + 4]) for k in range(params.num_gn)]
    return res


def bf_gauss_newton_batch(ctx, prob, frame_offsets, init_poses, params, out_poses=None, trace=False):
    """Independent problems over consecutive frame ranges of one DeviceProblem.
    frame_offsets: sequence of num_problems + 1 ints (host)."""
    _poses_check(init_poses, prob.num_frames)
    offs = [int(v) for v in frame_offsets]
    B = len(offs) - 1
    if out_poses is None:
        out_poses = torch.empty_like(init_poses)
    off_arr = (c_int32 * len(offs))(*offs)
    e = (c_double * (4 * max(B, 1)))()
    tr = (c_double * (4 * max(B, 1) * max(params.num_gn, 1)))() if trace else None
    ctx._check(ctx.lib.bf_gauss_newton_batch(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                             ctypes.byref(prob.corrs), prob._pairs_ref(), B, off_arr,
                                             _ptr(init_poses), ctypes.byref(params), _ptr(out_poses), e, tr))
    res = {"poses": out_poses,
           "energy": [{"total": e[4 * b], "sparse": e[4 * b + 1], "geo": e[4 * b + 2], "photo": e[4 * b + 3]}
                      for b in range(B)]}
    if trace:
        G = params.num_gn
        res["trace"] = [[list(tr[(b * G + k) * 4:(b * G + k) * 4 + 4]) for k in range(G)] for b in range(B)]
    return res


def concat_problems(problems):
    """Host-side concatenation of independent problems for bf_gauss_newton_batch:
    frames stacked in order, correspondence frame indices shifted by each problem's
    first frame.  Each problem provides depth, intensity, intrinsics, corr_i, corr_j,
    corr_p, corr_q and init_poses (numpy arrays); all must share the intrinsics."""
    import numpy as np
    intr = tuple(problems[0].intrinsics)
    offs = [0]
    for pr in problems:
        if tuple(pr.intrinsics) != intr:
            raise ValueError("all problems of a batch must share the intrinsics")
        offs.append(offs[-1] + pr.depth.shape[0])
    cat = lambda xs, dt: np.ascontiguousarray(np.concatenate(xs), dtype=dt)
    return {
        "depth": cat([pr.depth for pr in problems], np.float32),
        "intensity": cat([pr.intensity for pr in problems], np.float32),
        "intrinsics": intr,
        "corr_i": cat([np.asarray(pr.corr_i, np.int64) + o for pr, o in zip(problems, offs)], np.int32),
        "corr_j": cat([np.asarray(pr.corr_j, np.int64) + o for pr, o in zip(problems, offs)], np.int32),
        "corr_p": cat([np.asarray(pr.corr_p).reshape(-1, 3) for pr in problems], np.float32),
        "corr_q": cat([np.asarray(pr.corr_q).reshape(-1, 3) for pr in problems], np.float32),
        "init_poses": cat([pr.init_poses for pr in problems], np.float64),
        "offsets": offs,
    }


def device_batch(problems, device="cuda"):
    """DeviceProblem, frame offsets and initial poses (device) of a batch of problems."""
    b = concat_problems(problems)
    dp = DeviceProblem.from_numpy(b["depth"], b["intensity"], b["intrinsics"], b["corr_i"], b["corr_j"],
                                  b["corr_p"], b["corr_q"], device=device)
    init = torch.as_tensor(b["init_poses"]).to(device)
    return dp, b["offsets"], init


def bf_system_matvec(ctx, system, prob, x, mode):
    """y = H x of a system (mode 0 blocks, mode 1 matrix-free sparse term); returns
    (y, microseconds)."""
    _need(x, torch.float64, (6 * prob.num_frames,), "x")
    y = torch.empty_like(x)
    us = c_double()
    ctx._check(ctx.lib.bf_system_matvec(ctx.h, system.h, ctypes.byref(prob.corrs), _ptr(x), _ptr(y), mode,
                                        ctypes.byref(us)))
    return y, us.value


def bf_gauss_newton_pruned(ctx, prob, init_poses, params, r_prune=0.05, max_rounds=100, out_poses=None):
    """Solve with residual pruning; returns poses, energy, masks, rounds, r_max."""
    _poses_check(init_poses, prob.num_frames)
    if out_poses is None:
        out_poses = torch.empty_like(init_poses)
    dev = init_poses.device
    act = torch.empty((max(prob.num_corrs, 1),), dtype=torch.uint8, device=dev)
    val = torch.empty((prob.num_frames,), dtype=torch.uint8, device=dev)
    e = (c_double * 4)()
    rounds = c_int32()
    rmax = c_double()
    ctx._check(ctx.lib.bf_gauss_newton_pruned(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr),
                                              ctypes.byref(prob.corrs), prob._pairs_ref(), _ptr(init_poses),
                                              ctypes.byref(params), r_prune, max_rounds, _ptr(out_poses), e,
                                              _ptr(act), _ptr(val), ctypes.byref(rounds), ctypes.byref(rmax)))
    return {"poses": out_poses, "energy": {"total": e[0], "sparse": e[1], "geo": e[2], "photo": e[3]},
            "corr_active": act[:prob.num_corrs], "frame_valid": val, "rounds": rounds.value, "rmax": rmax.value}


def bf_verify_pairs(ctx, prob, pairs, poses, params, tau_c=0.1, max_err=0.075, min_frac=0.02):
    """Two-sided dense verification of the pairs [P,2] (device int32); returns
    (stats [P,4] float64, valid [P] bool)."""
    _poses_check(poses, prob.num_frames)
    _need(pairs, torch.int32, name="pairs")
    P = pairs.shape[0]
    stats = torch.empty((max(P, 1), 4), dtype=torch.float64, device=poses.device)
    valid = torch.empty((max(P, 1),), dtype=torch.uint8, device=poses.device)
    bp = bf_pairs(P, _ptr(pairs) if P else None)
    ctx._check(ctx.lib.bf_verify_pairs(ctx.h, ctypes.byref(prob.frames), ctypes.byref(prob.intr), ctypes.byref(bp),
                                       _ptr(poses), ctypes.byref(params), tau_c, max_err, min_frac, _ptr(stats),
                                       _ptr(valid)))
    return stats[:P], valid[:P].bool()


def bf_filter_correspondences(ctx, prob, max_res=0.02, max_cond=100.0, min_count=5, min_area=0.032, cond_mode=0):
    """Key-point and surface-area filters over the problem's correspondences;
    returns the keep mask [M] (device, bool) and the number kept.  cond_mode 0:
    condition numbers as largest / second largest value, 1: largest / smallest."""
    M = prob.num_corrs
    keep = torch.empty((max(M, 1),), dtype=torch.uint8, device="cuda")
    kept = c_int64()
    ctx._check(ctx.lib.bf_filter_correspondences(ctx.h, ctypes.byref(prob.corrs), prob.num_frames, max_res, max_cond,
                                                 cond_mode, min_count, min_area, _ptr(keep), ctypes.byref(kept)))
    return keep[:M].bool(), kept.value
