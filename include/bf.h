/*
 * bf.h -- C ABI of the MI355X global pose alignment library (libbf.so).
 *
 * The library solves the global alignment problem of Dai et al., "BundleFusion"
 * (arXiv:1604.01093), Sec. 4.3-4.4: given RGB-D frames, sparse 3D point
 * correspondences between frame pairs and initial camera poses, it minimises
 *
 *   E_align = w_sparse E_sparse + w_d (w_geo E_geo + w_photo E_photo)
 *
 * over the camera-to-world poses T_f (T_0 fixed) by Gauss-Newton with a
 * block-Jacobi preconditioned conjugate gradient solve of J^T J dX = -J^T F
 * (Sec. 4.4) and the SE(3) exponential update (Sec. 4.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers owned by the caller unless the comment says
 *   "host".  Device buffers must stay valid until the call has completed on the
 *   context's stream.  Calls are ordered on that stream.  A call that writes a
 *   host output synchronises the stream before returning; the others return after
 *   enqueueing their work (bf_prepare_frames only).
 * - Images are row-major [num_frames][height][width] float32.  Depth is in metres;
 *   0, non-finite or outside [depth_min, depth_max] means "no depth".  Intensity
 *   is used directly as luminance.  Pixel (x, y) has its centre at u = x, v = y.
 * - Poses are row-major 4x4 float64 camera-to-world matrices, [num_frames][4][4].
 *   A pose update is T_f <- T_f Exp(xi_f), xi_f = (omega_f, v_f), and increments
 *   are returned in that order, 6 per frame.
 * - Correspondence points are float32 [count][3] in the camera frame of their own
 *   frame, metres.  frame_i != frame_j; either order is accepted.
 * - Dense pairs are int32 [count][2] with ij[k][0] < ij[k][1], strictly
 *   increasing in (i, j).  The lower index is the source frame of the pair job.
 * - On any error the outputs are left unwritten and the message of the last error
 *   is available from bf_last_error().
 * - A context is not thread safe; use one context per stream.  Its workspace is
 *   allocated on first use, grown on demand, never inside a Gauss-Newton loop,
 *   and freed by bf_destroy().
 */
#ifndef BF_H
#define BF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bf_status {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = 1,    /* bad sizes, null pointers, indices out of range, unsorted pairs */
  BF_ERR_OUT_OF_MEMORY = 2,  /* device workspace could not be allocated */
  BF_ERR_DEVICE = 3,         /* a HIP runtime call failed */
  BF_ERR_NOT_PD = 4,         /* a 6x6 diagonal block of J^T J is not positive definite */
  BF_ERR_NONFINITE = 5,      /* non-finite correspondence point or pose */
  BF_ERR_UNSUPPORTED = 6     /* a parameter combination the library does not implement */
} bf_status;

typedef struct bf_context bf_context;

/* Camera intrinsics of the (downsampled) frames, Sec. 4.1.1 / 4.3. */
typedef struct bf_intrinsics {
  double fx, fy, cx, cy;
  int32_t width, height;
} bf_intrinsics;

/* RGB-D frames S = {f_i} (Sec. 4): depth and intensity, [F][H][W] float32 device. */
typedef struct bf_frames {
  int32_t num_frames;
  const float* depth;
  const float* intensity;
} bf_frames;

/* Sparse correspondences C(i,j) of E_sparse (Sec. 4.3). */
typedef struct bf_corrs {
  int64_t count;
  const int32_t* frame_i;   /* [count] */
  const int32_t* frame_j;   /* [count] */
  const float* p_i;         /* [count][3], point in camera frame_i */
  const float* p_j;         /* [count][3], point in camera frame_j */
} bf_corrs;

/* Dense frame-pair set E (Sec. 4.3). */
typedef struct bf_pairs {
  int64_t count;
  const int32_t* ij;        /* [count][2] */
} bf_pairs;

/* Solver parameters.  Values the paper gives: 60 degree pair angle (Sec. 4.3).
 * The paper gives no weights, pruning thresholds or iteration counts for the
 * dense energy; bf_params_default() fills the readings documented there. */
typedef struct bf_params {
  double w_sparse, w_dense, w_geo, w_photo;
  int32_t dense_ramp;       /* 1: w_d(k) = w_dense (k+1)/num_gn (Sec. 4.3 "linearly increased") */
  int32_t use_sparse;       /* 0 drops E_sparse */
  int32_t use_dense;        /* 0 drops E_geo and E_photo */
  int32_t num_gn;           /* Gauss-Newton iterations */
  int32_t num_pcg;          /* PCG iterations per Gauss-Newton iteration (early exit if r^T z <= 1e-30) */
  int32_t accumulate;       /* per-pixel residual/Jacobian values and J^T J lane sums:
                               0 = FP32, 1 = FP32 with two-sum compensated sums,
                               2 = FP64 values and sums (association decisions are FP32 in
                               every mode, so the masks do not depend on this choice) */
  int32_t pcg_storage;      /* PCG matrix and vectors: 0 = FP32 (dots and alpha/beta in FP64), 1 = FP64 */
  int32_t timing;           /* HIP events for bf_last_timings(): 0 none, 1 every phase, 2 only the
                               dense pair-job launches and the whole call (every event recorded
                               on the stream leaves the GPU idle for a few microseconds: level 1
                               costs about 6 % of a 200-keyframe solve) */
  int32_t solve_kernel;     /* PCG kernel: 0 = automatic, 1 = single workgroup (vectors in LDS),
                               2 = cooperative grid with owner-computed vectors (any size),
                               3 = replicated vectors (vectors in LDS of every workgroup; rows
                                   assembled and inverted by a separate launch; the workgroups
                                   must all be resident, every wait is bounded),
                               4 = one workgroup per problem (the kernel of bf_gauss_newton_batch;
                                   chosen automatically for problems of at most 64 free frames),
                               5 = distributed vectors (each workgroup owns an even share of the
                                   block products, its rows' owners keep their x, r and A p; every
                                   workgroup rebuilds the search direction in its LDS after each
                                   reduction; for problems whose vectors do not fit kernel 3 but
                                   whose search direction fits one workgroup's LDS: up to 4437 free
                                   frames in FP32, 2218 in FP64).  Automatic: 4 for small problems,
                                   else 3 if it fits, else 5 if it fits, else 2. */
  int32_t dense_threads;    /* threads per dense pair job (per tile): 64, 128, 256 or 512; 0
                               (default) = threads and tiles chosen together, the fastest of
                               several shapes timed once per image size, mode and job-count range
                               in this context (the first call of a shape synchronises once).  The
                               lane sums of a job are combined in an order fixed by these values,
                               so results are bitwise reproducible for fixed values. */
  double tau_dist;          /* dense association: |c - q| < tau_dist (metres) */
  double tau_normal;        /* dense association: normal dot product > tau_normal */
  double max_angle_deg;     /* dense pair test: viewing directions within this angle */
  double depth_min, depth_max;
  int32_t preconditioner;   /* PCG preconditioner: 0 = 6x6 block-Jacobi (one Cholesky-inverted
                               block per frame), 1 = Jacobi (the diagonal of J^T J, as in
                               Sec. 4.4) */
  int32_t graph;            /* 1: bf_gauss_newton and bf_gauss_newton_batch run the Gauss-Newton
                               loop (every iteration and the final energy, after the per-call
                               setup) as one HIP graph launch.  The loop is captured on the first
                               call and replayed while the parameters, intrinsics, structure sizes,
                               pose buffers and workspace are unchanged (else captured again), so
                               repeated solves of same-sized inputs skip the per-kernel launches.
                               Results are bitwise those of graph = 0.  Needs the per-problem PCG
                               kernel (a batch, or at most 64 free frames; else
                               BF_ERR_UNSUPPORTED); bf_gauss_newton_pruned ignores it.  With
                               timing = 1 only the setup and total times are reported. */
  int32_t bidirectional;    /* 1: the dense terms are summed over the pixels of both frames of every
                               pair (jobs i -> j and j -> i), not only over the lower frame's
                               (Sec. 4.3 sums over the pixels of frame i of each pair in E; this is
                               the symmetric variant).  Records then hold 2P jobs: pair p at p
                               and its reverse at P + p. */
  int32_t dense_tiles;      /* tiles per dense pair job (its pixels split into this many parts, each a
                               workgroup, their sums added in tile order); with dense_threads set,
                               0 means 1; with dense_threads = 0 both are chosen by timing */
  int32_t pcg_spin_limit;   /* polls after which a PCG kernel's wait for the other workgroups gives
                               up (then BF_ERR_DEVICE, nothing written); 0 = the default of 2^26
                               (about two seconds).  A small value forces the time-out path. */
  const uint32_t* fixed_association;
                            /* device, NULL (default) = decide the dense association at the
                               current poses as Sec. 4.3 describes.  Otherwise the association
                               to use, [jobs][H][W][2] uint32 in the layout bf_eval_residuals
                               writes to out_assoc (same job order): it is held fixed instead of
                               decided, e.g. to compare the residual arithmetic of two
                               implementations under one association, or to iterate on a smooth
                               energy.  Only pixels whose source and target normals (and
                               gradients, for the photometric term) are valid are used. */
  int32_t sparse_matrix_free;
                            /* 1: the PCG applies the sparse term matrix-free, as Sec. 4.4 does:
                               in every iteration, per sparse frame pair, J p for each of its
                               correspondences and at once J^T of it summed over the pair (FP64,
                               fixed order), instead of the pair's assembled 6x6 blocks; the
                               dense term keeps its blocks and the block-Jacobi preconditioner
                               keeps the full diagonal blocks.  Runs in the distributed-vector
                               PCG kernel (solve_kernel 0 or 5; BF_ERR_UNSUPPORTED where the
                               search direction does not fit one workgroup's LDS) and only in
                               bf_gauss_newton and bf_gauss_newton_noalloc. */
  int32_t pcg_threads;      /* threads per problem of the per-problem PCG kernel (batches, and
                               problems of at most 64 free frames): 64, 128, 256 or 1024; 0
                               (default) = 256; -1 = the fastest of the four, timed once per
                               (storage, problem count range, largest problem) in the context (the
                               timing runs solve the current system without writing any result; in
                               graph mode a choice not yet timed by an eager call is 256).  Each
                               size sums in its own fixed order: results agree within rounding. */
} bf_params;

void bf_params_default(bf_params* out);

bf_status bf_create(bf_context** out, void* hip_stream);   /* stream owned by the caller; NULL = default */
void bf_destroy(bf_context* ctx);
const char* bf_status_string(bf_status s);
const char* bf_last_error(const bf_context* ctx);

/*
 * Per-frame preprocessing (Sec. 4.1.1: camera-space positions and normals of the
 * low-resolution depth are cached per frame; Sec. 4.3: the photometric term uses
 * the gradient of the luminance).
 *   out_normal_depth: [F][H][W][4] float32 (nx, ny, nz, depth); the normal is NaN
 *                     where it is invalid (image border, centre or a 4-neighbour
 *                     without depth, vanishing cross product).  May be NULL.
 *   out_grad:         [F][H][W] float32 central-difference gradient magnitude of the
 *                     intensity, NaN on the border or next to non-finite intensity.
 *                     May be NULL.
 * The normal at (x,y) is the normalised cross product (P(x+1,y)-P(x-1,y)) x
 * (P(x,y+1)-P(x,y-1)) oriented towards the camera.  Does not synchronise.
 */
bf_status bf_prepare_frames(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                            const bf_params* params, float* out_normal_depth, float* out_grad);

/*
 * Dense pair set E (Sec. 4.3): pairs i < j whose viewing directions are within
 * max_angle_deg and where at least one pixel of a fixed 8x6 grid of frame i with
 * valid depth projects in front of camera j and inside its image, evaluated at
 * `poses`.  out_ij: [capacity][2] int32, sorted; *out_count (host) receives the
 * number of pairs found (also when it exceeds capacity: then BF_ERR_INVALID_ARG).
 */
bf_status bf_build_pairs(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                         const double* poses, const bf_params* params,
                         int32_t* out_ij, int64_t capacity, int64_t* out_count);

/* Problem structure exported for inspection (all device, caller-allocated, each may be NULL). */
typedef struct bf_structure {
  int64_t num_pairs;        /* host out: dense pair jobs */
  int64_t num_sparse_pairs; /* host out: distinct unordered frame pairs with correspondences */
  int64_t num_edges;        /* host out: union of the two pair sets */
  int64_t num_free;         /* host out: frames that are variables (not frame 0, at least one edge) */
  int32_t* pairs_ij;        /* [num_pairs][2] */
  int32_t* sparse_ij;       /* [num_sparse_pairs][2] */
  int64_t* sparse_ptr;      /* [num_sparse_pairs+1] CSR into the sorted correspondences */
  int64_t* corr_perm;       /* [corr count] stable sort of correspondences by (min, max) frame */
  int32_t* edges_ij;        /* [num_edges][2] */
  int32_t* free_frames;     /* [num_free] */
} bf_structure;

/*
 * Build the per-solve structure (prepared frames, dense pairs -- computed from
 * `poses` when pairs == NULL --, correspondence grouping, edge union, free frames)
 * and export it into `out`.  The capacities of the out arrays are the caller's
 * responsibility: call once with all pointers NULL to obtain the counts.
 */
bf_status bf_build_structure(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                             const bf_corrs* corrs, const bf_pairs* pairs, const double* poses,
                             const bf_params* params, bf_structure* out);

/*
 * Residual evaluation at fixed poses (Sec. 4.3-4.4): the energy terms with the
 * dense weight of Gauss-Newton iteration `gn_iter`.
 *   out_energy (host) [4]: total, sparse, geometric, photometric (weighted, no 1/2).
 *   out_counts (host) [3]: sparse correspondences, geometric and photometric
 *                          residuals that were associated.
 *   out_pair_records (device, may be NULL) [num_pairs][32] float64 ([2 num_pairs][32]
 *     with params->bidirectional, the reverse jobs after the forward ones): per dense pair job
 *     the upper triangle of sum w J_j^T J_j (21, row-major), sum w J_j^T r (6), the
 *     weighted geometric and photometric energies and the two residual counts, where
 *     J_j is the Jacobian with respect to the target frame's perturbation.
 *   out_assoc (device, may be NULL) [jobs][H][W][2] uint32: the association of every source
 *     pixel of every dense pair job (same job order as the records), for inspection and
 *     tests; the decisions are those every other entry point takes.  Word 0 is 0 when the
 *     pixel has no geometric residual, else (target pixel y*W + x) << 2 | 1, plus 2 when it
 *     also has a photometric one (the nearest pixel floor(u+1/2), floor(v+1/2) inside the
 *     image with a valid normal, |c - q| < tau_dist, m.N_j > tau_normal; photometric: G_i
 *     valid and the bilinear footprint inside the image and valid).  Word 1 is the first
 *     pixel y0*W + x0 of the bilinear footprint (floor(u), floor(v)), 0 when unused.
 */
bf_status bf_eval_residuals(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                            const bf_corrs* corrs, const bf_pairs* pairs, const double* poses,
                            const bf_params* params, int32_t gn_iter, double* out_energy,
                            int64_t* out_counts, double* out_pair_records, uint32_t* out_assoc);

/*
 * A system of normal equations J^T J dx = -J^T F (Sec. 4.4) built at fixed poses:
 * the per-edge 6x6 blocks, the right-hand side and the structure the PCG reads,
 * held in device memory owned by the system.  Created empty for a context and
 * used only with that context; bf_build_normal_equations fills it (again, when
 * reused), bf_system_export, bf_pcg_solve and bf_system_matvec read it.  Several
 * systems of one context can coexist; nothing refers to "the last system".
 * bf_system_destroy synchronises the context's stream (which must still exist)
 * and frees the system; it may be called after bf_destroy of its context.
 */
typedef struct bf_system bf_system;
bf_status bf_system_create(bf_context* ctx, bf_system** out);
void bf_system_destroy(bf_system* sys);

/*
 * Normal equations at fixed poses (Sec. 4.4): J^T J and J^T F of E_align with the
 * dense weight of iteration `gn_iter`, built into `sys` (created for this context).
 *   out_edge_blocks (device, may be NULL): [num_edges][128] float64 per edge (i,j):
 *     H_ii (36), H_jj (36), H_ij (36), g_i (6), g_j (6), sparse, geometric and
 *     photometric energy, and the three residual counts.
 *   out_energy (host, may be NULL) [4] as for bf_eval_residuals.
 * On error `sys` is left as it was.
 */
bf_status bf_build_normal_equations(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                                    const bf_corrs* corrs, const bf_pairs* pairs, const double* poses,
                                    const bf_params* params, int32_t gn_iter, bf_system* sys,
                                    double* out_edge_blocks, double* out_energy);

/*
 * The system as dense arrays (small problems, tests):
 *   out_H (device, may be NULL): [6F][6F] float64, all frames (frame 0 included).
 *   out_g (device, may be NULL): [6F] float64.
 *   out_num_free (host, may be NULL): frames that are variables.
 * Synchronises the stream.
 */
bf_status bf_system_export(bf_context* ctx, const bf_system* sys, double* out_H, double* out_g,
                           int64_t* out_num_free);

/*
 * Block-Jacobi PCG (Sec. 4.4) on `sys`: solves H' dx = -g' over the free frames
 * from dx = 0 with `num_iters` iterations, in the storage precision, preconditioner
 * and PCG kernel of the params the system was built with.  out_delta (device) [6F]
 * float64 receives dx in frame order with zeros for frame 0 and frames that are not
 * variables.  out_stats (host, may be NULL) [3]: r^T z at the start, at the end,
 * iterations run.  BF_ERR_NOT_PD if a diagonal block cannot be factorised;
 * BF_ERR_DEVICE if a wait of the PCG kernel for its other workgroups gave up
 * (params->pcg_spin_limit).
 */
bf_status bf_pcg_solve(bf_context* ctx, const bf_system* sys, int32_t num_iters, double* out_delta,
                       double* out_stats);

/*
 * The full solve (Sec. 4.3-4.4): params->num_gn Gauss-Newton iterations from
 * init_poses, each evaluating residuals and Jacobians, reducing them into 6x6
 * blocks, running params->num_pcg block-Jacobi PCG iterations and applying
 * T_f <- T_f Exp(dx_f).  The dense pair set is computed from init_poses when
 * pairs == NULL.  Frame 0 and frames without any constraint keep their pose
 * bit for bit.
 *   out_poses (device) [F][4][4] float64; may alias init_poses.
 *   out_energy (host) [4]: energy at the returned poses with the last iteration's w_d.
 *   out_trace (host, may be NULL) [num_gn][4]: energy at the start of each iteration.
 */
bf_status bf_gauss_newton(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                          const bf_corrs* corrs, const bf_pairs* pairs, const double* init_poses,
                          const bf_params* params, double* out_poses, double* out_energy,
                          double* out_trace);

/*
 * bf_gauss_newton without any allocation, for callers that cannot allocate device
 * or pinned host memory during the call: code inside a serving loop that must not
 * reach the allocator, harnesses that forbid hipMalloc, callers preparing to run
 * under stream capture.  Arguments, outputs and results are those of
 * bf_gauss_newton (the same kernels in the same order: the poses and energies are
 * bitwise those of bf_gauss_newton with the same params).
 *
 * The workspace is a fixed static device array of 64 MiB per GPU (held from the
 * first use of the library on that GPU until the process ends) instead of the
 * context's growing buffers; a problem whose workspace does not fit returns
 * BF_ERR_OUT_OF_MEMORY with nothing written (about 150 keyframes at 80x60 with
 * 300k correspondences fit, or any chunk of up to 11 frames at 160x120).  The call
 * makes no hipMalloc, hipFree, hipHostMalloc or hipEventCreate; host readbacks go
 * through a static host buffer.  params->dense_threads must be fixed (64, 128, 256
 * or 512), params->pcg_threads not -1, and params->timing and params->graph 0
 * (else BF_ERR_UNSUPPORTED).
 *
 * Every call on a GPU uses that GPU's one array: calls are serialised by a
 * process-wide lock and each call finishes its device work before releasing it;
 * the array keeps the last call's contents, and a call clears what it needs
 * cleared.  Work of other libraries that writes the array's memory would race with
 * it (nothing outside this entry point touches it).  The context's own
 * workspace and state are neither used nor changed.
 */
bf_status bf_gauss_newton_noalloc(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                                  const bf_corrs* corrs, const bf_pairs* pairs, const double* init_poses,
                                  const bf_params* params, double* out_poses, double* out_energy,
                                  double* out_trace);

/*
 * Key-point correspondence filter and surface-area filter (Sec. 4.1.1), run on
 * candidate correspondences before a solve.  Per unordered frame pair, the
 * candidates in their given order (the order of match distance) are added one at
 * a time; after each addition, while the set has at least 3 members, the least-
 * RMSD rigid transform (Kabsch) is computed and the set must have its largest
 * residual at most max_res (paper: 0.02 m) and be well determined: the ratio of
 * the largest to the second largest eigenvalue of the covariance of each side's
 * points, and of the largest to the second largest singular value of their
 * cross-covariance, at most max_cond (paper: 100); otherwise the member with the
 * largest residual is removed.  The pair keeps its final set if it passed with at
 * least max(min_count, 3) members (paper: 5) and each side's points span at least
 * min_area (paper: 0.032 m^2) as the box along their two principal axes.
 *   num_frames: frame indices of `corrs` must lie in [0, num_frames), i != j.
 *   out_keep (device) [M] uint8: 1 = kept.  out_kept (host, may be NULL): count.
 * Synchronises the stream.
 */
bf_status bf_filter_correspondences(bf_context* ctx, const bf_corrs* corrs, int32_t num_frames, double max_res,
                                   double max_cond, int32_t cond_mode, int32_t min_count, double min_area,
                                   uint8_t* out_keep, int64_t* out_kept);

/*
 * Dense two-sided verification of frame pairs (Sec. 4.1.1, "Dense Verification"),
 * e.g. of every pair of a chunk after its solve.  For each pair (i, j) and the
 * relative transform of `poses`, each pixel of i with a valid normal is associated
 * with the nearest pixel of j as in the dense term (FP32 decisions, tau_dist and
 * tau_normal of `params`) and must also satisfy |C_i(x,y) - C_j(x',y')| < tau_c
 * (intensities of `frames`); the re-projection errors |T_ji p - q| of the valid
 * associations are summed; likewise from j to i.  A pair is valid when in both
 * directions at least min_frac * W * H associations are valid and their mean
 * error is at most max_err (the paper: tau_c = 0.1, max_err = 0.075 m, min_frac =
 * 0.02).  Pairs need not be sorted; i != j, both in range.
 *   out_stats (device) [P][4] float64: error sum and count of i->j, then of j->i;
 *   out_valid (device) [P] uint8.  Synchronises the stream.
 */
bf_status bf_verify_pairs(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                          const bf_pairs* pairs, const double* poses, const bf_params* params, double tau_c,
                          double max_err, double min_frac, double* out_stats, uint8_t* out_valid);

/*
 * Solve with residual pruning (Sec. 4.4.1): after each full solve (as
 * bf_gauss_newton), the largest sparse residual |T_i p - T_j q| (metres, FP64)
 * over the active correspondences is found (per-workgroup candidates, final
 * maximum on the host; ties go to the smallest correspondence index).  If it
 * exceeds r_prune, every correspondence between that correspondence's two frames
 * is deactivated, a frame that had correspondences and has none left is marked
 * invalid (its dense pairs are dropped, its pose is kept), and the problem is
 * solved again from the current poses.  Stops when the largest residual is at
 * most r_prune or after max_rounds removals.  The dense pair set is fixed in the
 * first round (`pairs`, or the pair test at init_poses).
 *   out_poses (device) [F][4][4]; out_energy (host) [4] of the last solve;
 *   out_corr_active (device, may be NULL) [M] uint8: 1 = still active;
 *   out_frame_valid (device, may be NULL) [F] uint8: 0 = removed by pruning;
 *   out_rounds (host, may be NULL): removals done; out_rmax (host, may be NULL):
 *   the largest active residual at the returned poses (-1 if none is active).
 */
bf_status bf_gauss_newton_pruned(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                                 const bf_corrs* corrs, const bf_pairs* pairs, const double* init_poses,
                                 const bf_params* params, double r_prune, int32_t max_rounds, double* out_poses,
                                 double* out_energy, uint8_t* out_corr_active, uint8_t* out_frame_valid,
                                 int32_t* out_rounds, double* out_rmax);

/*
 * y = H x with the J^T J matrix of `sys` (all frames, 6F, frame 0 included), for
 * comparing representations (Sec. 4.4):
 *   mode 0: from the assembled per-edge 6x6 blocks (what the PCG kernels use);
 *   mode 1: the sparse term only, matrix-free as the paper does it: J x per
 *           correspondence, then J^T per frame over the frame's correspondences.
 *           `corrs` must be the correspondences the system was built from.  With a
 *           system built with use_dense = 0 both modes give the same product.
 * x, y: device [6F] float64.  out_us (host, may be NULL): time of the product's
 * kernels.  Synchronises the stream.
 */
bf_status bf_system_matvec(bf_context* ctx, const bf_system* sys, const bf_corrs* corrs, const double* x, double* y,
                           int32_t mode, double* out_us);

/*
 * Many independent problems in one call (Sec. 4.1: every chunk's intra-chunk
 * alignment is its own solve of the same energy).  Problem b owns the consecutive
 * frames [frame_offsets[b], frame_offsets[b+1]) of `frames`; its first frame is
 * its fixed gauge frame.  Correspondences and caller-given pairs use indices into
 * the concatenated frames and must not connect two problems (BF_ERR_INVALID_ARG).
 * All problems share the intrinsics and params; every kernel launch covers all
 * problems (dense pair jobs of all problems in one grid, one PCG workgroup per
 * problem), and each problem's result is the result it gets alone up to rounding
 * (bitwise the same with a fixed params->dense_threads).
 *   frame_offsets (host) [num_problems + 1], 0 = first, strictly increasing, last =
 *                 frames->num_frames.
 *   out_poses (device) [F][4][4]; out_energy (host) [num_problems][4];
 *   out_trace (host, may be NULL) [num_problems][num_gn][4].
 * params->solve_kernel must be 0 or 4.
 */
bf_status bf_gauss_newton_batch(bf_context* ctx, const bf_frames* frames, const bf_intrinsics* intr,
                                const bf_corrs* corrs, const bf_pairs* pairs, int32_t num_problems,
                                const int32_t* frame_offsets, const double* init_poses,
                                const bf_params* params, double* out_poses, double* out_energy,
                                double* out_trace);

/* Microseconds spent in each phase of the last bf_gauss_newton() call run with
 * params->timing = 1, measured with HIP events on the context's stream (host out,
 * [8]): setup, dense pair jobs (sum over iterations), edge blocks, assembly,
 * PCG + update, final energy, total, and the number of dense pair-job launches.
 * With params->timing = 2 only the dense pair jobs, the total and the launch count
 * are measured (the other phases read 0). */
bf_status bf_last_timings(const bf_context* ctx, double* out_us);

/* Workgroup size of this context's last per-problem PCG launch (params->pcg_threads
 * fixed, or the timed choice); 0 before any (host out, [1]). */
bf_status bf_pcg_threads(const bf_context* ctx, int32_t* out_threads);

/* Device memory held by this context's workspace, in bytes (host out, [1]): the sum
 * of its buffers' capacities.  They grow on demand (by a quarter more than asked)
 * and are kept until bf_destroy; inputs the caller owns are not counted.  A
 * caller that admits work by memory footprint can check its estimate against it. */
bf_status bf_workspace_bytes(const bf_context* ctx, int64_t* out_bytes);

/* Launch shape of this context's last dense pair-job launch with Jacobians and of
 * its last one without (the energy at the returned poses), as the caller fixed it
 * (params->dense_threads, params->dense_tiles) or the timing chose it (host out,
 * [4]): threads per workgroup, tiles per job, then the same for the energy-only
 * launch; zeros before any launch. */
bf_status bf_dense_shape(const bf_context* ctx, int32_t* out_shape);

/* Number of times this context has captured the Gauss-Newton loop into a HIP
 * graph (params->graph = 1); a call that replays the captured loop leaves it
 * unchanged.  -1 for a NULL context. */
int64_t bf_graph_captures(const bf_context* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BF_H */
