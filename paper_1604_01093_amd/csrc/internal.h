// Host-side context, workspace and launch declarations of libbf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace bf {

// A device buffer that only grows.
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct Error {
  bf_status status;
  std::string msg;
};

// Per-solve structure sizes (host copies of the device-side counts).
struct Shape {
  int F = 0, W = 0, H = 0;
  int64_t M = 0;            // correspondences
  int64_t P = 0;            // dense pair jobs
  int64_t S = 0;            // sparse pairs (distinct unordered frame pairs with correspondences)
  int64_t E = 0;            // edges (union)
  int64_t nfree = 0;        // free frames
  int nseg = 1;             // independent problems (segments of consecutive frames)
  int64_t max_seg_free = 0; // most free frames in one segment
};

struct Context {
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 0;
  std::string last_error;
  Shape shape;
  int pcg_storage = 0;
  int precond = 0;          // 0 = 6x6 block-Jacobi, 1 = scalar Jacobi
  int bidir = 0;            // 1: two dense pair jobs per pair (i -> j, then j -> i at job P + p)
  unsigned spin_limit = 1u << 26;  // polls before a PCG kernel's wait for other workgroups gives up
  int dense_tiles = 1;      // tiles per dense pair job of the last dense launch (records per job)
  double mf_w_sparse = 0.0; // sparse weight of the matrix-free sparse PCG product
  int dense_shape_last[4] = {0, 0, 0, 0};  // threads, tiles of the last dense launch with / without Jacobians
  double timings[8] = {0};

  // frames
  Buf nd, grad, kx, ky, kx64, ky64;
  // pairs
  Buf pair_flags, row_count, row_off, pairs, pair_keys;
  // correspondences
  Buf corr_key, corr_idx, corr_key_sorted, corr_perm, corr_head, corr_group, sparse_ij, sparse_keys, sparse_ptr,
      moments;
  // edges and incidence
  Buf in_b, common_scan, edge_ij, edge_keys, edge_dense, edge_sparse, ej_key, ej_idx, ej_key_sorted, ej_sorted,
      iptr, jptr, free_flag, var_of, frame_of_var, row_cnt, row_ptr, row_entries;
  // per-iteration data
  Buf records, eblocks, hij32, hij64, diag32, diag64, minv32, minv64, rhs, poses_work, pcg_vec, stats, trace;
  // residual pruning: active correspondences, frame counts and validity, compacted
  // correspondences and pairs, reduction candidates, the round's poses
  Buf pr_active, pr_cnt0, pr_cnt, pr_valid, pr_flag, pr_pos, pr_fi, pr_fj, pr_pi, pr_pj, pr_pflag, pr_ppos, pr_pairs,
      pr_pairs_all, pr_bval, pr_bidx, pr_poses;
  // the poses and sparse weight of the last assembled system; matrix-free scratch
  Buf sys_poses, mf_u;
  // matrix-free sparse PCG: sorted correspondence points, per-pair sums, dense diagonal parts
  Buf mf_pts, mf_y, ediag_dense;
  Buf dist_slots;  // reduction slots of the distributed-vector PCG
  Buf energy_parts;  // partial energy sums of a large problem
  double sys_w_sparse = 0.0;
  // independent problems: frame offsets, segment of each frame, variable and edge ranges
  Buf seg_start, seg_of, seg_var_ptr, seg_edge_ptr;
  std::vector<int> seg_host;  // offsets currently on the device (seg_start, seg_of)
  // scratch
  Buf cub_tmp, counts, flags, energy, pcg_partials, pcg_barrier, pcg_tags;
  // pinned host memory for device-to-host readbacks (a copy into pageable memory is
  // staged by the runtime and costs a round trip of its own): a fixed small area
  // for counts and flags and a growing one for per-problem arrays
  long long* rb_small = nullptr;
  void* rb_big = nullptr;
  size_t rb_big_cap = 0;
  // threads per dense pair job chosen by timing, per (pixels per frame, precision mode, Jacobians)
  std::map<long long, int> dense_threads;
  int pcg_threads = 0;                   // per-problem PCG workgroup size: 0 = 256, -1 = timed, else fixed
  bool in_capture = false;               // the Gauss-Newton loop is being captured into a graph
  int pcg_threads_last = 0;              // workgroup size of the last per-problem PCG launch
  std::map<long long, int> pcg_threads_timed;  // timed choices by (storage, problem count range, largest problem)
  int pcg_grid = 0;       // workgroups of the cooperative PCG kernel (0 = not yet chosen)
  // replicated-vector PCG: exchange tags used so far since the last clear
  unsigned pcg_tag_base = 0;
  unsigned dist_tag_base = 0;        // reduction tags of the distributed-vector PCG
  void* dist_slots_ptr = nullptr;
  void* pcg_tags_ptr = nullptr;
  bool pcg_tags_dirty = true;
  int solve_mode = 0;     // 0 = automatic, 1 = single workgroup, 2 = cooperative, 3 = replicated vectors,
                          // 4 = per problem, 5 = distributed vectors
  // the Gauss-Newton loop captured as a HIP graph: the instantiated graph, the
  // launch arguments it was captured with, and the stream capture runs on
  hipGraphExec_t gn_exec = nullptr;
  std::vector<unsigned char> gn_key;
  hipStream_t capture_stream = nullptr;
  long long gn_captures = 0;

  hipEvent_t ev[16] = {};
  bool events_ready = false;
};

// Error helpers: throw an Error from host code; the C entry points catch it.
[[noreturn]] void fail(bf_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);
void ensure(Buf& b, size_t bytes);
// Pinned host readback areas: kSmallReadbackWords words, and one of at least `bytes`.
constexpr int kSmallReadbackWords = 16;
long long* readback_small(Context& c);
void* readback_big(Context& c, size_t bytes);
// Count of workspace (re)allocations so far, in every context: a captured graph
// holds buffer addresses and is valid only while this count is unchanged.
unsigned long long alloc_generation();
// Contexts currently alive in the process: with more than one, kernels whose
// workgroups wait for each other are launched cooperatively (their co-residency is
// then guaranteed even while another context's kernels run).
int live_contexts();

// prep.hip
void launch_prepare(Context& c, const bf_frames& fr, const bf_intrinsics& in, const bf_params& prm);

// structure.hip
// Segments: frames [offsets[b], offsets[b+1]) form independent problem b (host array
// of nseg + 1 entries; nullptr = one problem of all frames).
void set_segments(Context& c, int F, const int32_t* offsets, int nseg);
int64_t group_correspondences(Context& c, const bf_corrs& co, int F);
void build_structure(Context& c, const bf_frames& fr, const bf_intrinsics& in, const bf_corrs* co,
                     const bf_pairs* pairs, const double* poses, const bf_params& prm);
int64_t launch_pair_search(Context& c, const bf_frames& fr, const bf_intrinsics& in, const double* poses,
                           const bf_params& prm);

// dense.hip
// assoc_out (may be null): per job and source pixel the association taken, two
// words ([jobs][H*W][2]): target pixel << 2 | photometric << 1 | geometric, and the
// first pixel of the bilinear footprint.  prm.fixed_association, when set, gives
// the association instead of deciding it (same layout).
void launch_dense(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                  bool with_jacobians, unsigned* assoc_out = nullptr);
// Launch shape launch_dense() will use, threads * 16 + tiles per job (timing the
// candidates first when params.dense_threads is 0 and the shape is new in this
// context); also sizes the records for it.
// Workgroup size of the per-problem PCG kernel for the current system (timed when
// asked for and allowed and not yet known).
int per_problem_pcg_threads(Context& c, bool may_time, int iters = 0);
int dense_threads_for(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                      bool with_jacobians);
// Whole-job records [jobs][kRecWords] of the last dense launch (its tiles summed).
void export_records(Context& c, double* out);

// solve.hip
void launch_edge_blocks(Context& c, const double* poses, const bf_params& prm, bool with_jacobians);
// Correspondence points in sorted order for the matrix-free sparse PCG.
void launch_mf_points(Context& c, const bf_corrs* co);
void launch_solve(Context& c, int iters, double* trace_slot, double* delta_out, double* poses_inout, double* stats,
                  bool update_poses, bool sparse_matrix_free = false);
void launch_energy(Context& c, double* dst8);
// The energy words of one problem with many edges, summed on several workgroups.
void launch_energy_split(Context& c, double* dst8);
// Whether the PCG of the current structure runs in the per-problem kernel (no state
// carried between launches, so it can be captured in a graph); prepare_solve()
// makes the one-time kernel attribute settings that capture must not make.
bool solve_per_problem(const Context& c);
void prepare_solve(Context& c);
void launch_export_dense(Context& c, double* H, double* g);

// filter.hip: key-point and surface-area filters over grouped correspondences
void launch_filters(Context& c, const bf_corrs& co, long long S, double max_res, double max_cond, int min_count,
                    double min_area, int cond_mode, uint8_t* keep);

// verify.hip: two-sided dense verification of frame pairs (frames prepared)
void launch_verify(Context& c, const bf_frames& fr, const bf_intrinsics& in, const int* pairs, long long P,
                   const double* poses, const bf_params& prm, double tau_c, double max_err, double min_frac,
                   double* stats, uint8_t* valid);

// prune.hip: residual pruning state and steps
void prune_init(Context& c, const bf_corrs& co, int F);
bf_corrs prune_active_corrs(Context& c, const bf_corrs& co);
bf_pairs prune_valid_pairs(Context& c, const int* ij, long long P);
double prune_max_residual(Context& c, const bf_corrs& co, const double* poses, long long* idx);
void prune_drop(Context& c, const bf_corrs& co, int F, int a, int b);

// matvec.hip: y = H x of the last assembled system; mode 0 from the edge blocks,
// mode 1 the sparse term matrix-free (J^T (J x)) over the correspondences `co`.
void launch_matvec(Context& c, const bf_corrs* co, double w_sparse, int mode, const double* x, double* y);

}  // namespace bf
