// C entry points of libbf (declared and documented in include/bf.h).
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

struct bf_context : bf::Context {
  std::vector<hipEvent_t> pool;
  // state of bf_gauss_newton_noalloc: a context whose workspace is carved from
  // the static scratch array (reset at every call; nullptr inside itself)
  bf_context* noalloc = nullptr;
};

// Normal equations built by bf_build_normal_equations: the assembled per-edge
// blocks and everything the PCG, the dense export and the matrix-free product read
// (incidence, row lists, variable maps, segment ranges), owned by the system.  A
// context works on a system by exchanging these buffers with its own for the
// duration of a call (pointer swaps, no copies).
struct bf_system {
  bf_context* owner = nullptr;
  hipStream_t stream = nullptr;  // the owner's stream, synchronised before the buffers are freed
  bool built = false;
  bf::Shape shape;
  int pcg_storage = 0, precond = 0, solve_mode = 0, bidir = 0, pcg_threads = 0;
  unsigned spin_limit = 1u << 26;
  double w_sparse = 0.0;
  bf::Buf eblocks, hij32, hij64, edge_ij, iptr, jptr, ej_sorted, row_ptr, row_entries, frame_of_var, var_of,
      seg_var_ptr, seg_edge_ptr, seg_start, seg_of, sys_poses, corr_perm, corr_group, sparse_ij, sparse_ptr,
      edge_sparse;
};

namespace bf {

void fail(bf_status s, const std::string& msg) { throw Error{s, msg}; }

// ----------------------------------------------------------------------------
// Workspace for bf_gauss_newton_noalloc: one static device array per GPU, of a
// fixed size, instead of hipMalloc.  In host code `scratch` only names the
// host-side stand-in of the array; its device address is looked up once per
// device (hipGetSymbolAddress, in bf_create with that device current) and only
// that address is ever handed to kernels or copies.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                     // guards the per-device lookup
void* g_scratch_ptr[kMaxDevices] = {};
int g_scratch_state[kMaxDevices] = {};       // 0 not looked up, 1 found, -1 lookup failed

// A bump allocator over the scratch array, active for the duration of one
// allocation-free call on the calling thread: ensure() carves from it and the
// pinned readback areas are replaced by static host memory.
struct Arena {
  char* base;
  size_t cap, off;
};
thread_local Arena* t_arena = nullptr;
constexpr size_t kArenaHostBytes = (size_t)256 << 10;
alignas(64) unsigned char g_arena_host[kArenaHostBytes];  // readback staging; calls are serialised
std::mutex g_noalloc_mu;                                   // one allocation-free call at a time
}  // namespace

void lookup_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_state[device] != 0) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr != nullptr) {
    g_scratch_ptr[device] = ptr;
    g_scratch_state[device] = 1;
  } else {
    (void)hipGetLastError();
    g_scratch_state[device] = -1;
  }
}

void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || g_scratch_state[device] != 1)
    fail(BF_ERR_DEVICE, "the static scratch array of this device could not be located");
  return g_scratch_ptr[device];
}

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(BF_ERR_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
    fail(BF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

namespace {
std::atomic<unsigned long long> g_alloc_generation{0};  // contexts may live on different threads
std::atomic<int> g_live_contexts{0};
}  // namespace

int live_contexts() { return g_live_contexts.load(); }

unsigned long long alloc_generation() { return g_alloc_generation.load(); }

// Buffers changed hands without an allocation (a system exchanged with the
// context): a captured graph holding their old addresses must be recaptured.
void bump_alloc_generation() { ++g_alloc_generation; }

void ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return;
  if (t_arena) {
    const size_t off = (t_arena->off + 255) & ~(size_t)255;
    if (off > t_arena->cap || bytes > t_arena->cap - off)
      fail(BF_ERR_OUT_OF_MEMORY, "the problem needs more than the " + std::to_string(t_arena->cap >> 20) +
                                     " MiB scratch array of the allocation-free entry point");
    b.p = t_arena->base + off;
    b.cap = bytes;
    t_arena->off = off + bytes;
    return;
  }
  ++g_alloc_generation;
  if (b.p) {
    check_hip(hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.cap = 0;
  }
  size_t cap = bytes + bytes / 4;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cap);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(BF_ERR_OUT_OF_MEMORY, "workspace allocation of " + std::to_string(cap) + " bytes failed");
  }
  b.p = p;
  b.cap = cap;
}

long long* readback_small(Context& c) {
  if (t_arena) return reinterpret_cast<long long*>(g_arena_host);
  if (!c.rb_small) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(long long) * kSmallReadbackWords, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      fail(BF_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
    }
    c.rb_small = static_cast<long long*>(p);
  }
  return c.rb_small;
}

void* readback_big(Context& c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (t_arena) {
    constexpr size_t kSmall = 4096;  // the small area stays at the start
    if (bytes > kArenaHostBytes - kSmall) fail(BF_ERR_UNSUPPORTED, "readback too large for the allocation-free entry point");
    return g_arena_host + kSmall;
  }
  if (c.rb_big_cap < bytes) {
    if (c.rb_big) {
      check_hip(hipStreamSynchronize(c.stream), "synchronise");
      check_hip(hipHostFree(c.rb_big), "hipHostFree");
      c.rb_big = nullptr;
      c.rb_big_cap = 0;
    }
    const size_t cap = bytes + bytes / 4;
    void* p = nullptr;
    if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      fail(BF_ERR_OUT_OF_MEMORY, "pinned host allocation of " + std::to_string(cap) + " bytes failed");
    }
    c.rb_big = p;
    c.rb_big_cap = cap;
  }
  return c.rb_big;
}

namespace {

__global__ void k_check_poses(const double* __restrict__ poses, int F, int* __restrict__ flags) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < F * 16 && !isfinite(poses[k])) raise_flag(flags, kFlagNonFinite);
}

__global__ void k_check_pair_range(const int* __restrict__ ij, long long P, int F, int* __restrict__ flags) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const int i = ij[2 * k], j = ij[2 * k + 1];
  if (!(i >= 0 && i < F && j >= 0 && j < F && i != j)) raise_flag(flags, kFlagBadIndex);
}

__global__ void k_copy_d(const double* __restrict__ src, double* __restrict__ dst, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

__global__ void k_copy_if_ok(const double* __restrict__ src, double* __restrict__ dst, int n,
                             const int* __restrict__ flags) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && flags[0] == 0) dst[k] = src[k];
}

void validate_common(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_params* prm) {
  if (!ctx) fail(BF_ERR_INVALID_ARG, "null context");
  if (!fr || !in || !prm) fail(BF_ERR_INVALID_ARG, "null frames, intrinsics or params");
  if (fr->num_frames < 1) fail(BF_ERR_INVALID_ARG, "num_frames must be >= 1");
  if (fr->num_frames > 16384) fail(BF_ERR_UNSUPPORTED, "more than 16384 frames");
  if (!fr->depth || !fr->intensity) fail(BF_ERR_INVALID_ARG, "null depth or intensity");
  if (in->width < 3 || in->height < 3 || in->width > 4096 || in->height > 4096)
    fail(BF_ERR_INVALID_ARG, "image size must be within [3, 4096]");
  if (!(in->fx > 0) || !(in->fy > 0) || !isfinite(in->fx) || !isfinite(in->fy) || !isfinite(in->cx) ||
      !isfinite(in->cy))
    fail(BF_ERR_INVALID_ARG, "bad intrinsics");
  if ((int64_t)in->width * in->height * fr->num_frames > (int64_t)1 << 34) fail(BF_ERR_UNSUPPORTED, "frames too large");
  if (prm->num_gn < 0 || prm->num_gn > 1000 || prm->num_pcg < 0 || prm->num_pcg > 100000)
    fail(BF_ERR_INVALID_ARG, "iteration counts out of range");
  if (!(prm->w_sparse >= 0) || !(prm->w_dense >= 0) || !(prm->w_geo >= 0) || !(prm->w_photo >= 0) ||
      !isfinite(prm->w_sparse) || !isfinite(prm->w_dense) || !isfinite(prm->w_geo) || !isfinite(prm->w_photo))
    fail(BF_ERR_INVALID_ARG, "weights must be finite and >= 0");
  if (prm->accumulate < 0 || prm->accumulate > 2) fail(BF_ERR_INVALID_ARG, "accumulate must be 0, 1 or 2");
  if (prm->timing < 0 || prm->timing > 2) fail(BF_ERR_INVALID_ARG, "timing must be 0, 1 or 2");
  if (prm->pcg_storage != 0 && prm->pcg_storage != 1) fail(BF_ERR_INVALID_ARG, "pcg_storage must be 0 or 1");
  if (prm->solve_kernel < 0 || prm->solve_kernel > 5) fail(BF_ERR_INVALID_ARG, "solve_kernel must be 0..5");
  if (prm->preconditioner != 0 && prm->preconditioner != 1) fail(BF_ERR_INVALID_ARG, "preconditioner must be 0 or 1");
  if (prm->graph != 0 && prm->graph != 1) fail(BF_ERR_INVALID_ARG, "graph must be 0 or 1");
  if (prm->bidirectional != 0 && prm->bidirectional != 1) fail(BF_ERR_INVALID_ARG, "bidirectional must be 0 or 1");
  if (prm->pcg_spin_limit < 0) fail(BF_ERR_INVALID_ARG, "pcg_spin_limit must be >= 0");
  if (prm->sparse_matrix_free != 0 && prm->sparse_matrix_free != 1)
    fail(BF_ERR_INVALID_ARG, "sparse_matrix_free must be 0 or 1");
  if (prm->sparse_matrix_free && prm->solve_kernel != 0 && prm->solve_kernel != 5)
    fail(BF_ERR_UNSUPPORTED, "the matrix-free sparse term runs in the distributed-vector PCG (solve_kernel 0 or 5)");
  if (prm->sparse_matrix_free && prm->graph)
    fail(BF_ERR_UNSUPPORTED, "the matrix-free sparse term is not replayed as a graph");
  if (prm->dense_tiles < 0 || prm->dense_tiles > 16) fail(BF_ERR_INVALID_ARG, "dense_tiles must be within [0, 16]");
  if (prm->pcg_threads != -1 && prm->pcg_threads != 0 && prm->pcg_threads != 64 && prm->pcg_threads != 128 &&
      prm->pcg_threads != 256 && prm->pcg_threads != 1024)
    fail(BF_ERR_INVALID_ARG, "pcg_threads must be -1, 0, 64, 128, 256 or 1024");
  if (prm->dense_threads != 0 && prm->dense_threads != 64 && prm->dense_threads != 128 &&
      prm->dense_threads != 256 && prm->dense_threads != 512)
    fail(BF_ERR_INVALID_ARG, "dense_threads must be 0, 64, 128, 256 or 512");
  if (!(prm->tau_dist > 0) || !isfinite(prm->tau_normal) || !(prm->depth_max > prm->depth_min) ||
      !isfinite(prm->max_angle_deg))
    fail(BF_ERR_INVALID_ARG, "bad thresholds");
}

void validate_corrs(const bf_corrs* co) {
  if (co) {
    if (co->count < 0) fail(BF_ERR_INVALID_ARG, "negative correspondence count");
    if (co->count > 0 && (!co->frame_i || !co->frame_j || !co->p_i || !co->p_j))
      fail(BF_ERR_INVALID_ARG, "null correspondence arrays");
    if (co->count > ((int64_t)1 << 31) - 2) fail(BF_ERR_UNSUPPORTED, "too many correspondences");
  }
}

void validate_problem(const bf_corrs* co, const bf_pairs* pairs, const double* poses) {
  if (!poses) fail(BF_ERR_INVALID_ARG, "null poses");
  validate_corrs(co);
  if (pairs) {
    if (pairs->count < 0) fail(BF_ERR_INVALID_ARG, "negative pair count");
    if (pairs->count > 0 && !pairs->ij) fail(BF_ERR_INVALID_ARG, "null pair array");
  }
}

double dense_weight(const bf_params& p, int k) {
  if (!p.dense_ramp || p.num_gn <= 0) return p.w_dense;
  return p.w_dense * (double)(k + 1) / (double)p.num_gn;
}

void check_poses(Context& c, const double* poses, int F) {
  ensure(c.flags, sizeof(int));
  hipLaunchKernelGGL(k_check_poses, dim3((F * 16 + 255) / 256), dim3(256), 0, c.stream, poses, F, c.flags.as<int>());
}

void ensure_pcg_buffers(Context& c);

// Structure + per-iteration buffers for the current shape (offsets: host frame
// offsets of nseg independent problems, or nullptr for one problem).
void setup(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co, const bf_pairs* pairs,
           const double* poses, const bf_params* prm, const int32_t* offsets = nullptr, int nseg = 1) {
  Context& c = *ctx;
  c.pcg_storage = prm->pcg_storage;
  c.solve_mode = prm->solve_kernel;
  c.precond = prm->preconditioner;
  c.bidir = prm->bidirectional;
  c.spin_limit = prm->pcg_spin_limit > 0 ? (unsigned)prm->pcg_spin_limit : (1u << 26);
  c.pcg_threads = prm->pcg_threads;
  ensure(c.counts, 8 * sizeof(long long));
  ensure(c.flags, sizeof(int));
  set_segments(c, fr->num_frames, offsets, nseg);
  build_structure(c, *fr, *in, co, pairs, poses, *prm);
  const Shape& s = c.shape;
  c.mf_w_sparse = prm->use_sparse ? prm->w_sparse : 0.0;
  if (prm->sparse_matrix_free) launch_mf_points(c, co);
  ensure(c.records, sizeof(double) * kRecWords * ((c.bidir ? 2 : 1) * s.P + 1));
  ensure(c.eblocks, sizeof(double) * kEdgeWords * (s.E + 1));
  ensure_pcg_buffers(c);
  ensure(c.trace, sizeof(double) * 8 * s.nseg * (prm->num_gn + 1));
}

// PCG storage and scratch for the current shape (off-diagonal blocks, diagonal
// blocks and inverses, right-hand side, vectors) and the per-problem outputs.
void ensure_pcg_buffers(Context& c) {
  const Shape& s = c.shape;
  if (c.pcg_storage == 1) {
    ensure(c.hij64, sizeof(double) * 36 * (s.E + 1));
    ensure(c.diag64, sizeof(double) * 36 * (s.nfree + 1));
    ensure(c.minv64, sizeof(double) * 36 * (s.nfree + 1));
    ensure(c.rhs, sizeof(double) * 6 * (s.nfree + 1));
    ensure(c.pcg_vec, sizeof(double) * 6 * 6 * (s.nfree + 1));
  } else {
    ensure(c.hij32, sizeof(float) * 36 * (s.E + 1));
    ensure(c.diag32, sizeof(float) * 36 * (s.nfree + 1));
    ensure(c.minv32, sizeof(float) * 36 * (s.nfree + 1));
    ensure(c.rhs, sizeof(float) * 6 * (s.nfree + 1));
    ensure(c.pcg_vec, sizeof(float) * 6 * 6 * (s.nfree + 1));
  }
  ensure(c.energy, sizeof(double) * 8 * s.nseg);
  ensure(c.stats, sizeof(double) * 4 * s.nseg);
}

// Exchange the system's buffers and sizes with the context's (see bf_system).
void swap_system(Context& c, bf_system& y) {
  std::swap(c.eblocks, y.eblocks);
  std::swap(c.hij32, y.hij32);
  std::swap(c.hij64, y.hij64);
  std::swap(c.edge_ij, y.edge_ij);
  std::swap(c.iptr, y.iptr);
  std::swap(c.jptr, y.jptr);
  std::swap(c.ej_sorted, y.ej_sorted);
  std::swap(c.row_ptr, y.row_ptr);
  std::swap(c.row_entries, y.row_entries);
  std::swap(c.frame_of_var, y.frame_of_var);
  std::swap(c.var_of, y.var_of);
  std::swap(c.seg_var_ptr, y.seg_var_ptr);
  std::swap(c.seg_edge_ptr, y.seg_edge_ptr);
  std::swap(c.seg_start, y.seg_start);
  std::swap(c.seg_of, y.seg_of);
  std::swap(c.sys_poses, y.sys_poses);
  std::swap(c.corr_perm, y.corr_perm);
  std::swap(c.corr_group, y.corr_group);
  std::swap(c.sparse_ij, y.sparse_ij);
  std::swap(c.sparse_ptr, y.sparse_ptr);
  std::swap(c.edge_sparse, y.edge_sparse);
  std::swap(c.shape, y.shape);
  std::swap(c.pcg_storage, y.pcg_storage);
  std::swap(c.precond, y.precond);
  std::swap(c.solve_mode, y.solve_mode);
  std::swap(c.bidir, y.bidir);
  std::swap(c.spin_limit, y.spin_limit);
  std::swap(c.pcg_threads, y.pcg_threads);
  std::swap(c.sys_w_sparse, y.w_sparse);
  c.seg_host.clear();  // the segment arrays on the device changed hands
  bump_alloc_generation();
}

// A system lent to the context for one call and taken back on every exit path.
struct SystemLoan {
  Context& c;
  bf_system& y;
  SystemLoan(Context& cc, const bf_system* sys) : c(cc), y(*const_cast<bf_system*>(sys)) {
    swap_system(c, y);
    try {
      ensure_pcg_buffers(c);
    } catch (...) {
      swap_system(c, y);
      throw;
    }
  }
  ~SystemLoan() { swap_system(c, y); }
};

void check_system(const bf_context* ctx, const bf_system* sys) {
  if (!sys) fail(BF_ERR_INVALID_ARG, "null system");
  if (sys->owner != ctx) fail(BF_ERR_INVALID_ARG, "the system belongs to another context");
  if (!sys->built) fail(BF_ERR_INVALID_ARG, "the system has not been built");
}

void sync_and_flags(Context& c, int* hf) {
  int* rb = reinterpret_cast<int*>(readback_small(c));
  check_hip(hipMemcpyAsync(rb, c.flags.p, sizeof(int), hipMemcpyDeviceToHost, c.stream), "copy flags");
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  *hf = *rb;
  if (*hf & kFlagTimeout) c.pcg_tags_dirty = true;  // a solve stopped early: clear its exchange state
}

void raise_flags(int fl) {
  if (fl & kFlagBadIndex) fail(BF_ERR_INVALID_ARG, "index out of range");
  if (fl & kFlagUnsorted) fail(BF_ERR_INVALID_ARG, "dense pairs are not strictly increasing");
  if (fl & kFlagNonFinite) fail(BF_ERR_NONFINITE, "non-finite input");
  if (fl & kFlagShape)
    fail(BF_ERR_UNSUPPORTED, "the distributed-vector PCG cannot split this problem's rows (solve_kernel 2 can)");
  // a wait that gave up leaves partial sums behind: other flags of that launch are not reliable
  if (fl & kFlagTimeout) fail(BF_ERR_DEVICE, "grid barrier of the PCG kernel did not complete");
  if (fl & kFlagNotPD) fail(BF_ERR_NOT_PD, "a diagonal block of J^T J is not positive definite");
}

// HIP events on the context's stream.  Level 1 marks every phase; level 2 only the
// dense launches and the whole call.  The events only time (their elapsed times are
// read after the call's final synchronisation), so they are recorded without the
// system-scope fence a default event carries: that fence's cache write-back and
// invalidation left the GPU idle for about 5 us per event.
struct Timer {
  bf_context* ctx;
  bool on;
  int level;
  std::vector<std::pair<int, int>> spans[6];
  int used = 0;
  Timer(bf_context* c, int lvl) : ctx(c), on(lvl != 0), level(lvl) {}
  // a mark of the phases beyond the dense launches (level 1 only)
  int mark_phase() { return level == 1 ? mark() : -1; }
  int mark() {
    if (!on) return -1;
    if (used >= (int)ctx->pool.size()) {
      hipEvent_t e;
      check_hip(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreateWithFlags");
      ctx->pool.push_back(e);
    }
    check_hip(hipEventRecord(ctx->pool[used], ctx->stream), "hipEventRecord");
    return used++;
  }
  void span(int slot, int a, int b) {
    if (on && a >= 0 && b >= 0) spans[slot].push_back({a, b});
  }
  void finish(double* out) {
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    if (!on) return;
    for (int s = 0; s < 6; ++s)
      for (auto& ab : spans[s]) {
        float ms = 0.f;
        check_hip(hipEventElapsedTime(&ms, ctx->pool[ab.first], ctx->pool[ab.second]), "hipEventElapsedTime");
        out[s] += 1000.0 * ms;
      }
    out[7] = (double)spans[1].size();
  }
};

template <class Fn>
bf_status guarded(bf_context* ctx, Fn fn) {
  try {
    fn();
    if (ctx) ctx->last_error.clear();
    return BF_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "host allocation failed";
    return BF_ERR_OUT_OF_MEMORY;
  } catch (...) {
    if (ctx) ctx->last_error = "unexpected exception";
    return BF_ERR_DEVICE;
  }
}

}  // namespace
}  // namespace bf

using namespace bf;

extern "C" {

void bf_params_default(bf_params* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->w_sparse = 1.0;
  o->w_dense = 1.0;
  o->w_geo = 1.0;
  o->w_photo = 1.178;
  o->dense_ramp = 1;
  o->use_sparse = 1;
  o->use_dense = 1;
  o->num_gn = 5;
  o->num_pcg = 10;
  o->accumulate = 0;
  o->pcg_storage = 0;
  o->timing = 0;
  o->solve_kernel = 0;
  o->dense_threads = 0;
  o->tau_dist = 0.15;
  o->tau_normal = 0.9;
  o->max_angle_deg = 60.0;
  o->depth_min = 0.1;
  o->depth_max = 10.0;
}

bf_status bf_create(bf_context** out, void* hip_stream) {
  if (!out) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  bf_context* c = new (std::nothrow) bf_context();
  if (!c) return BF_ERR_OUT_OF_MEMORY;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return BF_ERR_DEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    delete c;
    return BF_ERR_DEVICE;
  }
  c->num_cus = cus;
  c->noalloc = new (std::nothrow) bf_context();
  if (!c->noalloc) {
    delete c;
    return BF_ERR_OUT_OF_MEMORY;
  }
  lookup_scratch(c->device);
  ++g_live_contexts;
  *out = c;
  return BF_OK;
}

// Every device buffer a context owns (grown on demand, freed by bf_destroy).
static std::vector<Buf*> context_buffers(bf_context* c) {
  return {&c->nd, &c->grad, &c->kx, &c->ky, &c->kx64, &c->ky64, &c->pair_flags, &c->row_count, &c->row_off, &c->pairs,
          &c->pair_keys, &c->corr_key, &c->corr_idx, &c->corr_key_sorted, &c->corr_perm, &c->corr_head,
          &c->corr_group, &c->sparse_ij, &c->sparse_keys, &c->sparse_ptr, &c->moments, &c->in_b,
          &c->common_scan, &c->edge_ij, &c->edge_keys, &c->edge_dense, &c->edge_sparse, &c->ej_key,
          &c->ej_idx, &c->ej_key_sorted, &c->ej_sorted, &c->iptr, &c->jptr, &c->free_flag, &c->var_of,
          &c->frame_of_var, &c->records, &c->eblocks, &c->hij32, &c->hij64, &c->diag32, &c->diag64,
          &c->minv32, &c->minv64, &c->rhs, &c->poses_work, &c->pcg_vec, &c->stats, &c->trace,
          &c->cub_tmp, &c->counts, &c->flags, &c->energy,
          &c->pcg_partials, &c->pcg_barrier, &c->pcg_tags, &c->seg_start, &c->seg_of,
          &c->seg_var_ptr, &c->seg_edge_ptr, &c->sys_poses, &c->mf_u, &c->pr_active, &c->pr_cnt0,
          &c->pr_cnt, &c->pr_valid, &c->pr_flag, &c->pr_pos, &c->pr_fi, &c->pr_fj, &c->pr_pi, &c->pr_pj,
          &c->pr_pflag, &c->pr_ppos, &c->pr_pairs, &c->pr_pairs_all, &c->pr_bval, &c->pr_bidx,
          &c->pr_poses, &c->row_cnt, &c->row_ptr, &c->row_entries, &c->mf_pts, &c->mf_y,
          &c->ediag_dense, &c->dist_slots, &c->energy_parts};
}

void bf_destroy(bf_context* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  const std::vector<Buf*> bufs = context_buffers(c);
  for (Buf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (c->rb_small) (void)hipHostFree(c->rb_small);
  if (c->rb_big) (void)hipHostFree(c->rb_big);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->gn_exec) (void)hipGraphExecDestroy(c->gn_exec);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  delete c->noalloc;  // its buffers lie in the static scratch array: nothing to free
  delete c;
  --g_live_contexts;
}

bf_status bf_pcg_threads(const bf_context* ctx, int32_t* out_threads) {
  if (!ctx || !out_threads) return BF_ERR_INVALID_ARG;
  *out_threads = ctx->pcg_threads_last;
  return BF_OK;
}

bf_status bf_workspace_bytes(const bf_context* ctx, int64_t* out_bytes) {
  if (!ctx || !out_bytes) return BF_ERR_INVALID_ARG;
  int64_t total = 0;
  for (const Buf* b : context_buffers(const_cast<bf_context*>(ctx))) total += (int64_t)b->cap;
  *out_bytes = total;
  return BF_OK;
}

const char* bf_status_string(bf_status s) {
  switch (s) {
    case BF_OK: return "ok";
    case BF_ERR_INVALID_ARG: return "invalid argument";
    case BF_ERR_OUT_OF_MEMORY: return "out of memory";
    case BF_ERR_DEVICE: return "device error";
    case BF_ERR_NOT_PD: return "matrix not positive definite";
    case BF_ERR_NONFINITE: return "non-finite input";
    case BF_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* bf_last_error(const bf_context* c) { return c ? c->last_error.c_str() : "null context"; }

bf_status bf_prepare_frames(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_params* prm,
                            float* out_nd, float* out_grad) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    Context& c = *ctx;
    size_t HW = (size_t)in->width * in->height;
    ensure(c.nd, sizeof(float4) * HW * fr->num_frames);
    ensure(c.grad, sizeof(float) * HW * fr->num_frames);
    ensure(c.kx, sizeof(float) * in->width);
    ensure(c.ky, sizeof(float) * in->height);
    ensure(c.kx64, sizeof(double) * in->width);
    ensure(c.ky64, sizeof(double) * in->height);
    launch_prepare(c, *fr, *in, *prm);
    if (out_nd)
      check_hip(hipMemcpyAsync(out_nd, c.nd.p, sizeof(float4) * HW * fr->num_frames, hipMemcpyDeviceToDevice,
                               c.stream), "copy normals");
    if (out_grad)
      check_hip(hipMemcpyAsync(out_grad, c.grad.p, sizeof(float) * HW * fr->num_frames, hipMemcpyDeviceToDevice,
                               c.stream), "copy gradients");
  });
}

bf_status bf_build_pairs(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const double* poses,
                         const bf_params* prm, int32_t* out_ij, int64_t capacity, int64_t* out_count) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(nullptr, nullptr, poses);
    if (!out_count) fail(BF_ERR_INVALID_ARG, "null out_count");
    Context& c = *ctx;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, poses, fr->num_frames);
    set_segments(c, fr->num_frames, nullptr, 1);
    int64_t P = launch_pair_search(c, *fr, *in, poses, *prm);
    int hf = 0;
    sync_and_flags(c, &hf);
    raise_flags(hf);
    *out_count = P;
    if (P > capacity) fail(BF_ERR_INVALID_ARG, "pair capacity too small");
    if (P > 0) {
      if (!out_ij) fail(BF_ERR_INVALID_ARG, "null out_ij");
      check_hip(hipMemcpyAsync(out_ij, c.pairs.p, sizeof(int) * 2 * P, hipMemcpyDeviceToDevice, c.stream), "copy");
      check_hip(hipStreamSynchronize(c.stream), "synchronise");
    }
  });
}

bf_status bf_build_structure(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                             const bf_pairs* pairs, const double* poses, const bf_params* prm, bf_structure* out) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, poses);
    if (!out) fail(BF_ERR_INVALID_ARG, "null out");
    Context& c = *ctx;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, poses, fr->num_frames);
    setup(ctx, fr, in, co, pairs, poses, prm);
    const Shape& s = c.shape;
    out->num_pairs = s.P;
    out->num_sparse_pairs = s.S;
    out->num_edges = s.E;
    out->num_free = s.nfree;
    auto cp = [&](void* dst, const Buf& src, size_t bytes) {
      if (dst && bytes) check_hip(hipMemcpyAsync(dst, src.p, bytes, hipMemcpyDeviceToDevice, c.stream), "copy");
    };
    cp(out->pairs_ij, c.pairs, sizeof(int) * 2 * s.P);
    cp(out->sparse_ij, c.sparse_ij, sizeof(int) * 2 * s.S);
    if (s.S > 0) cp(out->sparse_ptr, c.sparse_ptr, sizeof(long long) * (s.S + 1));
    cp(out->corr_perm, c.corr_perm, sizeof(long long) * s.M);
    cp(out->edges_ij, c.edge_ij, sizeof(int) * 2 * s.E);
    cp(out->free_frames, c.frame_of_var, sizeof(int) * s.nfree);
    check_hip(hipStreamSynchronize(c.stream), "synchronise");
  });
}

bf_status bf_eval_residuals(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                            const bf_pairs* pairs, const double* poses, const bf_params* prm, int32_t gn_iter,
                            double* out_energy, int64_t* out_counts, double* out_records, uint32_t* out_assoc) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, poses);
    if (!out_energy) fail(BF_ERR_INVALID_ARG, "null out_energy");
    Context& c = *ctx;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, poses, fr->num_frames);
    setup(ctx, fr, in, co, pairs, poses, prm);
    double wd = dense_weight(*prm, gn_iter);
    bool jac = out_records != nullptr;
    launch_dense(c, *in, poses, *prm, wd, jac, out_assoc);
    launch_edge_blocks(c, poses, *prm, false);
    launch_energy(c, c.energy.as<double>());
    if (out_records && c.shape.P > 0) export_records(c, out_records);
    double e8[8];
    int hf = 0;
    check_hip(hipMemcpyAsync(e8, c.energy.p, sizeof(e8), hipMemcpyDeviceToHost, c.stream), "copy energy");
    sync_and_flags(c, &hf);
    raise_flags(hf);
    for (int k = 0; k < 4; ++k) out_energy[k] = e8[k];
    if (out_counts)
      for (int k = 0; k < 3; ++k) out_counts[k] = (int64_t)llround(e8[4 + k]);
  });
}

bf_status bf_system_create(bf_context* ctx, bf_system** out) {
  if (!ctx || !out) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  bf_system* y = new (std::nothrow) bf_system();
  if (!y) return BF_ERR_OUT_OF_MEMORY;
  y->owner = ctx;
  y->stream = ctx->stream;
  *out = y;
  return BF_OK;
}

void bf_system_destroy(bf_system* y) {
  if (!y) return;
  (void)hipStreamSynchronize(y->stream);
  Buf* bufs[] = {&y->eblocks, &y->hij32, &y->hij64, &y->edge_ij, &y->iptr, &y->jptr, &y->ej_sorted, &y->row_ptr,
                 &y->row_entries, &y->frame_of_var, &y->var_of, &y->seg_var_ptr, &y->seg_edge_ptr, &y->seg_start,
                 &y->seg_of, &y->sys_poses, &y->corr_perm, &y->corr_group, &y->sparse_ij, &y->sparse_ptr,
                 &y->edge_sparse};
  for (Buf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  delete y;
}

bf_status bf_build_normal_equations(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in,
                                    const bf_corrs* co, const bf_pairs* pairs, const double* poses,
                                    const bf_params* prm, int32_t gn_iter, bf_system* sys,
                                    double* out_edge_blocks, double* out_energy) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, poses);
    if (!sys) fail(BF_ERR_INVALID_ARG, "null system");
    if (sys->owner != ctx) fail(BF_ERR_INVALID_ARG, "the system belongs to another context");
    if (prm->sparse_matrix_free) fail(BF_ERR_UNSUPPORTED, "a system holds assembled blocks (sparse_matrix_free = 0)");
    Context& c = *ctx;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, poses, fr->num_frames);
    setup(ctx, fr, in, co, pairs, poses, prm);
    double wd = dense_weight(*prm, gn_iter);
    launch_dense(c, *in, poses, *prm, wd, true);
    launch_edge_blocks(c, poses, *prm, true);
    launch_energy(c, c.energy.as<double>());
    ensure(c.sys_poses, sizeof(double) * 16 * fr->num_frames);
    check_hip(hipMemcpyAsync(c.sys_poses.p, poses, sizeof(double) * 16 * fr->num_frames, hipMemcpyDeviceToDevice,
                             c.stream), "copy poses");
    c.sys_w_sparse = prm->use_sparse ? prm->w_sparse : 0.0;
    if (out_edge_blocks && c.shape.E > 0)
      check_hip(hipMemcpyAsync(out_edge_blocks, c.eblocks.p, sizeof(double) * kEdgeWords * c.shape.E,
                               hipMemcpyDeviceToDevice, c.stream), "copy edge blocks");
    double e8[8];
    int hf = 0;
    check_hip(hipMemcpyAsync(e8, c.energy.p, sizeof(e8), hipMemcpyDeviceToHost, c.stream), "copy energy");
    sync_and_flags(c, &hf);
    raise_flags(hf & ~kFlagNotPD);
    // the system takes the assembled blocks and the structure the PCG reads; the
    // context keeps the system's previous buffers for reuse
    sys->built = false;
    swap_system(c, *sys);
    sys->built = true;
    if (out_energy)
      for (int k = 0; k < 4; ++k) out_energy[k] = e8[k];
  });
}

bf_status bf_system_export(bf_context* ctx, const bf_system* sys, double* out_H, double* out_g,
                           int64_t* out_num_free) {
  return guarded(ctx, [&] {
    if (!ctx) fail(BF_ERR_INVALID_ARG, "null context");
    check_system(ctx, sys);
    Context& c = *ctx;
    SystemLoan loan(c, sys);
    if (out_H || out_g) launch_export_dense(c, out_H, out_g);
    if (out_num_free) *out_num_free = c.shape.nfree;
    check_hip(hipStreamSynchronize(c.stream), "synchronise");
  });
}

bf_status bf_pcg_solve(bf_context* ctx, const bf_system* sys, int32_t num_iters, double* out_delta,
                       double* out_stats) {
  return guarded(ctx, [&] {
    if (!ctx) fail(BF_ERR_INVALID_ARG, "null context");
    check_system(ctx, sys);
    if (num_iters < 0) fail(BF_ERR_INVALID_ARG, "negative iteration count");
    if (!out_delta) fail(BF_ERR_INVALID_ARG, "null out_delta");
    Context& c = *ctx;
    SystemLoan loan(c, sys);
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    if (c.shape.nfree == 0) {
      check_hip(hipMemsetAsync(out_delta, 0, sizeof(double) * 6 * c.shape.F, c.stream), "memset");
    } else {
      launch_solve(c, num_iters, nullptr, out_delta, nullptr, c.stats.as<double>(), false);
    }
    double st[4] = {0, 0, 0, 0};
    int hf = 0;
    if (c.shape.nfree > 0)
      check_hip(hipMemcpyAsync(st, c.stats.p, sizeof(double) * 3, hipMemcpyDeviceToHost, c.stream), "copy stats");
    sync_and_flags(c, &hf);
    raise_flags(hf);
    if (out_stats)
      for (int k = 0; k < 3; ++k) out_stats[k] = st[k];
  });
}

}  // extern "C"

namespace bf {
namespace {

// Every launch of the Gauss-Newton loop over the structure built by setup(), in
// order on c.stream: the initial poses into the work buffer, num_gn iterations of
// (dense pair jobs, edge blocks, PCG + SE(3) update, or the energy alone when no
// frame is free), then the energy at the final poses and the poses out (kept only
// when no error flag is raised).  tm may be null: no timing events.
void enqueue_loop(Context& c, const bf_intrinsics* in, const bf_params* prm, const double* init_poses,
                  double* out_poses, Timer* tm) {
  const int F = c.shape.F;
  const int nseg = c.shape.nseg;
  double* poses = c.poses_work.as<double>();
  auto mark = [&] { return tm ? tm->mark() : -1; };
  auto mark_phase = [&] { return tm ? tm->mark_phase() : -1; };
  hipLaunchKernelGGL(k_copy_d, dim3((16 * F + 255) / 256), dim3(256), 0, c.stream, init_poses, poses, 16 * F);
  for (int k = 0; k < prm->num_gn; ++k) {
    double wd = dense_weight(*prm, k);
    double* slot = c.trace.as<double>() + 8 * (size_t)nseg * k;
    int a = mark();
    launch_dense(c, *in, poses, *prm, wd, true);
    int b = mark();
    launch_edge_blocks(c, poses, *prm, true);
    int d = mark_phase();
    if (c.shape.nfree > 0) launch_solve(c, prm->num_pcg, slot, nullptr, poses, nullptr, true, prm->sparse_matrix_free);
    else launch_energy(c, slot);
    int f = mark_phase();
    if (tm) {
      tm->span(1, a, b);
      tm->span(2, b, d);
      tm->span(4, d, f);
    }
  }
  int g0 = mark_phase();
  double wd = dense_weight(*prm, prm->num_gn > 0 ? prm->num_gn - 1 : 0);
  launch_dense(c, *in, poses, *prm, wd, false);
  launch_edge_blocks(c, poses, *prm, false);
  launch_energy(c, c.energy.as<double>());
  hipLaunchKernelGGL(k_copy_if_ok, dim3((16 * F + 255) / 256), dim3(256), 0, c.stream, poses, out_poses, 16 * F,
                     c.flags.as<int>());
  int g1 = mark_phase();
  if (tm) tm->span(5, g0, g1);
}

// What a captured loop depends on beyond the contents of device memory: the
// parameters and intrinsics, the structure's sizes (grids, shared memory), the
// dense workgroup sizes, the caller's pose buffers and the workspace addresses
// (through the allocation count).
std::vector<unsigned char> graph_key(const Context& c, const bf_intrinsics* in, const bf_params* prm,
                                     const double* init_poses, const double* out_poses, int nt_jac, int nt_eval) {
  std::vector<unsigned char> k;
  auto add = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    k.insert(k.end(), b, b + n);
  };
  bf_params q = *prm;
  q.timing = 0;
  add(&q, sizeof q);
  add(in, sizeof *in);
  const Shape& s = c.shape;
  const int64_t sizes[] = {s.F, s.W, s.H, s.M, s.P, s.S, s.E, s.nfree, s.nseg, s.max_seg_free};
  add(sizes, sizeof sizes);
  const unsigned long long gen = alloc_generation();
  add(&gen, sizeof gen);
  add(&init_poses, sizeof init_poses);
  add(&out_poses, sizeof out_poses);
  const int other[] = {nt_jac, nt_eval, c.pcg_storage, c.precond, c.solve_mode, per_problem_pcg_threads(const_cast<Context&>(c), false)};
  add(other, sizeof other);
  return k;
}

// Run the loop as one graph launch on c.stream, capturing it first (on a private
// stream) when nothing is captured yet or the key has changed.
void launch_loop_graph(Context& c, const bf_intrinsics* in, const bf_params* prm, const double* init_poses,
                       double* out_poses) {
  if (c.shape.nfree > 0 && !solve_per_problem(c))
    fail(BF_ERR_UNSUPPORTED,
         "graph mode needs the per-problem PCG kernel (a batch, or a problem of at most 64 free frames)");
  // settle, eagerly, what capture must not do: dense workgroup-size timing and
  // kernel attribute settings
  const int nt_jac = prm->num_gn > 0 ? dense_threads_for(c, *in, init_poses, *prm, dense_weight(*prm, 0), true) : 0;
  const int nt_eval = dense_threads_for(c, *in, init_poses, *prm,
                                        dense_weight(*prm, prm->num_gn > 0 ? prm->num_gn - 1 : 0), false);
  prepare_solve(c);
  std::vector<unsigned char> key = graph_key(c, in, prm, init_poses, out_poses, nt_jac, nt_eval);
  if (!c.gn_exec || key != c.gn_key) {
    if (c.gn_exec) {
      check_hip(hipGraphExecDestroy(c.gn_exec), "destroy graph");
      c.gn_exec = nullptr;
      c.gn_key.clear();
    }
    if (!c.capture_stream)
      check_hip(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking), "create capture stream");
    hipStream_t user = c.stream;
    c.stream = c.capture_stream;
    hipGraph_t g = nullptr;
    check_hip(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal), "begin capture");
    c.in_capture = true;
    try {
      enqueue_loop(c, in, prm, init_poses, out_poses, nullptr);
    } catch (...) {
      (void)hipStreamEndCapture(c.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      c.stream = user;
      c.in_capture = false;
      throw;
    }
    c.in_capture = false;
    hipError_t e = hipStreamEndCapture(c.stream, &g);
    c.stream = user;
    check_hip(e, "end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check_hip(e, "instantiate graph");
    c.gn_exec = x;
    c.gn_key = std::move(key);
    ++c.gn_captures;
  }
  check_hip(hipGraphLaunch(c.gn_exec, c.stream), "graph launch");
}

// The Gauss-Newton loop, eager or as a graph (params.graph), then the single copy
// of energies (and trace) to the host: energies [nseg][4], trace (host, may be
// NULL) [nseg][num_gn][4].
void run_gauss_newton(bf_context* ctx, const bf_intrinsics* in, const bf_params* prm, const double* init_poses,
                      double* out_poses, double* out_energy, double* out_trace, Timer& tm, int t_start,
                      bool allow_graph = true) {
  Context& c = *ctx;
  const int F = c.shape.F;
  const int nseg = c.shape.nseg;
  ensure(c.poses_work, sizeof(double) * 16 * F);
  int t_setup = tm.mark_phase();
  tm.span(0, t_start, t_setup);
  if (allow_graph && prm->graph) launch_loop_graph(c, in, prm, init_poses, out_poses);
  else enqueue_loop(c, in, prm, init_poses, out_poses, &tm);
  int g1 = tm.mark();
  const size_t n_e8 = 8 * (size_t)nseg;
  const size_t n_tr = (out_trace && prm->num_gn > 0) ? 8 * (size_t)nseg * prm->num_gn : 0;
  double* e8 = static_cast<double*>(readback_big(c, sizeof(double) * (n_e8 + n_tr)));
  double* tr = e8 + n_e8;
  int hf = 0;
  check_hip(hipMemcpyAsync(e8, c.energy.p, sizeof(double) * n_e8, hipMemcpyDeviceToHost, c.stream), "copy energy");
  if (n_tr)
    check_hip(hipMemcpyAsync(tr, c.trace.p, sizeof(double) * n_tr, hipMemcpyDeviceToHost, c.stream), "copy trace");
  sync_and_flags(c, &hf);
  raise_flags(hf);
  for (int b = 0; b < nseg; ++b)
    for (int l = 0; l < 4; ++l) out_energy[4 * b + l] = e8[8 * b + l];
  if (out_trace)
    for (int b = 0; b < nseg; ++b)
      for (int k = 0; k < prm->num_gn; ++k)
        for (int l = 0; l < 4; ++l) out_trace[((size_t)b * prm->num_gn + k) * 4 + l] = tr[8 * ((size_t)nseg * k + b) + l];
  tm.finish(c.timings);
  if (tm.on) {
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, ctx->pool[t_start], ctx->pool[g1]), "hipEventElapsedTime");
    c.timings[6] = 1000.0 * ms;
  }
}

}  // namespace
}  // namespace bf

extern "C" {

bf_status bf_gauss_newton(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                          const bf_pairs* pairs, const double* init_poses, const bf_params* prm, double* out_poses,
                          double* out_energy, double* out_trace) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, init_poses);
    if (!out_poses || !out_energy) fail(BF_ERR_INVALID_ARG, "null out_poses or out_energy");
    Context& c = *ctx;
    Timer tm(ctx, prm->timing);
    int t_start = tm.mark();
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, init_poses, fr->num_frames);
    setup(ctx, fr, in, co, pairs, init_poses, prm);
    run_gauss_newton(ctx, in, prm, init_poses, out_poses, out_energy, out_trace, tm, t_start);
  });
}

bf_status bf_gauss_newton_noalloc(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                                  const bf_pairs* pairs, const double* init_poses, const bf_params* prm,
                                  double* out_poses, double* out_energy, double* out_trace) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, init_poses);
    if (!out_poses || !out_energy) fail(BF_ERR_INVALID_ARG, "null out_poses or out_energy");
    if (prm->timing || prm->graph)
      fail(BF_ERR_UNSUPPORTED, "the allocation-free entry point runs without timing events or graph capture");
    if (prm->dense_threads == 0)
      fail(BF_ERR_UNSUPPORTED, "the allocation-free entry point needs a fixed params->dense_threads");
    if (prm->pcg_threads < 0)
      fail(BF_ERR_UNSUPPORTED, "the allocation-free entry point needs params->pcg_threads fixed (not -1)");
    if (!ctx->noalloc) fail(BF_ERR_DEVICE, "context has no allocation-free state");
    char* base = static_cast<char*>(scratch_address(ctx->device));
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    // fresh state every call: every buffer is carved anew from the start of the
    // array, and everything that must start at zero (flags, counters, the PCG
    // exchange tags) is cleared on the way as in a newly created context
    bf_context& na = *ctx->noalloc;
    na = bf_context();
    na.stream = ctx->stream;
    na.device = ctx->device;
    na.num_cus = ctx->num_cus;
    Arena arena{base, kScratchBytes, 0};
    struct Scope {
      hipStream_t stream;
      explicit Scope(Arena* a, hipStream_t s) : stream(s) { t_arena = a; }
      // the array is free for the next call only once this call's work is done
      ~Scope() {
        (void)hipStreamSynchronize(stream);
        t_arena = nullptr;
      }
    } scope(&arena, na.stream);
    Timer tm(&na, false);
    ensure(na.flags, sizeof(int));
    check_hip(hipMemsetAsync(na.flags.p, 0, sizeof(int), na.stream), "memset flags");
    check_poses(na, init_poses, fr->num_frames);
    setup(&na, fr, in, co, pairs, init_poses, prm);
    run_gauss_newton(&na, in, prm, init_poses, out_poses, out_energy, out_trace, tm, -1, false);
  });
}

bf_status bf_gauss_newton_batch(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                                const bf_pairs* pairs, int32_t num_problems, const int32_t* frame_offsets,
                                const double* init_poses, const bf_params* prm, double* out_poses,
                                double* out_energy, double* out_trace) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, init_poses);
    if (num_problems < 1 || !frame_offsets) fail(BF_ERR_INVALID_ARG, "num_problems must be >= 1 with frame offsets");
    if (!out_poses || !out_energy) fail(BF_ERR_INVALID_ARG, "null out_poses or out_energy");
    if (prm->solve_kernel != 0 && prm->solve_kernel != 4)
      fail(BF_ERR_UNSUPPORTED, "a batch is solved by the per-problem kernel (solve_kernel 0 or 4)");
    if (prm->sparse_matrix_free) fail(BF_ERR_UNSUPPORTED, "a batch uses assembled sparse blocks (sparse_matrix_free = 0)");
    Context& c = *ctx;
    Timer tm(ctx, prm->timing);
    int t_start = tm.mark();
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, init_poses, fr->num_frames);
    setup(ctx, fr, in, co, pairs, init_poses, prm, frame_offsets, num_problems);
    run_gauss_newton(ctx, in, prm, init_poses, out_poses, out_energy, out_trace, tm, t_start);
  });
}

bf_status bf_filter_correspondences(bf_context* ctx, const bf_corrs* co, int32_t num_frames, double max_res,
                                   double max_cond, int32_t cond_mode, int32_t min_count, double min_area,
                                   uint8_t* out_keep, int64_t* out_kept) {
  return guarded(ctx, [&] {
    if (!ctx) fail(BF_ERR_INVALID_ARG, "null context");
    validate_corrs(co);
    if (!co) fail(BF_ERR_INVALID_ARG, "null correspondences");
    if (num_frames < 1 || num_frames > 16384) fail(BF_ERR_INVALID_ARG, "num_frames out of range");
    if (!(max_res >= 0.0) || !(max_cond >= 1.0) || min_count < 0 || !(min_area >= 0.0))
      fail(BF_ERR_INVALID_ARG, "bad filter thresholds");
    if (cond_mode != 0 && cond_mode != 1) fail(BF_ERR_INVALID_ARG, "cond_mode must be 0 or 1");
    if (co->count > 0 && !out_keep) fail(BF_ERR_INVALID_ARG, "null out_keep");
    Context& c = *ctx;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    const long long S = group_correspondences(c, *co, num_frames);
    launch_filters(c, *co, S, max_res, max_cond, min_count, min_area, cond_mode, out_keep);
    check_hip(hipStreamSynchronize(c.stream), "synchronise");
    if (out_kept) {
      long long kept = 0;
      if (co->count > 0) {
        std::vector<uint8_t> h((size_t)co->count);
        check_hip(hipMemcpy(h.data(), out_keep, (size_t)co->count, hipMemcpyDeviceToHost), "copy");
        for (uint8_t v : h) kept += v;
      }
      *out_kept = kept;
    }
  });
}

bf_status bf_verify_pairs(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_pairs* pairs,
                          const double* poses, const bf_params* prm, double tau_c, double max_err, double min_frac,
                          double* out_stats, uint8_t* out_valid) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(nullptr, pairs, poses);
    if (!pairs) fail(BF_ERR_INVALID_ARG, "null pairs");
    if (!(tau_c >= 0.0) || !(max_err >= 0.0) || !(min_frac >= 0.0)) fail(BF_ERR_INVALID_ARG, "bad thresholds");
    if (pairs->count > 0 && (!out_stats || !out_valid)) fail(BF_ERR_INVALID_ARG, "null outputs");
    Context& c = *ctx;
    const int F = fr->num_frames;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, poses, F);
    if (pairs->count > 0)
      hipLaunchKernelGGL(k_check_pair_range, dim3((unsigned)((pairs->count + 255) / 256)), dim3(256), 0, c.stream,
                         pairs->ij, (long long)pairs->count, F, c.flags.as<int>());
    int hf = 0;
    sync_and_flags(c, &hf);
    raise_flags(hf);
    size_t HW = (size_t)in->width * in->height;
    ensure(c.nd, sizeof(float4) * HW * F);
    ensure(c.grad, sizeof(float) * HW * F);
    ensure(c.kx, sizeof(float) * in->width);
    ensure(c.ky, sizeof(float) * in->height);
    ensure(c.kx64, sizeof(double) * in->width);
    ensure(c.ky64, sizeof(double) * in->height);
    launch_prepare(c, *fr, *in, *prm);
    launch_verify(c, *fr, *in, pairs->ij, pairs->count, poses, *prm, tau_c, max_err, min_frac, out_stats, out_valid);
    check_hip(hipStreamSynchronize(c.stream), "synchronise");
  });
}

bf_status bf_gauss_newton_pruned(bf_context* ctx, const bf_frames* fr, const bf_intrinsics* in, const bf_corrs* co,
                                 const bf_pairs* pairs, const double* init_poses, const bf_params* prm,
                                 double r_prune, int32_t max_rounds, double* out_poses, double* out_energy,
                                 uint8_t* out_corr_active, uint8_t* out_frame_valid, int32_t* out_rounds,
                                 double* out_rmax) {
  return guarded(ctx, [&] {
    validate_common(ctx, fr, in, prm);
    validate_problem(co, pairs, init_poses);
    if (!co) fail(BF_ERR_INVALID_ARG, "null correspondences");
    if (!out_poses || !out_energy) fail(BF_ERR_INVALID_ARG, "null out_poses or out_energy");
    if (!(r_prune >= 0.0) || max_rounds < 0) fail(BF_ERR_INVALID_ARG, "bad pruning threshold or round limit");
    if (prm->sparse_matrix_free) fail(BF_ERR_UNSUPPORTED, "pruning uses assembled sparse blocks (sparse_matrix_free = 0)");
    Context& c = *ctx;
    const int F = fr->num_frames;
    ensure(c.flags, sizeof(int));
    check_hip(hipMemsetAsync(c.flags.p, 0, sizeof(int), c.stream), "memset flags");
    check_poses(c, init_poses, F);
    prune_init(c, *co, F);
    ensure(c.pr_poses, sizeof(double) * 16 * F);
    check_hip(hipMemcpyAsync(c.pr_poses.p, init_poses, sizeof(double) * 16 * F, hipMemcpyDeviceToDevice, c.stream),
              "copy poses");
    // the dense pair set is fixed by the first round (given, or found at init_poses)
    long long P = 0;
    if (prm->use_dense) {
      if (pairs) {
        P = pairs->count;
        ensure(c.pr_pairs_all, sizeof(int) * 2 * (P + 1));
        if (P > 0)
          check_hip(hipMemcpyAsync(c.pr_pairs_all.p, pairs->ij, sizeof(int) * 2 * P, hipMemcpyDeviceToDevice,
                                   c.stream), "copy pairs");
      } else {
        set_segments(c, F, nullptr, 1);
        P = launch_pair_search(c, *fr, *in, init_poses, *prm);
        ensure(c.pr_pairs_all, sizeof(int) * 2 * (P + 1));
        if (P > 0)
          check_hip(hipMemcpyAsync(c.pr_pairs_all.p, c.pairs.p, sizeof(int) * 2 * P, hipMemcpyDeviceToDevice,
                                   c.stream), "copy pairs");
      }
    }
    int rounds = 0;
    double e4[4] = {0, 0, 0, 0};
    double rmax = -1.0;
    for (;;) {
      bf_corrs cc = prune_active_corrs(c, *co);
      bf_pairs pp = prune_valid_pairs(c, c.pr_pairs_all.as<int>(), P);
      Timer tm(ctx, false);
      setup(ctx, fr, in, &cc, &pp, c.pr_poses.as<double>(), prm);
      run_gauss_newton(ctx, in, prm, c.pr_poses.as<double>(), c.pr_poses.as<double>(), e4, nullptr, tm, -1,
                       false);
      long long idx = -1;
      rmax = prune_max_residual(c, *co, c.pr_poses.as<double>(), &idx);
      if (idx < 0 || rmax <= r_prune || rounds >= max_rounds) break;
      int ab[2];
      check_hip(hipMemcpyAsync(&ab[0], co->frame_i + idx, sizeof(int), hipMemcpyDeviceToHost, c.stream), "copy");
      check_hip(hipMemcpyAsync(&ab[1], co->frame_j + idx, sizeof(int), hipMemcpyDeviceToHost, c.stream), "copy");
      check_hip(hipStreamSynchronize(c.stream), "synchronise");
      prune_drop(c, *co, F, ab[0], ab[1]);
      ++rounds;
    }
    check_hip(hipMemcpyAsync(out_poses, c.pr_poses.p, sizeof(double) * 16 * F, hipMemcpyDeviceToDevice, c.stream),
              "copy poses");
    if (out_corr_active && co->count > 0)
      check_hip(hipMemcpyAsync(out_corr_active, c.pr_active.p, co->count, hipMemcpyDeviceToDevice, c.stream), "copy");
    if (out_frame_valid)
      check_hip(hipMemcpyAsync(out_frame_valid, c.pr_valid.p, F, hipMemcpyDeviceToDevice, c.stream), "copy");
    check_hip(hipStreamSynchronize(c.stream), "synchronise");
    for (int k = 0; k < 4; ++k) out_energy[k] = e4[k];
    if (out_rounds) *out_rounds = rounds;
    if (out_rmax) *out_rmax = rmax;
  });
}

bf_status bf_system_matvec(bf_context* ctx, const bf_system* sys, const bf_corrs* co, const double* x, double* y,
                           int32_t mode, double* out_us) {
  return guarded(ctx, [&] {
    if (!ctx) fail(BF_ERR_INVALID_ARG, "null context");
    check_system(ctx, sys);
    if (!x || !y) fail(BF_ERR_INVALID_ARG, "null x or y");
    if (mode != 0 && mode != 1) fail(BF_ERR_INVALID_ARG, "mode must be 0 or 1");
    if (mode == 1 && (!co || co->count != sys->shape.M))
      fail(BF_ERR_INVALID_ARG, "mode 1 needs the correspondences the system was built from");
    Context& c = *ctx;
    SystemLoan loan(c, sys);
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    check_hip(hipEventRecord(e0, c.stream), "hipEventRecord");
    launch_matvec(c, co, c.sys_w_sparse, mode, x, y);
    check_hip(hipEventRecord(e1, c.stream), "hipEventRecord");
    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (out_us) *out_us = 1000.0 * ms;
  });
}

int64_t bf_graph_captures(const bf_context* ctx) { return ctx ? ctx->gn_captures : -1; }

bf_status bf_last_timings(const bf_context* ctx, double* out_us) {
  if (!ctx || !out_us) return BF_ERR_INVALID_ARG;
  for (int k = 0; k < 8; ++k) out_us[k] = ctx->timings[k];
  return BF_OK;
}

bf_status bf_dense_shape(const bf_context* ctx, int32_t* out_shape) {
  if (!ctx || !out_shape) return BF_ERR_INVALID_ARG;
  for (int k = 0; k < 4; ++k) out_shape[k] = ctx->dense_shape_last[k];
  return BF_OK;
}

}  // extern "C"
