// Residual pruning after a solve (paper Sec. 4.4.1, last paragraph): the largest
// sparse residual over the active correspondences is found by a parallel
// reduction (one candidate per workgroup; the final maximum is taken on the host,
// as in the paper); if it exceeds the threshold, every correspondence between the
// two frames of the offending correspondence is deactivated, and a frame left
// without any correspondence is removed from the problem.
//
// The residual of a correspondence between frames i and j (p in camera i, q in
// camera j) is |T_i p - T_j q| in metres, in FP64.  Ties resolve to the smallest
// correspondence index.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace bf {

namespace {

template <class Fn>
void cub_call(Context& c, Fn fn) {
  size_t bytes = 0;
  check_hip(fn(nullptr, bytes), "hipcub size query");
  ensure(c.cub_tmp, bytes + 256);
  check_hip(fn(c.cub_tmp.p, bytes), "hipcub call");
}

// Per workgroup of 256: the largest residual among its correspondences and its
// index (-1 when none is active).
__global__ void __launch_bounds__(256) k_resid_max(const int* __restrict__ fi, const int* __restrict__ fj,
                                                   const float* __restrict__ pi, const float* __restrict__ pj,
                                                   const uint8_t* __restrict__ active, long long M,
                                                   const double* __restrict__ poses, double* __restrict__ blk_val,
                                                   long long* __restrict__ blk_idx) {
  __shared__ double sv[256];
  __shared__ long long si[256];
  const int tid = threadIdx.x;
  const long long c = (long long)blockIdx.x * 256 + tid;
  double best = -1.0;
  long long bi = -1;
  if (c < M && active[c]) {
    const double* Ti = poses + (size_t)fi[c] * 16;
    const double* Tj = poses + (size_t)fj[c] * 16;
    double s = 0.0;
    for (int r = 0; r < 3; ++r) {
      const double a = Ti[4 * r] * pi[3 * c] + Ti[4 * r + 1] * pi[3 * c + 1] + Ti[4 * r + 2] * pi[3 * c + 2] + Ti[4 * r + 3];
      const double b = Tj[4 * r] * pj[3 * c] + Tj[4 * r + 1] * pj[3 * c + 1] + Tj[4 * r + 2] * pj[3 * c + 2] + Tj[4 * r + 3];
      s += (a - b) * (a - b);
    }
    best = sqrt(s);
    bi = c;
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      const double v = sv[tid + o];
      const long long k = si[tid + o];
      if (v > sv[tid] || (v == sv[tid] && k >= 0 && (si[tid] < 0 || k < si[tid]))) {
        sv[tid] = v;
        si[tid] = k;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    blk_val[blockIdx.x] = sv[0];
    blk_idx[blockIdx.x] = si[0];
  }
}

// Deactivate every correspondence between frames a and b (either order).
__global__ void k_drop_pair(const int* __restrict__ fi, const int* __restrict__ fj, long long M, int a, int b,
                            uint8_t* __restrict__ active) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  const int x = fi[c], y = fj[c];
  if ((x == a && y == b) || (x == b && y == a)) active[c] = 0;
}

// Active correspondences per frame (integer counts; the order of the atomic adds
// does not change the result).
__global__ void k_frame_counts(const int* __restrict__ fi, const int* __restrict__ fj,
                               const uint8_t* __restrict__ active, long long M, int* __restrict__ cnt) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M || !active[c]) return;
  atomicAdd(&cnt[fi[c]], 1);
  atomicAdd(&cnt[fj[c]], 1);
}

// A frame that had correspondences and has none left is invalid.
__global__ void k_frame_valid(const int* __restrict__ cnt0, const int* __restrict__ cnt, int F,
                              uint8_t* __restrict__ valid) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < F) valid[f] = (cnt0[f] > 0 && cnt[f] == 0) ? 0 : 1;
}

__global__ void k_flags_u8_to_ll(const uint8_t* __restrict__ a, long long n, long long* __restrict__ o) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) o[k] = a[k];
}

__global__ void k_pair_flags(const int* __restrict__ ij, long long P, const uint8_t* __restrict__ valid,
                             long long* __restrict__ o) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < P) o[k] = (valid[ij[2 * k]] && valid[ij[2 * k + 1]]) ? 1 : 0;
}

__global__ void k_scatter_corrs(const int* __restrict__ fi, const int* __restrict__ fj, const float* __restrict__ pi,
                                const float* __restrict__ pj, const long long* __restrict__ flag,
                                const long long* __restrict__ pos, long long M, int* __restrict__ ofi,
                                int* __restrict__ ofj, float* __restrict__ opi, float* __restrict__ opj) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M || !flag[c]) return;
  const long long d = pos[c];
  ofi[d] = fi[c];
  ofj[d] = fj[c];
  for (int k = 0; k < 3; ++k) {
    opi[3 * d + k] = pi[3 * c + k];
    opj[3 * d + k] = pj[3 * c + k];
  }
}

__global__ void k_scatter_pairs(const int* __restrict__ ij, const long long* __restrict__ flag,
                                const long long* __restrict__ pos, long long P, int* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P || !flag[k]) return;
  out[2 * pos[k]] = ij[2 * k];
  out[2 * pos[k] + 1] = ij[2 * k + 1];
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

long long exclusive_count(Context& c, long long* flag, long long* pos, long long n) {
  cub_call(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::ExclusiveSum(t, b, flag, pos, (int)(n + 1), c.stream); });
  long long cnt = 0;
  check_hip(hipMemcpyAsync(&cnt, pos + n, sizeof(long long), hipMemcpyDeviceToHost, c.stream), "copy count");
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  return cnt;
}

}  // namespace

void prune_init(Context& c, const bf_corrs& co, int F) {
  const long long M = co.count;
  ensure(c.pr_active, M + 1);
  ensure(c.pr_cnt0, sizeof(int) * F);
  ensure(c.pr_cnt, sizeof(int) * F);
  ensure(c.pr_valid, F);
  check_hip(hipMemsetAsync(c.pr_active.p, 1, M + 1, c.stream), "memset");
  check_hip(hipMemsetAsync(c.pr_cnt0.p, 0, sizeof(int) * F, c.stream), "memset");
  if (M > 0)
    hipLaunchKernelGGL(k_frame_counts, dim3(blocks_for(M)), dim3(256), 0, c.stream, co.frame_i, co.frame_j,
                       c.pr_active.as<uint8_t>(), M, c.pr_cnt0.as<int>());
  hipLaunchKernelGGL(k_frame_valid, dim3(blocks_for(F)), dim3(256), 0, c.stream, c.pr_cnt0.as<int>(),
                     c.pr_cnt0.as<int>(), F, c.pr_valid.as<uint8_t>());
}

bf_corrs prune_active_corrs(Context& c, const bf_corrs& co) {
  const long long M = co.count;
  ensure(c.pr_flag, sizeof(long long) * (M + 1));
  ensure(c.pr_pos, sizeof(long long) * (M + 1));
  long long* flag = c.pr_flag.as<long long>();
  check_hip(hipMemsetAsync(flag + M, 0, sizeof(long long), c.stream), "memset");
  if (M > 0)
    hipLaunchKernelGGL(k_flags_u8_to_ll, dim3(blocks_for(M)), dim3(256), 0, c.stream, c.pr_active.as<uint8_t>(), M,
                       flag);
  const long long n = exclusive_count(c, flag, c.pr_pos.as<long long>(), M);
  ensure(c.pr_fi, sizeof(int) * (n + 1));
  ensure(c.pr_fj, sizeof(int) * (n + 1));
  ensure(c.pr_pi, sizeof(float) * 3 * (n + 1));
  ensure(c.pr_pj, sizeof(float) * 3 * (n + 1));
  if (M > 0)
    hipLaunchKernelGGL(k_scatter_corrs, dim3(blocks_for(M)), dim3(256), 0, c.stream, co.frame_i, co.frame_j, co.p_i,
                       co.p_j, flag, c.pr_pos.as<long long>(), M, c.pr_fi.as<int>(), c.pr_fj.as<int>(),
                       c.pr_pi.as<float>(), c.pr_pj.as<float>());
  return bf_corrs{n, c.pr_fi.as<int>(), c.pr_fj.as<int>(), c.pr_pi.as<float>(), c.pr_pj.as<float>()};
}

bf_pairs prune_valid_pairs(Context& c, const int* ij, long long P) {
  ensure(c.pr_pflag, sizeof(long long) * (P + 1));
  ensure(c.pr_ppos, sizeof(long long) * (P + 1));
  long long* flag = c.pr_pflag.as<long long>();
  check_hip(hipMemsetAsync(flag + P, 0, sizeof(long long), c.stream), "memset");
  if (P > 0)
    hipLaunchKernelGGL(k_pair_flags, dim3(blocks_for(P)), dim3(256), 0, c.stream, ij, P, c.pr_valid.as<uint8_t>(),
                       flag);
  const long long n = exclusive_count(c, flag, c.pr_ppos.as<long long>(), P);
  ensure(c.pr_pairs, sizeof(int) * 2 * (n + 1));
  if (P > 0)
    hipLaunchKernelGGL(k_scatter_pairs, dim3(blocks_for(P)), dim3(256), 0, c.stream, ij, flag,
                       c.pr_ppos.as<long long>(), P, c.pr_pairs.as<int>());
  return bf_pairs{n, c.pr_pairs.as<int>()};
}

double prune_max_residual(Context& c, const bf_corrs& co, const double* poses, long long* idx) {
  const long long M = co.count;
  *idx = -1;
  if (M == 0) return -1.0;
  const unsigned G = blocks_for(M);
  ensure(c.pr_bval, sizeof(double) * G);
  ensure(c.pr_bidx, sizeof(long long) * G);
  hipLaunchKernelGGL(k_resid_max, dim3(G), dim3(256), 0, c.stream, co.frame_i, co.frame_j, co.p_i, co.p_j,
                     c.pr_active.as<uint8_t>(), M, poses, c.pr_bval.as<double>(), c.pr_bidx.as<long long>());
  std::vector<double> v(G);
  std::vector<long long> k(G);
  check_hip(hipMemcpyAsync(v.data(), c.pr_bval.p, sizeof(double) * G, hipMemcpyDeviceToHost, c.stream), "copy");
  check_hip(hipMemcpyAsync(k.data(), c.pr_bidx.p, sizeof(long long) * G, hipMemcpyDeviceToHost, c.stream), "copy");
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  double best = -1.0;
  for (unsigned g = 0; g < G; ++g)  // blocks are in index order: the first maximum keeps the smallest index
    if (k[g] >= 0 && v[g] > best) {
      best = v[g];
      *idx = k[g];
    }
  return best;
}

void prune_drop(Context& c, const bf_corrs& co, int F, int a, int b) {
  const long long M = co.count;
  hipLaunchKernelGGL(k_drop_pair, dim3(blocks_for(M)), dim3(256), 0, c.stream, co.frame_i, co.frame_j, M, a, b,
                     c.pr_active.as<uint8_t>());
  check_hip(hipMemsetAsync(c.pr_cnt.p, 0, sizeof(int) * F, c.stream), "memset");
  hipLaunchKernelGGL(k_frame_counts, dim3(blocks_for(M)), dim3(256), 0, c.stream, co.frame_i, co.frame_j,
                     c.pr_active.as<uint8_t>(), M, c.pr_cnt.as<int>());
  hipLaunchKernelGGL(k_frame_valid, dim3(blocks_for(F)), dim3(256), 0, c.stream, c.pr_cnt0.as<int>(),
                     c.pr_cnt.as<int>(), F, c.pr_valid.as<uint8_t>());
}

}  // namespace bf
