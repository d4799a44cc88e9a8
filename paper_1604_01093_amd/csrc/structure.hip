// Per-solve structure of the energy.
//
// * Dense pair set E (paper Sec. 4.3: viewing directions within 60 degrees and
//   non-zero overlap).  Overlap is tested on a fixed 8x6 pixel grid of the lower
//   frame: at least one grid pixel with valid depth must land in front of the
//   other camera and inside its image.  FP64, fixed operation order, no
//   contraction, so the set is reproducible bit for bit.
// * Sparse correspondences (Sec. 4.3, E_sparse) grouped by unordered frame pair
//   with a stable radix sort, and reduced once per solve to FP64 moments
//   (count, sums of p and q, and of p p^T, q q^T, p q^T).  The sparse residual
//   is affine in p and q, so its J^T J blocks, J^T r and energy at any poses are
//   functions of these moments (evaluated per edge in solve.hip).
// * Edges: the sorted union of dense pairs and sparse pairs; per-frame incidence
//   (edges where the frame is the lower index are contiguous; the others come
//   from a stable sort by the upper index); free frames (not the first frame of
//   their problem, at least one edge) numbered in frame order.
// * Several independent problems can share one structure: problem b owns the
//   consecutive frames [offsets[b], offsets[b+1]); pairs and correspondences never
//   cross problems, the first frame of each problem is its gauge (Sec. 4.3 fixes
//   T_0), and the variables and edges of a problem are contiguous ranges.
#include <hipcub/hipcub.hpp>

#include <math.h>

#include <algorithm>

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

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 63 && (1ull << b) <= v) ++b;
  return b;
}

// depth_min <= d <= depth_max compared exactly (the FP32 depth widened to FP64)
__device__ __forceinline__ bool depth_valid(float d, double dmin, double dmax) {
  const double w = (double)d;
  return (d == d) && w >= dmin && w <= dmax && d != __builtin_inff();
}

// ---------------------------------------------------------------- dense pair test

// Does grid point p of frame i land in front of camera j and inside its image?
__device__ __forceinline__ bool grid_point_hits(const double* R, const double* t, double p0, double p1, double p2,
                                                double fx, double fy, double cx, double cy, int W, int H) {
#pragma clang fp contract(off)
  double c0 = ((R[0] * p0 + R[1] * p1) + R[2] * p2) + t[0];
  double c1 = ((R[3] * p0 + R[4] * p1) + R[5] * p2) + t[1];
  double c2 = ((R[6] * p0 + R[7] * p1) + R[8] * p2) + t[2];
  if (!(c2 > 0.0)) return false;
  double u = ((fx * c0) / c2) + cx;
  double v = ((fy * c1) / c2) + cy;
  return u >= 0.0 && u <= (double)(W - 1) && v >= 0.0 && v <= (double)(H - 1);
}

// Segment of every frame (binary search in the offsets).
__global__ void k_seg_of(const int* __restrict__ seg_start, int nseg, int F, int* __restrict__ seg_of) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  int lo = 0, hi = nseg;  // seg_start[lo] <= f < seg_start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg_start[mid] <= f) lo = mid;
    else hi = mid;
  }
  seg_of[f] = lo;
}

// One workgroup per source frame i.  The candidates j > i of the same problem are
// taken in chunks: first each candidate's orientation test and relative pose (one
// thread each, into LDS), then all (candidate, grid point) projection tests of the
// chunk spread over the workgroup, grid point by grid point.  A pair exists if any
// grid point hits, an OR, so neither the order of the tests nor the tests skipped
// once a candidate has a hit change the outcome.
// NT threads per workgroup: 1024, or 256 when no problem has more than 32 frames.
constexpr int kPairChunk = 256;
constexpr int kGridPoints = 48;

template <int NT>
__global__ void __launch_bounds__(NT) k_pair_rows(const float* __restrict__ depth,
                                                            const double* __restrict__ poses, int F, int W, int H,
                                                            double fx, double fy, double cx, double cy, double dmin,
                                                            double dmax, double cos_lim,
                                                            const int* __restrict__ seg_of,
                                                            const int* __restrict__ seg_start,
                                                            uint8_t* __restrict__ flags,
                                                            long long* __restrict__ row_count) {
  const int i = blockIdx.x;
  const int jend = seg_start[seg_of[i] + 1];
  __shared__ double gp[3][kGridPoints];
  __shared__ int gvalid[kGridPoints];
  __shared__ double Ti[16];
  __shared__ double rel[12][kPairChunk];  // R (row-major) and t of each candidate, one column each
  __shared__ int live[kPairChunk];        // orientation test passed
  __shared__ volatile int hit[kPairChunk];
  __shared__ int total;
  const int tid = threadIdx.x;
  if (tid < kGridPoints) {
    // grid pixels 5, 15, ..., 75 by 5, 15, ..., 55 at 80x60, scaled with the image
    const int a = tid % 8, b = tid / 8;
    const int x = (int)((long long)(5 + 10 * a) * W / 80), y = (int)((long long)(5 + 10 * b) * H / 60);
    int ok = 0;
    double p0 = 0, p1 = 0, p2 = 0;
    if (x < W && y < H) {
      float d = depth[(size_t)i * W * H + (size_t)y * W + x];
      if (depth_valid(d, dmin, dmax)) {
#pragma clang fp contract(off)
        double D = (double)d;
        p0 = (((double)x - cx) / fx) * D;
        p1 = (((double)y - cy) / fy) * D;
        p2 = D;
        ok = 1;
      }
    }
    gp[0][tid] = p0;
    gp[1][tid] = p1;
    gp[2][tid] = p2;
    gvalid[tid] = ok;
  }
  if (tid < 16) Ti[tid] = poses[(size_t)i * 16 + tid];
  if (tid == 0) total = 0;
  __syncthreads();
  int cnt = 0;
  for (int j0 = i + 1; j0 < jend; j0 += kPairChunk) {
    const int nc = jend - j0 < kPairChunk ? jend - j0 : kPairChunk;
    if (tid < nc) {
      const double* Tj = poses + (size_t)(j0 + tid) * 16;
      double dot;
      {
#pragma clang fp contract(off)
        dot = (Ti[2] * Tj[2] + Ti[6] * Tj[6]) + Ti[10] * Tj[10];
      }
      const bool ok = dot > cos_lim;
      if (ok) {
        double R[9], t[3];
        relative_pose_nc(Ti, Tj, R, t);
        for (int q = 0; q < 9; ++q) rel[q][tid] = R[q];
        for (int q = 0; q < 3; ++q) rel[9 + q][tid] = t[q];
      }
      live[tid] = ok ? 1 : 0;
      hit[tid] = 0;
    }
    __syncthreads();
    for (int q = tid; q < nc * kGridPoints; q += NT) {
      const int jj = q % nc, k = q / nc;
      if (live[jj] && gvalid[k] && !hit[jj]) {
        double R[9], t[3];
        for (int m = 0; m < 9; ++m) R[m] = rel[m][jj];
        for (int m = 0; m < 3; ++m) t[m] = rel[9 + m][jj];
        if (grid_point_hits(R, t, gp[0][k], gp[1][k], gp[2][k], fx, fy, cx, cy, W, H)) hit[jj] = 1;
      }
    }
    __syncthreads();
    if (tid < nc) {
      const int h = hit[tid];
      flags[(size_t)i * F + j0 + tid] = (uint8_t)h;
      cnt += h;
    }
    __syncthreads();  // the next chunk rewrites rel, live and hit
  }
  if (cnt) atomicAdd(&total, cnt);
  __syncthreads();
  if (tid == 0) row_count[i] = total;
}

// One workgroup per row: block-scan the row's flags and write the pairs in order.
__global__ void __launch_bounds__(256) k_pair_compact(const uint8_t* __restrict__ flags,
                                                      const long long* __restrict__ row_off, int F,
                                                      const int* __restrict__ seg_of,
                                                      const int* __restrict__ seg_start, int* __restrict__ pairs,
                                                      long long* __restrict__ keys) {
  const int i = blockIdx.x;
  __shared__ int sc[256];
  const int tid = threadIdx.x;
  const int jend = seg_start[seg_of[i] + 1];
  long long base = row_off[i];
  for (int j0 = i + 1; j0 < jend; j0 += 256) {
    int j = j0 + tid;
    int f = (j < jend) ? flags[(size_t)i * F + j] : 0;
    sc[tid] = f;
    __syncthreads();
    // inclusive Hillis-Steele scan
    for (int o = 1; o < 256; o <<= 1) {
      int v = (tid >= o) ? sc[tid - o] : 0;
      __syncthreads();
      sc[tid] += v;
      __syncthreads();
    }
    if (f) {
      long long r = base + sc[tid] - 1;
      pairs[2 * r] = i;
      pairs[2 * r + 1] = j;
      keys[r] = (long long)i * F + j;
    }
    base += sc[255];
    __syncthreads();
  }
}

// Caller-given pairs: range / order validation and keys.
__global__ void k_pairs_check(const int* __restrict__ ij, long long P, int F, const int* __restrict__ seg_of,
                              int* __restrict__ pairs_out, long long* __restrict__ keys, int* __restrict__ flags) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  int i = ij[2 * k], j = ij[2 * k + 1];
  bool ok = i >= 0 && j < F && i < j;
  ok = ok && seg_of[i] == seg_of[j];
  if (!ok) raise_flag(flags, kFlagBadIndex);
  if (k > 0) {
    int pi = ij[2 * k - 2], pj = ij[2 * k - 1];
    if (!(pi < i || (pi == i && pj < j))) raise_flag(flags, kFlagUnsorted);
  }
  pairs_out[2 * k] = ok ? i : 0;
  pairs_out[2 * k + 1] = ok ? j : 1;
  keys[k] = ok ? (long long)i * F + j : 1;
}

// ---------------------------------------------------------------- correspondences

// Keys and identity indices, written twice: as the sort's input and as its output
// for input that already arrives grouped (where the sort would be the identity and
// is skipped; otherwise the sort overwrites the second copy).
__global__ void k_corr_keys(const int* __restrict__ fi, const int* __restrict__ fj, const float* __restrict__ pi,
                            const float* __restrict__ pj, long long M, int F, const int* __restrict__ seg_of,
                            long long* __restrict__ key, long long* __restrict__ idx,
                            long long* __restrict__ key_sorted, long long* __restrict__ perm,
                            int* __restrict__ flags) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  int a = fi[c], b = fj[c];
  bool ok = a >= 0 && a < F && b >= 0 && b < F && a != b;
  ok = ok && seg_of[a] == seg_of[b];
  if (!ok) raise_flag(flags, kFlagBadIndex);
  for (int k = 0; k < 3; ++k)
    if (!isfinite(pi[3 * c + k]) || !isfinite(pj[3 * c + k])) raise_flag(flags, kFlagNonFinite);
  int lo = a < b ? a : b, hi = a < b ? b : a;
  const long long k = ok ? (long long)lo * F + hi : 1;
  key[c] = k;
  idx[c] = c;
  key_sorted[c] = k;
  perm[c] = c;
}

__global__ void k_corr_heads(const long long* __restrict__ ks, long long M, long long* __restrict__ head) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  head[c] = (c == 0 || ks[c] != ks[c - 1]) ? 1 : 0;
}

__global__ void k_corr_groups(const long long* __restrict__ ks, const long long* __restrict__ grp, long long M, int F,
                              int* __restrict__ sparse_ij, long long* __restrict__ sparse_keys,
                              long long* __restrict__ sparse_ptr, long long* __restrict__ counts) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  bool head = (c == 0 || ks[c] != ks[c - 1]);
  if (head) {
    long long g = grp[c] - 1;
    long long k = ks[c];
    sparse_keys[g] = k;
    sparse_ij[2 * g] = (int)(k / F);
    sparse_ij[2 * g + 1] = (int)(k % F);
    sparse_ptr[g] = c;
  }
  if (c == M - 1) {
    sparse_ptr[grp[c]] = M;
    counts[1] = grp[c];
  }
}

// One wavefront per sparse pair: FP64 moments of its correspondences in sorted order,
// with the lower frame's point as p.  Fixed reduction tree, read from lane 0.  The
// grid may exceed the number of pairs (counts[1]); the extra wavefronts return.
__global__ void __launch_bounds__(64) k_moments(const int* __restrict__ fi, const int* __restrict__ fj,
                                                const float* __restrict__ pi, const float* __restrict__ pj,
                                                const long long* __restrict__ perm,
                                                const long long* __restrict__ ptr,
                                                const long long* __restrict__ counts,
                                                double* __restrict__ mom) {
  long long g = blockIdx.x;
  if (g >= counts[1]) return;
  const int lane = threadIdx.x;
  double acc[kMomWords - 2];
  for (int k = 0; k < kMomWords - 2; ++k) acc[k] = 0.0;
  // a lane's correspondences k = k0 + lane + 64 m, in increasing m; the loads of
  // kAhead of them are issued before any is summed
  constexpr int kAhead = 4;
  const long long k0 = ptr[g], k1 = ptr[g + 1];
  for (long long kb = k0 + lane; kb < k1; kb += 64 * kAhead) {
    long long cs[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const long long k = kb + 64LL * u;
      cs[u] = k < k1 ? perm[k] : -1;
    }
    float a_[kAhead][3], b_[kAhead][3];
    bool sw[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const long long c = cs[u] < 0 ? 0 : cs[u];
      sw[u] = fi[c] > fj[c];
      for (int m = 0; m < 3; ++m) {
        a_[u][m] = pi[3 * c + m];
        b_[u][m] = pj[3 * c + m];
      }
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      if (cs[u] < 0) break;
      double p[3], q[3];
      for (int m = 0; m < 3; ++m) {
        p[m] = sw[u] ? b_[u][m] : a_[u][m];
        q[m] = sw[u] ? a_[u][m] : b_[u][m];
      }
      acc[kMN] += 1.0;
      for (int a = 0; a < 3; ++a) {
        acc[kMP + a] += p[a];
        acc[kMQ + a] += q[a];
        for (int b = 0; b < 3; ++b) {
          acc[kMPP + 3 * a + b] += p[a] * p[b];
          acc[kMQQ + 3 * a + b] += q[a] * q[b];
          acc[kMPQ + 3 * a + b] += p[a] * q[b];
        }
      }
    }
  }
  // butterfly over the lanes, all sums step by step (per sum the same tree)
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < kMomWords - 2; ++k) acc[k] += __shfl_xor(acc[k], o);
  if (lane == 0) {
    for (int k = 0; k < kMomWords - 2; ++k) mom[g * kMomWords + k] = acc[k];
    mom[g * kMomWords + kMomWords - 2] = 0.0;
    mom[g * kMomWords + kMomWords - 1] = 0.0;
  }
}

// ---------------------------------------------------------------- edges

__device__ __forceinline__ long long lower_bound_ll(const long long* a, long long n, long long key) {
  long long lo = 0, hi = n;
  while (lo < hi) {
    long long mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The number of sparse pairs nB is read on the device (counts[1]), clamped to the
// bound the buffers were sized for.
__device__ __forceinline__ long long sparse_count(const long long* counts, long long nB_max) {
  const long long n = counts[1];
  return n < nB_max ? n : nB_max;
}

__global__ void k_union_inb(const long long* __restrict__ A, long long nA, const long long* __restrict__ B,
                            const long long* __restrict__ counts, long long nB_max, long long* __restrict__ inb) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nA) return;
  const long long nB = sparse_count(counts, nB_max);
  if (k == nA) {
    inb[k] = 0;
    return;
  }
  long long pos = lower_bound_ll(B, nB, A[k]);
  inb[k] = (pos < nB && B[pos] == A[k]) ? 1 : 0;
}

// rank of a in the union = (#A < a) + (#B < a) - (#common < a); cA = exclusive scan of inb.
__global__ void k_union_write(const long long* __restrict__ A, long long nA, const long long* __restrict__ B,
                              long long nB_max, const long long* __restrict__ cA, int F, long long* __restrict__ ekeys,
                              int* __restrict__ eij, long long* __restrict__ edense, long long* __restrict__ esparse,
                              long long* __restrict__ counts) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nB = sparse_count(counts, nB_max);
  if (k == 0) counts[2] = nA + nB - cA[nA];
  if (k < nA) {
    long long key = A[k];
    long long pos = lower_bound_ll(B, nB, key);
    bool found = pos < nB && B[pos] == key;
    long long r = k + pos - cA[k];
    ekeys[r] = key;
    eij[2 * r] = (int)(key / F);
    eij[2 * r + 1] = (int)(key % F);
    edense[r] = k;
    esparse[r] = found ? pos : -1;
  } else if (k < nA + nB) {
    long long ib = k - nA;
    long long key = B[ib];
    long long pos = lower_bound_ll(A, nA, key);
    if (pos < nA && A[pos] == key) return;
    long long r = ib + pos - cA[pos];
    ekeys[r] = key;
    eij[2 * r] = (int)(key / F);
    eij[2 * r + 1] = (int)(key % F);
    edense[r] = -1;
    esparse[r] = ib;
  }
}

__global__ void k_ej_keys(const int* __restrict__ eij, long long cap, const long long* __restrict__ counts, int F,
                          int* __restrict__ kj, long long* __restrict__ idx) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cap) return;
  long long E = counts[2];
  kj[e] = e < E ? eij[2 * e + 1] : F;
  idx[e] = e;
}

__global__ void k_incidence(const long long* __restrict__ ekeys, const int* __restrict__ kj_sorted,
                            const long long* __restrict__ counts, int F, const int* __restrict__ seg_of,
                            const int* __restrict__ seg_start, long long* __restrict__ iptr,
                            long long* __restrict__ jptr, long long* __restrict__ free_flag) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > F) return;
  const long long E = counts[2];
  // four lower bounds, advanced together: first edge with i >= f and with i >= f + 1
  // (keys i*F + j), first with j >= f and with j >= f + 1 (kj_sorted)
  const long long ka = (long long)f * F, kb = (long long)(f + 1) * F;
  long long lo[4] = {0, 0, 0, 0}, hi[4] = {E, E, E, E};
  while (lo[0] < hi[0] || lo[1] < hi[1] || lo[2] < hi[2] || lo[3] < hi[3]) {
    long long mid[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) mid[s] = (lo[s] + hi[s]) >> 1;
    const bool go[4] = {lo[0] < hi[0], lo[1] < hi[1], lo[2] < hi[2], lo[3] < hi[3]};
    const long long v0 = go[0] ? ekeys[mid[0]] : 0, v1 = go[1] ? ekeys[mid[1]] : 0;
    const int v2 = go[2] ? kj_sorted[mid[2]] : 0, v3 = go[3] ? kj_sorted[mid[3]] : 0;
    const bool below[4] = {v0 < ka, v1 < kb, v2 < f, v3 < f + 1};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (go[s]) {
        if (below[s]) lo[s] = mid[s] + 1;
        else hi[s] = mid[s];
      }
  }
  iptr[f] = lo[0];
  jptr[f] = lo[2];
  if (f == F) {
    free_flag[F] = 0;
    return;
  }
  const long long deg = (lo[1] - lo[0]) + (lo[3] - lo[2]);
  free_flag[f] = (f != seg_start[seg_of[f]] && deg > 0) ? 1 : 0;
}

// Per problem: first variable (exclusive scan of the free flags at its first frame)
// and first edge (edges are sorted by i*F + j, and a problem's frames are consecutive).
__global__ void k_seg_ptrs(const int* __restrict__ seg_start, int nseg, const long long* __restrict__ free_scan,
                           const long long* __restrict__ ekeys, const long long* __restrict__ counts, int F,
                           long long* __restrict__ seg_var_ptr, long long* __restrict__ seg_edge_ptr) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nseg) return;
  const long long E = counts[2];
  const int f = seg_start[b];
  seg_var_ptr[b] = free_scan[f];
  seg_edge_ptr[b] = b == nseg ? E : lower_bound_ll(ekeys, E, (long long)f * F);
}

__global__ void k_free_write(const long long* __restrict__ free_flag, const long long* __restrict__ scan, int F,
                             int* __restrict__ var_of, int* __restrict__ frame_of_var, long long* __restrict__ counts) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > F) return;
  if (f == F) {
    counts[3] = scan[F];
    return;
  }
  if (free_flag[f]) {
    var_of[f] = (int)scan[f];
    frame_of_var[scan[f]] = f;
  } else {
    var_of[f] = -1;
  }
}

// Per free frame (PCG row): number of incident edges whose other frame is free.
// One wavefront per row, lanes over the incident edges.
__global__ void __launch_bounds__(64) k_row_count(const long long* __restrict__ iptr,
                                                  const long long* __restrict__ jptr,
                                                  const long long* __restrict__ ej_sorted,
                                                  const int* __restrict__ eij, const int* __restrict__ var_of,
                                                  const int* __restrict__ frame_of_var, long long nfree,
                                                  long long* __restrict__ cnt) {
  const long long v = blockIdx.x;
  const int lane = threadIdx.x;
  if (v == nfree) {
    if (lane == 0) cnt[v] = 0;
    return;
  }
  const int f = frame_of_var[v];
  long long n = 0;
  for (long long k = iptr[f] + lane; k < iptr[f + 1]; k += 64) n += var_of[eij[2 * k + 1]] >= 0 ? 1 : 0;
  for (long long k = jptr[f] + lane; k < jptr[f + 1]; k += 64) n += var_of[eij[2 * ej_sorted[k]]] >= 0 ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if (lane == 0) cnt[v] = n;
}

// Row entries (partner variable, 2*edge+transposed) in incidence order: one
// wavefront per row, positions from a ballot prefix over each 64-edge chunk.
__global__ void __launch_bounds__(64) k_row_fill(const long long* __restrict__ iptr,
                                                 const long long* __restrict__ jptr,
                                                 const long long* __restrict__ ej_sorted,
                                                 const int* __restrict__ eij, const int* __restrict__ var_of,
                                                 const int* __restrict__ frame_of_var, long long nfree,
                                                 const long long* __restrict__ row_ptr, int2* __restrict__ entries) {
  const long long v = blockIdx.x;
  if (v >= nfree) return;
  const int lane = threadIdx.x;
  const int f = frame_of_var[v];
  long long o = row_ptr[v];
  for (int side = 0; side < 2; ++side) {
    const long long k0 = side == 0 ? iptr[f] : jptr[f], k1 = side == 0 ? iptr[f + 1] : jptr[f + 1];
    for (long long kb = k0; kb < k1; kb += 64) {
      const long long k = kb + lane;
      int w = -1;
      long long e = 0;
      if (k < k1) {
        e = side == 0 ? k : ej_sorted[k];
        w = var_of[side == 0 ? eij[2 * e + 1] : eij[2 * e]];
      }
      const bool keep = w >= 0;
      const unsigned long long mask = __ballot(keep);
      const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
      if (keep) entries[o + rank] = make_int2(w, (int)(2 * e + side));
      o += __popcll(mask);
    }
  }
}

// 1 in *flag if the correspondence keys are not in non-decreasing order.
__global__ void k_keys_unsorted(const long long* __restrict__ key, long long M, int* __restrict__ flag) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > 0 && c < M && key[c] < key[c - 1]) *flag = 1;
}

// Largest bound on the number of sparse pairs for which that number is not read
// back before the edge union (larger bounds would size the union and the
// incidence sort far beyond the real count).
constexpr long long kSparseBoundNoSync = 1 << 17;

inline unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// Counts, flags and optionally `n_extra` words at `extra` (device memory), read back
// in one round trip through pinned host memory.
void read_counts(Context& c, long long* host_counts, int* host_flags, const long long* extra = nullptr,
                 size_t n_extra = 0, long long* host_extra = nullptr) {
  long long* rb = readback_small(c);
  long long* rbx = n_extra ? static_cast<long long*>(readback_big(c, sizeof(long long) * n_extra)) : nullptr;
  check_hip(hipMemcpyAsync(rb, c.counts.p, 8 * sizeof(long long), hipMemcpyDeviceToHost, c.stream), "copy counts");
  check_hip(hipMemcpyAsync(rb + 8, c.flags.p, sizeof(int), hipMemcpyDeviceToHost, c.stream), "copy flags");
  if (n_extra)
    check_hip(hipMemcpyAsync(rbx, extra, sizeof(long long) * n_extra, hipMemcpyDeviceToHost, c.stream), "copy");
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  for (int k = 0; k < 8; ++k) host_counts[k] = rb[k];
  *host_flags = *reinterpret_cast<const int*>(rb + 8);
  for (size_t k = 0; k < n_extra; ++k) host_extra[k] = rbx[k];
}

void raise_device_flags(int fl) {
  if (fl & kFlagBadIndex) fail(BF_ERR_INVALID_ARG, "frame index out of range, equal frames or i >= j");
  if (fl & kFlagUnsorted) fail(BF_ERR_INVALID_ARG, "dense pairs are not strictly increasing");
  if (fl & kFlagNonFinite) fail(BF_ERR_NONFINITE, "non-finite correspondence point");
}

}  // namespace

// Pair search in two halves around one host synchronisation: the first launches
// the per-row tests and the scan (the count ends up in row_off[F]), the second
// compacts the pairs once the count is known on the host.
void pair_search_begin(Context& c, const bf_frames& fr, const bf_intrinsics& in, const double* poses,
                       const bf_params& prm) {
  const int F = fr.num_frames;
  ensure(c.pair_flags, (size_t)F * F);
  ensure(c.row_count, sizeof(long long) * (F + 1));
  ensure(c.row_off, sizeof(long long) * (F + 1));
  double cos_lim = cos(prm.max_angle_deg * (M_PI / 180.0));
  int max_frames = 0;
  for (size_t b = 0; b + 1 < c.seg_host.size(); ++b) max_frames = std::max(max_frames, c.seg_host[b + 1] - c.seg_host[b]);
  const bool small = max_frames <= 32;
  hipLaunchKernelGGL(small ? k_pair_rows<256> : k_pair_rows<1024>, dim3(F), dim3(small ? 256 : 1024), 0, c.stream, fr.depth, poses, F, in.width, in.height, in.fx,
                     in.fy, in.cx, in.cy, prm.depth_min, prm.depth_max, cos_lim,
                     c.seg_of.as<int>(), c.seg_start.as<int>(), c.pair_flags.as<uint8_t>(),
                     c.row_count.as<long long>());
  check_hip(hipMemsetAsync(c.row_count.as<long long>() + F, 0, sizeof(long long), c.stream), "memset");
  long long* rc = c.row_count.as<long long>();
  long long* ro = c.row_off.as<long long>();
  cub_call(c, [&](void* t, size_t& b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, rc, ro, F + 1, c.stream);
  });
}

void pair_search_finish(Context& c, int F, long long P) {
  ensure(c.pairs, sizeof(int) * 2 * (P + 1));
  ensure(c.pair_keys, sizeof(long long) * (P + 1));
  hipLaunchKernelGGL(k_pair_compact, dim3(F), dim3(256), 0, c.stream, c.pair_flags.as<uint8_t>(),
                     c.row_off.as<long long>(), F, c.seg_of.as<int>(), c.seg_start.as<int>(), c.pairs.as<int>(),
                     c.pair_keys.as<long long>());
}

int64_t launch_pair_search(Context& c, const bf_frames& fr, const bf_intrinsics& in, const double* poses,
                           const bf_params& prm) {
  const int F = fr.num_frames;
  pair_search_begin(c, fr, in, poses, prm);
  long long* rb = readback_small(c);
  check_hip(hipMemcpyAsync(rb, c.row_off.as<long long>() + F, sizeof(long long), hipMemcpyDeviceToHost, c.stream),
            "copy pair count");
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  const long long P = rb[0];
  pair_search_finish(c, F, P);
  return P;
}

// Correspondences grouped by unordered frame pair (stable: input order within a
// pair): fills corr_perm (sorted position -> input index), sparse_ptr and
// sparse_ij; returns the number of pairs.  One problem of F frames.
int64_t group_correspondences(Context& c, const bf_corrs& co, int F) {
  set_segments(c, F, nullptr, 1);
  const long long M = co.count;
  ensure(c.counts, 8 * sizeof(long long));
  ensure(c.flags, sizeof(int));
  check_hip(hipMemsetAsync(c.counts.p, 0, 8 * sizeof(long long), c.stream), "memset counts");
  ensure(c.corr_key, sizeof(long long) * (M + 1));
  ensure(c.corr_idx, sizeof(long long) * (M + 1));
  ensure(c.corr_key_sorted, sizeof(long long) * (M + 1));
  ensure(c.corr_perm, sizeof(long long) * (M + 1));
  ensure(c.corr_head, sizeof(long long) * (M + 1));
  ensure(c.corr_group, sizeof(long long) * (M + 1));
  ensure(c.sparse_ij, sizeof(int) * 2 * (M + 1));
  ensure(c.sparse_keys, sizeof(long long) * (M + 1));
  ensure(c.sparse_ptr, sizeof(long long) * (M + 2));
  if (M == 0) return 0;
  hipLaunchKernelGGL(k_corr_keys, dim3(blocks_for(M)), dim3(256), 0, c.stream, co.frame_i, co.frame_j, co.p_i, co.p_j,
                     M, F, c.seg_of.as<int>(), c.corr_key.as<long long>(), c.corr_idx.as<long long>(),
                     c.corr_key_sorted.as<long long>(), c.corr_perm.as<long long>(), c.flags.as<int>());
  int endbit = bits_for((uint64_t)F * (uint64_t)F);
  long long* k_in = c.corr_key.as<long long>();
  long long* k_out = c.corr_key_sorted.as<long long>();
  long long* v_in = c.corr_idx.as<long long>();
  long long* v_out = c.corr_perm.as<long long>();
  cub_call(c, [&](void* t, size_t& b) {
    return hipcub::DeviceRadixSort::SortPairs(t, b, k_in, k_out, v_in, v_out, (int)M, 0, endbit, c.stream);
  });
  hipLaunchKernelGGL(k_corr_heads, dim3(blocks_for(M)), dim3(256), 0, c.stream, k_out, M, c.corr_head.as<long long>());
  long long* hd = c.corr_head.as<long long>();
  long long* gp = c.corr_group.as<long long>();
  cub_call(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::InclusiveSum(t, b, hd, gp, (int)M, c.stream); });
  hipLaunchKernelGGL(k_corr_groups, dim3(blocks_for(M)), dim3(256), 0, c.stream, k_out, gp, M, F,
                     c.sparse_ij.as<int>(), c.sparse_keys.as<long long>(), c.sparse_ptr.as<long long>(),
                     c.counts.as<long long>());
  long long hc[8];
  int hf = 0;
  read_counts(c, hc, &hf);
  raise_device_flags(hf);
  return hc[1];
}

void set_segments(Context& c, int F, const int32_t* offsets, int nseg) {
  std::vector<int> h;
  if (offsets) {
    if (nseg < 1) fail(BF_ERR_INVALID_ARG, "num_problems must be >= 1");
    if (offsets[0] != 0 || offsets[nseg] != F) fail(BF_ERR_INVALID_ARG, "frame offsets must run from 0 to num_frames");
    for (int b = 0; b < nseg; ++b)
      if (offsets[b + 1] <= offsets[b]) fail(BF_ERR_INVALID_ARG, "frame offsets must be strictly increasing");
    h.assign(offsets, offsets + nseg + 1);
  } else {
    nseg = 1;
    h = {0, F};
  }
  if (h == c.seg_host && c.seg_of.cap >= sizeof(int) * F) {  // already on the device
    c.shape.nseg = nseg;
    return;
  }
  c.seg_host.clear();
  ensure(c.seg_start, sizeof(int) * (nseg + 1));
  ensure(c.seg_of, sizeof(int) * F);
  check_hip(hipMemcpyAsync(c.seg_start.p, h.data(), sizeof(int) * (nseg + 1), hipMemcpyHostToDevice, c.stream),
            "copy frame offsets");
  hipLaunchKernelGGL(k_seg_of, dim3(blocks_for(F)), dim3(256), 0, c.stream, c.seg_start.as<int>(), nseg, F,
                     c.seg_of.as<int>());
  // the host vector must outlive the copy
  check_hip(hipStreamSynchronize(c.stream), "synchronise");
  c.seg_host = h;
  c.shape.nseg = nseg;
}

void build_structure(Context& c, const bf_frames& fr, const bf_intrinsics& in, const bf_corrs* co,
                     const bf_pairs* pairs, const double* poses, const bf_params& prm) {
  const int F = fr.num_frames;
  Shape sh;
  sh.nseg = c.shape.nseg;
  sh.F = F;
  sh.W = in.width;
  sh.H = in.height;
  ensure(c.counts, 8 * sizeof(long long));
  ensure(c.flags, sizeof(int));
  check_hip(hipMemsetAsync(c.counts.p, 0, 8 * sizeof(long long), c.stream), "memset counts");

  // a1: frames
  size_t HW = (size_t)in.width * in.height;
  ensure(c.nd, sizeof(float4) * HW * F);
  ensure(c.grad, sizeof(float) * HW * F);
  ensure(c.kx, sizeof(float) * in.width);
  ensure(c.ky, sizeof(float) * in.height);
  ensure(c.kx64, sizeof(double) * in.width);
  ensure(c.ky64, sizeof(double) * in.height);
  launch_prepare(c, fr, in, prm);

  // a2: dense pairs (the search's count is read together with the correspondence
  // check below, in one host synchronisation)
  const bool search = prm.use_dense && !pairs;
  if (!prm.use_dense) {
    sh.P = 0;
    ensure(c.pairs, 8);
    ensure(c.pair_keys, 8);
  } else if (pairs) {
    sh.P = pairs->count;
    ensure(c.pairs, sizeof(int) * 2 * (sh.P + 1));
    ensure(c.pair_keys, sizeof(long long) * (sh.P + 1));
    if (sh.P > 0)
      hipLaunchKernelGGL(k_pairs_check, dim3(blocks_for(sh.P)), dim3(256), 0, c.stream, pairs->ij, (long long)sh.P, F,
                         c.seg_of.as<int>(), c.pairs.as<int>(), c.pair_keys.as<long long>(), c.flags.as<int>());
  } else {
    pair_search_begin(c, fr, in, poses, prm);
  }

  // correspondences: keys; a stable sort groups them by frame pair -- skipped when
  // they already arrive grouped in key order (the sort would be the identity)
  const long long M = (prm.use_sparse && co) ? co->count : 0;
  sh.M = M;
  ensure(c.corr_key, sizeof(long long) * (M + 1));
  ensure(c.corr_idx, sizeof(long long) * (M + 1));
  ensure(c.corr_key_sorted, sizeof(long long) * (M + 1));
  ensure(c.corr_perm, sizeof(long long) * (M + 1));
  ensure(c.corr_head, sizeof(long long) * (M + 1));
  ensure(c.corr_group, sizeof(long long) * (M + 1));
  ensure(c.sparse_ij, sizeof(int) * 2 * (M + 1));
  ensure(c.sparse_keys, sizeof(long long) * (M + 1));
  ensure(c.sparse_ptr, sizeof(long long) * (M + 2));
  if (M > 0) {
    hipLaunchKernelGGL(k_corr_keys, dim3(blocks_for(M)), dim3(256), 0, c.stream, co->frame_i, co->frame_j, co->p_i,
                       co->p_j, M, F, c.seg_of.as<int>(), c.corr_key.as<long long>(), c.corr_idx.as<long long>(),
                       c.corr_key_sorted.as<long long>(), c.corr_perm.as<long long>(), c.flags.as<int>());
    hipLaunchKernelGGL(k_keys_unsorted, dim3(blocks_for(M)), dim3(256), 0, c.stream, c.corr_key.as<long long>(), M,
                       reinterpret_cast<int*>(c.counts.as<long long>() + 7));
  }
  long long hc0[8];
  int hf0 = 0;
  long long P_found = 0;
  if (search) read_counts(c, hc0, &hf0, c.row_off.as<long long>() + F, 1, &P_found);
  else read_counts(c, hc0, &hf0);
  raise_device_flags(hf0);
  const bool unsorted = hc0[7] != 0;
  if (search) {
    sh.P = P_found;
    pair_search_finish(c, F, P_found);
  }
  if (M > 0) {
    long long* k_out = c.corr_key_sorted.as<long long>();
    long long* v_out = c.corr_perm.as<long long>();
    if (unsorted) {
      int endbit = bits_for((uint64_t)F * (uint64_t)F);
      long long* k_in = c.corr_key.as<long long>();
      long long* v_in = c.corr_idx.as<long long>();
      cub_call(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, k_in, k_out, v_in, v_out, (int)M, 0, endbit, c.stream);
      });
    }  // else k_corr_keys has already written k_out and v_out
    hipLaunchKernelGGL(k_corr_heads, dim3(blocks_for(M)), dim3(256), 0, c.stream, k_out, M,
                       c.corr_head.as<long long>());
    long long* hd = c.corr_head.as<long long>();
    long long* gp = c.corr_group.as<long long>();
    cub_call(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::InclusiveSum(t, b, hd, gp, (int)M, c.stream); });
    hipLaunchKernelGGL(k_corr_groups, dim3(blocks_for(M)), dim3(256), 0, c.stream, k_out, gp, M, F,
                       c.sparse_ij.as<int>(), c.sparse_keys.as<long long>(), c.sparse_ptr.as<long long>(),
                       c.counts.as<long long>());
  }

  // The number of sparse pairs S stays on the device while its bound is small: the
  // kernels up to the incidence are sized by the bound and read S there, and the
  // host learns it with the edge count.  Distinct keys are pairs inside one problem,
  // plus the stand-in key of a rejected correspondence.
  long long hc[8];
  int hf = 0;
  long long s_bound = 0;
  if (M > 0) {
    long long within = 1;
    for (size_t b = 0; b + 1 < c.seg_host.size(); ++b) {
      const long long n = c.seg_host[b + 1] - c.seg_host[b];
      within += n * (n - 1) / 2;
    }
    s_bound = std::min(M, within);
    if (s_bound > kSparseBoundNoSync) {
      read_counts(c, hc, &hf);
      raise_device_flags(hf);
      s_bound = hc[1];
    }
  }

  ensure(c.moments, sizeof(double) * kMomWords * (s_bound + 1));
  if (s_bound > 0)
    hipLaunchKernelGGL(k_moments, dim3((unsigned)s_bound), dim3(64), 0, c.stream, co->frame_i, co->frame_j, co->p_i,
                       co->p_j, c.corr_perm.as<long long>(), c.sparse_ptr.as<long long>(), c.counts.as<long long>(),
                       c.moments.as<double>());

  // edges = union(dense pairs, sparse pairs)
  const long long cap = sh.P + s_bound;
  ensure(c.in_b, sizeof(long long) * (sh.P + 1));
  ensure(c.common_scan, sizeof(long long) * (sh.P + 1));
  ensure(c.edge_keys, sizeof(long long) * (cap + 1));
  ensure(c.edge_ij, sizeof(int) * 2 * (cap + 1));
  ensure(c.edge_dense, sizeof(long long) * (cap + 1));
  ensure(c.edge_sparse, sizeof(long long) * (cap + 1));
  long long* A = c.pair_keys.as<long long>();
  long long* B = c.sparse_keys.as<long long>();
  hipLaunchKernelGGL(k_union_inb, dim3(blocks_for(sh.P + 1)), dim3(256), 0, c.stream, A, (long long)sh.P, B,
                     c.counts.as<long long>(), s_bound, c.in_b.as<long long>());
  long long* ib = c.in_b.as<long long>();
  long long* cs = c.common_scan.as<long long>();
  cub_call(c, [&](void* t, size_t& b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, ib, cs, (int)(sh.P + 1), c.stream);
  });
  hipLaunchKernelGGL(k_union_write, dim3(blocks_for(cap > 0 ? cap : 1)), dim3(256), 0, c.stream, A, (long long)sh.P, B,
                     s_bound, cs, F, c.edge_keys.as<long long>(), c.edge_ij.as<int>(),
                     c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.counts.as<long long>());

  // incidence: edges sorted by the upper frame (stable), per-frame ranges
  ensure(c.ej_key, sizeof(int) * (cap + 1));
  ensure(c.ej_idx, sizeof(long long) * (cap + 1));
  ensure(c.ej_key_sorted, sizeof(int) * (cap + 1));
  ensure(c.ej_sorted, sizeof(long long) * (cap + 1));
  ensure(c.iptr, sizeof(long long) * (F + 1));
  ensure(c.jptr, sizeof(long long) * (F + 1));
  ensure(c.free_flag, sizeof(long long) * (F + 1));
  ensure(c.var_of, sizeof(int) * (F + 1));
  ensure(c.frame_of_var, sizeof(int) * (F + 1));
  if (cap > 0) {
    hipLaunchKernelGGL(k_ej_keys, dim3(blocks_for(cap)), dim3(256), 0, c.stream, c.edge_ij.as<int>(), (long long)cap,
                       c.counts.as<long long>(), F, c.ej_key.as<int>(), c.ej_idx.as<long long>());
    int* kin = c.ej_key.as<int>();
    int* kout = c.ej_key_sorted.as<int>();
    long long* vin = c.ej_idx.as<long long>();
    long long* vout = c.ej_sorted.as<long long>();
    int endbit = bits_for((uint64_t)F + 1);
    cub_call(c, [&](void* t, size_t& b) {
      return hipcub::DeviceRadixSort::SortPairs(t, b, kin, kout, vin, vout, (int)cap, 0, endbit, c.stream);
    });
  }
  hipLaunchKernelGGL(k_incidence, dim3(blocks_for(F + 1)), dim3(256), 0, c.stream, c.edge_keys.as<long long>(),
                     c.ej_key_sorted.as<int>(), c.counts.as<long long>(), F, c.seg_of.as<int>(),
                     c.seg_start.as<int>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                     c.free_flag.as<long long>());
  long long* ff = c.free_flag.as<long long>();
  ensure(c.row_off, sizeof(long long) * (F + 1));
  long long* fs = c.row_off.as<long long>();
  cub_call(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::ExclusiveSum(t, b, ff, fs, F + 1, c.stream); });
  hipLaunchKernelGGL(k_free_write, dim3(blocks_for(F + 1)), dim3(256), 0, c.stream, ff, fs, F, c.var_of.as<int>(),
                     c.frame_of_var.as<int>(), c.counts.as<long long>());
  const int nseg = c.shape.nseg;
  ensure(c.seg_var_ptr, sizeof(long long) * (nseg + 1));
  ensure(c.seg_edge_ptr, sizeof(long long) * (nseg + 1));
  hipLaunchKernelGGL(k_seg_ptrs, dim3(blocks_for(nseg + 1)), dim3(256), 0, c.stream, c.seg_start.as<int>(), nseg, fs,
                     c.edge_keys.as<long long>(), c.counts.as<long long>(), F, c.seg_var_ptr.as<long long>(),
                     c.seg_edge_ptr.as<long long>());
  std::vector<long long> svp(nseg + 1);
  read_counts(c, hc, &hf, c.seg_var_ptr.as<long long>(), (size_t)nseg + 1, svp.data());
  raise_device_flags(hf);
  sh.S = M > 0 ? hc[1] : 0;
  if (sh.S > s_bound) fail(BF_ERR_DEVICE, "sparse pair count exceeds its bound");
  sh.E = hc[2];
  sh.nfree = hc[3];
  sh.nseg = nseg;
  sh.max_seg_free = 0;
  for (int b = 0; b < nseg; ++b) sh.max_seg_free = std::max<int64_t>(sh.max_seg_free, svp[b + 1] - svp[b]);

  // PCG rows: (partner variable, edge) lists of every free frame
  ensure(c.row_cnt, sizeof(long long) * (sh.nfree + 1));
  ensure(c.row_ptr, sizeof(long long) * (sh.nfree + 1));
  ensure(c.row_entries, sizeof(int2) * (2 * sh.E + 1));
  hipLaunchKernelGGL(k_row_count, dim3((unsigned)(sh.nfree + 1)), dim3(64), 0, c.stream, c.iptr.as<long long>(),
                     c.jptr.as<long long>(), c.ej_sorted.as<long long>(), c.edge_ij.as<int>(), c.var_of.as<int>(),
                     c.frame_of_var.as<int>(), (long long)sh.nfree, c.row_cnt.as<long long>());
  long long* rcnt = c.row_cnt.as<long long>();
  long long* rptr = c.row_ptr.as<long long>();
  cub_call(c, [&](void* t, size_t& b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, rcnt, rptr, (int)(sh.nfree + 1), c.stream);
  });
  if (sh.nfree > 0)
    hipLaunchKernelGGL(k_row_fill, dim3((unsigned)sh.nfree), dim3(64), 0, c.stream, c.iptr.as<long long>(),
                       c.jptr.as<long long>(), c.ej_sorted.as<long long>(), c.edge_ij.as<int>(), c.var_of.as<int>(),
                       c.frame_of_var.as<int>(), (long long)sh.nfree, rptr, c.row_entries.as<int2>());
  c.shape = sh;
}

}  // namespace bf
