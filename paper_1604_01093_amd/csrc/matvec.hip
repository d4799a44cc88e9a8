// Products y = H x with the normal-equation matrix of the last assembled system,
// in two representations (paper Sec. 4.4):
//
// * assembled: from the per-edge 6x6 blocks (H_ii, H_jj, H_ij), one wavefront per
//   frame over its incident edges -- the representation the PCG kernels use;
// * matrix-free sparse term: the paper's two-step product J^T (J x) over the
//   sparse correspondences, never forming the blocks: one thread per
//   correspondence computes u = J_i x_i + J_j x_j (3 values), then one workgroup
//   per frame sums J_f^T u over every correspondence of the frame (per-frame lists
//   from the edge incidence and the correspondence grouping).
//
// For a correspondence between frames a < b with points p (camera a) and q
// (camera b): r = T_a p - T_b q, J_a = R_a [-[p]x | I], J_b = -R_b [-[q]x | I]
// with respect to right perturbations (omega, v).  Both products are deterministic
// (fixed summation orders).
#include "internal.h"

namespace bf {

namespace {

__device__ __forceinline__ void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// One wavefront per frame: lanes take the frame's incident edges, then a fixed
// butterfly.  H from the FP64 edge records.
__global__ void __launch_bounds__(64) k_matvec_blocks(const double* __restrict__ eb, const int* __restrict__ eij,
                                                      const long long* __restrict__ iptr,
                                                      const long long* __restrict__ jptr,
                                                      const long long* __restrict__ ej_sorted, int F,
                                                      const double* __restrict__ x, double* __restrict__ y) {
  const int f = blockIdx.x, lane = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long k = iptr[f] + lane; k < iptr[f + 1]; k += 64) {
    const double* B = eb + (size_t)k * kEdgeWords;
    const int j = eij[2 * k + 1];
    for (int a = 0; a < 6; ++a) {
      double s = 0.0;
      for (int b = 0; b < 6; ++b) s += B[kEHii + 6 * a + b] * x[6 * f + b] + B[kEHij + 6 * a + b] * x[6 * j + b];
      acc[a] += s;
    }
  }
  for (long long k = jptr[f] + lane; k < jptr[f + 1]; k += 64) {
    const long long e = ej_sorted[k];
    const double* B = eb + (size_t)e * kEdgeWords;
    const int i = eij[2 * e];
    for (int a = 0; a < 6; ++a) {
      double s = 0.0;
      for (int b = 0; b < 6; ++b) s += B[kEHjj + 6 * a + b] * x[6 * f + b] + B[kEHij + 6 * b + a] * x[6 * i + b];
      acc[a] += s;
    }
  }
  for (int a = 0; a < 6; ++a) {
    double v = acc[a];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) y[6 * f + a] = v;
  }
}

// u_k = J_a x_a + J_b x_b for the correspondence at sorted position k (FP32, the
// precision of the correspondence points).
__global__ void k_mf_jx(const int* __restrict__ fi, const int* __restrict__ fj, const float* __restrict__ pi,
                        const float* __restrict__ pj, const long long* __restrict__ perm,
                        const long long* __restrict__ group, const int* __restrict__ sparse_ij, long long M,
                        const double* __restrict__ poses, const double* __restrict__ x, float* __restrict__ u) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const long long c = perm[k];
  const long long g = group[k] - 1;
  const int a = sparse_ij[2 * g], b = sparse_ij[2 * g + 1];
  const bool sw = fi[c] > fj[c];
  const float* P = sw ? pj : pi;
  const float* Q = sw ? pi : pj;
  float out[3] = {0.f, 0.f, 0.f};
  for (int side = 0; side < 2; ++side) {
    const int f = side == 0 ? a : b;
    const float* pt = side == 0 ? P : Q;
    const float s = side == 0 ? 1.0f : -1.0f;
    const float w[3] = {(float)x[6 * f], (float)x[6 * f + 1], (float)x[6 * f + 2]};
    const float v[3] = {(float)x[6 * f + 3], (float)x[6 * f + 4], (float)x[6 * f + 5]};
    const float p3[3] = {pt[3 * c], pt[3 * c + 1], pt[3 * c + 2]};
    // omega x p + v, then R_f
    const float l[3] = {w[1] * p3[2] - w[2] * p3[1] + v[0], w[2] * p3[0] - w[0] * p3[2] + v[1],
                        w[0] * p3[1] - w[1] * p3[0] + v[2]};
    const double* T = poses + (size_t)f * 16;
    for (int r = 0; r < 3; ++r)
      out[r] += s * ((float)T[4 * r] * l[0] + (float)T[4 * r + 1] * l[1] + (float)T[4 * r + 2] * l[2]);
  }
  u[3 * k] = out[0];
  u[3 * k + 1] = out[1];
  u[3 * k + 2] = out[2];
}

// y_f = w sum_k J_f^T u_k over the frame's correspondences: one workgroup of 256
// per frame, threads striding over each incident edge's correspondences, a fixed
// tree at the end (FP64 sums).
__global__ void __launch_bounds__(256) k_mf_jtu(const int* __restrict__ fi, const int* __restrict__ fj,
                                                const float* __restrict__ pi, const float* __restrict__ pj,
                                                const long long* __restrict__ perm,
                                                const long long* __restrict__ sparse_ptr,
                                                const long long* __restrict__ edge_sparse,
                                                const long long* __restrict__ iptr, const long long* __restrict__ jptr,
                                                const long long* __restrict__ ej_sorted,
                                                const double* __restrict__ poses, const float* __restrict__ u,
                                                double w, double* __restrict__ y) {
  __shared__ double red[256];
  const int f = blockIdx.x, tid = threadIdx.x;
  const double* T = poses + (size_t)f * 16;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int side = 0; side < 2; ++side) {
    const long long e0 = side == 0 ? iptr[f] : jptr[f], e1 = side == 0 ? iptr[f + 1] : jptr[f + 1];
    for (long long k = e0; k < e1; ++k) {
      const long long e = side == 0 ? k : ej_sorted[k];
      const long long g = edge_sparse[e];
      if (g < 0) continue;
      for (long long m = sparse_ptr[g] + tid; m < sparse_ptr[g + 1]; m += 256) {
        const long long c = perm[m];
        const bool sw = fi[c] > fj[c];
        const float* pt = (side == 0) == !sw ? pi : pj;  // this frame's point of the correspondence
        const double p3[3] = {pt[3 * c], pt[3 * c + 1], pt[3 * c + 2]};
        double aR[3];  // R_f^T u
        for (int r = 0; r < 3; ++r)
          aR[r] = T[r] * (double)u[3 * m] + T[4 + r] * (double)u[3 * m + 1] + T[8 + r] * (double)u[3 * m + 2];
        double cr[3];
        cross3(p3, aR, cr);
        const double s = side == 0 ? 1.0 : -1.0;
        for (int r = 0; r < 3; ++r) {
          acc[r] += s * cr[r];
          acc[3 + r] += s * aR[r];
        }
      }
    }
  }
  for (int a = 0; a < 6; ++a) {
    red[tid] = acc[a];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) y[6 * f + a] = w * red[0];
    __syncthreads();
  }
}

}  // namespace

void launch_matvec(Context& c, const bf_corrs* co, double w_sparse, int mode, const double* x, double* y) {
  const int F = c.shape.F;
  if (mode == 0) {
    if (c.shape.E == 0) {
      check_hip(hipMemsetAsync(y, 0, sizeof(double) * 6 * F, c.stream), "memset");
      return;
    }
    hipLaunchKernelGGL(k_matvec_blocks, dim3(F), dim3(64), 0, c.stream, c.eblocks.as<double>(), c.edge_ij.as<int>(),
                       c.iptr.as<long long>(), c.jptr.as<long long>(), c.ej_sorted.as<long long>(), F, x, y);
    return;
  }
  const long long M = c.shape.M;
  if (M == 0 || c.shape.S == 0 || !co) {
    check_hip(hipMemsetAsync(y, 0, sizeof(double) * 6 * F, c.stream), "memset");
    return;
  }
  ensure(c.mf_u, sizeof(float) * 3 * (size_t)M);
  hipLaunchKernelGGL(k_mf_jx, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, c.stream, co->frame_i, co->frame_j,
                     co->p_i, co->p_j, c.corr_perm.as<long long>(), c.corr_group.as<long long>(),
                     c.sparse_ij.as<int>(), M, c.sys_poses.as<double>(), x, c.mf_u.as<float>());
  hipLaunchKernelGGL(k_mf_jtu, dim3(F), dim3(256), 0, c.stream, co->frame_i, co->frame_j, co->p_i, co->p_j,
                     c.corr_perm.as<long long>(), c.sparse_ptr.as<long long>(), c.edge_sparse.as<long long>(),
                     c.iptr.as<long long>(), c.jptr.as<long long>(), c.ej_sorted.as<long long>(),
                     c.sys_poses.as<double>(), c.mf_u.as<float>(), w_sparse, y);
}

}  // namespace bf
