// Normal equations, block-Jacobi PCG and pose update (paper Sec. 4.4).
//
// Per edge (i, j) in FP64:
//  * sparse term from the pair's moments (E_sparse of Sec. 4.3 is quadratic in the
//    correspondence points, so its blocks need only sums of p, q, p p^T, q q^T and
//    p q^T).  With (R, t) = T_ji and A_p = [-[p]x | I]:
//      H_ii = sum A_p^T A_p,  H_jj = sum A_q^T A_q,  H_ij = -sum A_p^T R^T A_q,
//      g_i  = sum A_p^T R^T e,  g_j = -sum A_q^T e,  e = R p + t - q,  E = sum |e|^2.
//  * dense term lifted from the pair job's frame-j block with the adjoint of T_ji:
//      H_ii = Ad^T H_jj Ad,  H_ij = -Ad^T H_jj,  g_i = -Ad^T g_j.
// Per free frame: the diagonal block and gradient summed over incident edges in
// a fixed order, and the 6x6 Cholesky inverse for the block-Jacobi preconditioner.
// PCG: x0 = 0, fixed iteration count, early exit when r^T z <= 1e-30, FP64 dot
// products and alpha/beta; matrix and vectors in FP32 (default) or FP64.
// Update: T_f <- T_f Exp(x_f) in FP64 (Sec. 4.3 exponential map).
#include "internal.h"

namespace bf {

namespace {

__device__ __forceinline__ int eps3(int a, int b, int c) {
  // Levi-Civita symbol for indices in {0,1,2}
  return ((a - b) * (b - c) * (c - a)) / 2;
}

__device__ __forceinline__ void skew(const double* v, double* S) {
  S[0] = 0;
  S[1] = -v[2];
  S[2] = v[1];
  S[3] = v[2];
  S[4] = 0;
  S[5] = -v[0];
  S[6] = -v[1];
  S[7] = v[0];
  S[8] = 0;
}

template <class T>
__global__ void __launch_bounds__(64) k_edge_blocks(const int* __restrict__ eij, long long E,
                                                    const long long* __restrict__ edense,
                                                    const long long* __restrict__ esparse,
                                                    const double* __restrict__ mom, const double* __restrict__ rec,
                                                    const double* __restrict__ poses, double w_sparse, int jac,
                                                    double* __restrict__ eb, T* __restrict__ hij_store) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int i = eij[2 * e], j = eij[2 * e + 1];
  double R[9], t[3];
  relative_pose_nc(poses + (size_t)i * 16, poses + (size_t)j * 16, R, t);
  double* out = eb + (size_t)e * kEdgeWords;
  const long long s = esparse[e];
  const long long d = edense[e];

  double Hjj_d[36];
  double gj_d[6];
  for (int k = 0; k < 36; ++k) Hjj_d[k] = 0.0;
  for (int k = 0; k < 6; ++k) gj_d[k] = 0.0;
  double Eg = 0, Ep = 0, ng = 0, np = 0;
  if (d >= 0) {
    const double* r = rec + (size_t)d * kRecWords;
    if (jac) {
      int k = 0;
      for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) {
          Hjj_d[6 * a + b] = r[k];
          Hjj_d[6 * b + a] = r[k];
          ++k;
        }
      for (int a = 0; a < 6; ++a) gj_d[a] = r[kRecG + a];
    }
    Eg = r[kRecEg];
    Ep = r[kRecEp];
    ng = r[kRecNg];
    np = r[kRecNp];
  }
  double Es = 0, ns = 0;
  // sparse moments
  double n = 0, sp[3] = {0, 0, 0}, sq[3] = {0, 0, 0}, Spp[9], Sqq[9], Spq[9];
  for (int k = 0; k < 9; ++k) Spp[k] = Sqq[k] = Spq[k] = 0.0;
  if (s >= 0) {
    const double* m = mom + (size_t)s * kMomWords;
    n = m[kMN];
    for (int a = 0; a < 3; ++a) {
      sp[a] = m[kMP + a];
      sq[a] = m[kMQ + a];
    }
    for (int k = 0; k < 9; ++k) {
      Spp[k] = m[kMPP + k];
      Sqq[k] = m[kMQQ + k];
      Spq[k] = m[kMPQ + k];
    }
    ns = n;
    // E = w [tr Spp + tr Sqq + n |t|^2 + 2 t^T R sp - 2 t^T sq - 2 sum_cd R_cd Spq[d][c]]
    double Rsp[3];
    for (int a = 0; a < 3; ++a) Rsp[a] = R[3 * a] * sp[0] + R[3 * a + 1] * sp[1] + R[3 * a + 2] * sp[2];
    double qRp = 0.0;
    for (int c2 = 0; c2 < 3; ++c2)
      for (int d2 = 0; d2 < 3; ++d2) qRp += R[3 * c2 + d2] * Spq[3 * d2 + c2];
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double tRsp = t[0] * Rsp[0] + t[1] * Rsp[1] + t[2] * Rsp[2];
    double tsq = t[0] * sq[0] + t[1] * sq[1] + t[2] * sq[2];
    Es = w_sparse * ((Spp[0] + Spp[4] + Spp[8]) + (Sqq[0] + Sqq[4] + Sqq[8]) + n * tt + 2.0 * tRsp - 2.0 * tsq -
                     2.0 * qRp);
  }
  if (jac) {
    const double w = w_sparse;
    // H_jj
    {
      double S[9];
      skew(sq, S);
      double trq = Sqq[0] + Sqq[4] + Sqq[8];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double top = (a == b ? trq : 0.0) - Sqq[3 * a + b];
          out[kEHjj + 6 * a + b] = Hjj_d[6 * a + b] + w * top;
          out[kEHjj + 6 * a + (b + 3)] = Hjj_d[6 * a + b + 3] + w * S[3 * a + b];
          out[kEHjj + 6 * (a + 3) + b] = Hjj_d[6 * (a + 3) + b] - w * S[3 * a + b];
          out[kEHjj + 6 * (a + 3) + (b + 3)] = Hjj_d[6 * (a + 3) + b + 3] + (a == b ? w * n : 0.0);
        }
    }
    // H_ii sparse part
    double Hii[36];
    {
      double S[9];
      skew(sp, S);
      double trp = Spp[0] + Spp[4] + Spp[8];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          Hii[6 * a + b] = w * ((a == b ? trp : 0.0) - Spp[3 * a + b]);
          Hii[6 * a + b + 3] = w * S[3 * a + b];
          Hii[6 * (a + 3) + b] = -w * S[3 * a + b];
          Hii[6 * (a + 3) + b + 3] = (a == b ? w * n : 0.0);
        }
    }
    // Ad(T_ji) = [[R, 0], [[t]x R, R]];  Y = Ad^T Hjj_d;  H_ii += Y Ad;  H_ij = -Y (+ sparse)
    double TR[9];
    {
      double Tx[9];
      skew(t, Tx);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) TR[3 * a + b] = Tx[3 * a] * R[b] + Tx[3 * a + 1] * R[3 + b] + Tx[3 * a + 2] * R[6 + b];
    }
    auto ad = [&](int r, int c) -> double {
      if (r < 3) return c < 3 ? R[3 * r + c] : 0.0;
      return c < 3 ? TR[3 * (r - 3) + c] : R[3 * (r - 3) + (c - 3)];
    };
    double Y[36];
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) {
        double v = 0.0;
        for (int k = 0; k < 6; ++k) v += ad(k, a) * Hjj_d[6 * k + b];
        Y[6 * a + b] = v;
      }
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) {
        double v = 0.0;
        for (int k = 0; k < 6; ++k) v += Y[6 * a + k] * ad(k, b);
        Hii[6 * a + b] += v;
      }
    // symmetrise: both triangles from the same sums
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b) {
        double v = 0.5 * (Hii[6 * a + b] + Hii[6 * b + a]);
        Hii[6 * a + b] = v;
        Hii[6 * b + a] = v;
      }
    for (int k = 0; k < 36; ++k) out[kEHii + k] = Hii[k];
    // H_ij: sparse = -sum A_p^T R^T A_q = [[sum [p]x R^T [q]x, -[sp]x R^T], [R^T [sq]x, -n R^T]]
    double Hij[36];
    {
      double Rt[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Rt[3 * a + b] = R[3 * b + a];
      double Sp[9], Sq[9];
      skew(sp, Sp);
      skew(sq, Sq);
      for (int r = 0; r < 3; ++r)
        for (int c2 = 0; c2 < 3; ++c2) {
          // sum_k [p_k]x Rt [q_k]x = sum eps(r,k,m) eps(l,c,n) Rt[k][l] Spq[m][n]
          double tl = 0.0;
          for (int k = 0; k < 3; ++k)
            for (int m = 0; m < 3; ++m) {
              int e1 = eps3(r, k, m);
              if (!e1) continue;
              for (int l = 0; l < 3; ++l)
                for (int nn = 0; nn < 3; ++nn) {
                  int e2 = eps3(l, c2, nn);
                  if (!e2) continue;
                  tl += (double)(e1 * e2) * Rt[3 * k + l] * Spq[3 * m + nn];
                }
            }
          double tr = 0.0, bl = 0.0;
          for (int k = 0; k < 3; ++k) {
            tr -= Sp[3 * r + k] * Rt[3 * k + c2];
            bl += Rt[3 * r + k] * Sq[3 * k + c2];
          }
          Hij[6 * r + c2] = w * tl;
          Hij[6 * r + c2 + 3] = w * tr;
          Hij[6 * (r + 3) + c2] = w * bl;
          Hij[6 * (r + 3) + c2 + 3] = -w * n * Rt[3 * r + c2];
        }
    }
    for (int k = 0; k < 36; ++k) {
      double v = Hij[k] - Y[k];
      out[kEHij + k] = v;
      hij_store[(size_t)e * 36 + k] = (T)v;
    }
    // gradients.  g_i sparse = w [sp x (R^T t) - sum p x (R^T q); sp + n R^T t - R^T sq]
    //             g_j sparse = -w [sum q x (R p) + sq x t; R sp + n t - sq]
    double Rtt[3], Rtsq[3], Rsp[3];
    for (int a = 0; a < 3; ++a) {
      Rtt[a] = R[a] * t[0] + R[3 + a] * t[1] + R[6 + a] * t[2];
      Rtsq[a] = R[a] * sq[0] + R[3 + a] * sq[1] + R[6 + a] * sq[2];
      Rsp[a] = R[3 * a] * sp[0] + R[3 * a + 1] * sp[1] + R[3 * a + 2] * sp[2];
    }
    double gi[6], gj[6];
    for (int a = 0; a < 3; ++a) {
      int b = (a + 1) % 3, c2 = (a + 2) % 3;
      double sx = sp[b] * Rtt[c2] - sp[c2] * Rtt[b];
      double pxRq = 0.0, qxRp = 0.0;
      for (int bb = 0; bb < 3; ++bb)
        for (int cc = 0; cc < 3; ++cc) {
          int ep = eps3(a, bb, cc);
          if (!ep) continue;
          for (int dd = 0; dd < 3; ++dd) {
            pxRq += ep * R[3 * dd + cc] * Spq[3 * bb + dd];   // sum p_b (R^T q)_c
            qxRp += ep * R[3 * cc + dd] * Spq[3 * dd + bb];   // sum q_b (R p)_c
          }
        }
      double sqxt = sq[b] * t[c2] - sq[c2] * t[b];
      gi[a] = w * (sx - pxRq);
      gi[a + 3] = w * (sp[a] + n * Rtt[a] - Rtsq[a]);
      gj[a] = -w * (qxRp + sqxt);
      gj[a + 3] = -w * (Rsp[a] + n * t[a] - sq[a]);
    }
    // dense: g_j += gj_d, g_i -= Ad^T gj_d
    for (int a = 0; a < 6; ++a) {
      double v = 0.0;
      for (int k = 0; k < 6; ++k) v += ad(k, a) * gj_d[k];
      out[kEGi + a] = gi[a] - v;
      out[kEGj + a] = gj[a] + gj_d[a];
    }
  }
  out[kEEs] = Es;
  out[kEEg] = Eg;
  out[kEEp] = Ep;
  out[kENs] = ns;
  out[kENg] = ng;
  out[kENp] = np;
}

// One wavefront per free frame: diagonal block and gradient from the incident edges
// (lower-index edges first, in edge order, then upper-index edges in edge order).
template <class T>
__global__ void __launch_bounds__(64) k_assemble(const double* __restrict__ eb, const long long* __restrict__ iptr,
                                                 const long long* __restrict__ jptr,
                                                 const long long* __restrict__ ej_sorted,
                                                 const int* __restrict__ frame_of_var, long long nfree,
                                                 T* __restrict__ diag, T* __restrict__ minv, T* __restrict__ rhs,
                                                 int* __restrict__ flags) {
  long long v = blockIdx.x;
  if (v >= nfree) return;
  const int lane = threadIdx.x;
  const int f = frame_of_var[v];
  __shared__ double blk[48];
  if (lane < 42) {
    const int offH = lane < 36 ? kEHii + lane : kEGi + (lane - 36);
    const int offHj = lane < 36 ? kEHjj + lane : kEGj + (lane - 36);
    double s = 0.0;
    for (long long k = iptr[f]; k < iptr[f + 1]; ++k) s += eb[(size_t)k * kEdgeWords + offH];
    for (long long k = jptr[f]; k < jptr[f + 1]; ++k) s += eb[(size_t)ej_sorted[k] * kEdgeWords + offHj];
    blk[lane] = s;
  }
  __syncthreads();
  if (lane < 36) diag[(size_t)v * 36 + lane] = (T)blk[lane];
  if (lane < 6) rhs[(size_t)v * 6 + lane] = (T)(-blk[36 + lane]);
  if (lane == 0) {
    double A[36];
    for (int k = 0; k < 36; ++k) A[k] = blk[k];
    bool ok = spd_inverse6(A);
    if (!ok) {
      raise_flag(flags, kFlagNotPD);
      for (int k = 0; k < 36; ++k) A[k] = (k % 7 == 0) ? 1.0 : 0.0;
    }
    for (int k = 0; k < 36; ++k) minv[(size_t)v * 36 + k] = (T)A[k];
  }
}

// Deterministic block reduction of one double per thread (blockDim.x = 1024).
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) sh[tid] += sh[tid + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Single-workgroup PCG over all free frames (1024 threads), then the pose update.
template <class T>
__global__ void __launch_bounds__(1024) k_pcg_single(
    long long nfree, int F, int iters, const T* __restrict__ diag, const T* __restrict__ minv,
    const T* __restrict__ rhs, const T* __restrict__ hij, const int* __restrict__ eij,
    const long long* __restrict__ iptr, const long long* __restrict__ jptr, const long long* __restrict__ ej_sorted,
    const int* __restrict__ frame_of_var, const int* __restrict__ var_of, T* __restrict__ x, T* __restrict__ r,
    T* __restrict__ z, T* __restrict__ p, T* __restrict__ Ap, double* __restrict__ delta_out,
    double* __restrict__ poses, int update, double* __restrict__ stats, const int* __restrict__ flags) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  const long long n = 6 * nfree;
  const bool bad = flags[0] & kFlagNotPD;
  // x = 0, r = b, z = M^-1 r, p = z
  for (long long o = tid; o < n; o += 1024) {
    x[o] = (T)0;
    r[o] = rhs[o];
  }
  __syncthreads();
  double part = 0.0;
  for (long long o = tid; o < n; o += 1024) {
    long long v = o / 6;
    int a = (int)(o % 6);
    double s = 0.0;
    for (int b = 0; b < 6; ++b) s += (double)minv[v * 36 + 6 * a + b] * (double)r[6 * v + b];
    z[o] = (T)s;
    p[o] = (T)s;
    part += (double)r[o] * (double)(T)s;
  }
  double rz = block_sum(part, sh);
  const double rz0 = rz;
  int done = 0;
  for (int it = 0; it < iters && !bad; ++it) {
    if (rz <= 1e-30) break;
    part = 0.0;
    for (long long o = tid; o < n; o += 1024) {
      long long v = o / 6;
      int a = (int)(o % 6);
      int f = frame_of_var[v];
      T s = (T)0;
      for (int b = 0; b < 6; ++b) s += diag[v * 36 + 6 * a + b] * p[6 * v + b];
      for (long long k = iptr[f]; k < iptr[f + 1]; ++k) {
        int w = var_of[eij[2 * k + 1]];
        if (w < 0) continue;
        const T* B = hij + (size_t)k * 36 + 6 * a;
        for (int b = 0; b < 6; ++b) s += B[b] * p[6 * (long long)w + b];
      }
      for (long long k = jptr[f]; k < jptr[f + 1]; ++k) {
        long long e = ej_sorted[k];
        int w = var_of[eij[2 * e]];
        if (w < 0) continue;
        const T* B = hij + (size_t)e * 36 + a;
        for (int b = 0; b < 6; ++b) s += B[6 * b] * p[6 * (long long)w + b];
      }
      Ap[o] = s;
      part += (double)p[o] * (double)s;
    }
    double pAp = block_sum(part, sh);
    double alpha = rz / pAp;
    for (long long o = tid; o < n; o += 1024) {
      x[o] = (T)((double)x[o] + alpha * (double)p[o]);
      r[o] = (T)((double)r[o] - alpha * (double)Ap[o]);
    }
    __syncthreads();
    part = 0.0;
    for (long long o = tid; o < n; o += 1024) {
      long long v = o / 6;
      int a = (int)(o % 6);
      double s = 0.0;
      for (int b = 0; b < 6; ++b) s += (double)minv[v * 36 + 6 * a + b] * (double)r[6 * v + b];
      z[o] = (T)s;
      part += (double)r[o] * (double)(T)s;
    }
    double rz_new = block_sum(part, sh);
    ++done;
    double beta = rz_new / rz;
    rz = rz_new;
    for (long long o = tid; o < n; o += 1024) p[o] = (T)((double)z[o] + beta * (double)p[o]);
    __syncthreads();
  }
  if (delta_out) {
    for (long long o = tid; o < 6LL * F; o += 1024) {
      int f = (int)(o / 6);
      int w = var_of[f];
      delta_out[o] = (w >= 0 && !bad) ? (double)x[6LL * w + (o % 6)] : 0.0;
    }
  }
  if (update && !bad) {
    for (long long v = tid; v < nfree; v += 1024) {
      int f = frame_of_var[v];
      double xi[6];
      for (int k = 0; k < 6; ++k) xi[k] = (double)x[6 * v + k];
      double dR[9], dt[3];
      exp_se3(xi, dR, dt);
      double* T4 = poses + (size_t)f * 16;
      double Rn[9], tn[3];
      for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
          Rn[3 * a + b] = T4[4 * a] * dR[b] + T4[4 * a + 1] * dR[3 + b] + T4[4 * a + 2] * dR[6 + b];
        tn[a] = T4[4 * a] * dt[0] + T4[4 * a + 1] * dt[1] + T4[4 * a + 2] * dt[2] + T4[4 * a + 3];
      }
      for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) T4[4 * a + b] = Rn[3 * a + b];
        T4[4 * a + 3] = tn[a];
      }
    }
  }
  if (tid == 0 && stats) {
    stats[0] = rz0;
    stats[1] = rz;
    stats[2] = done;
  }
}

// Energy and counts over all edges, fixed order (one workgroup of 1024).
__global__ void __launch_bounds__(1024) k_energy(const double* __restrict__ eb, long long E, double* __restrict__ dst) {
  __shared__ double sh[1024];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long e = threadIdx.x; e < E; e += 1024)
    for (int k = 0; k < 6; ++k) acc[k] += eb[(size_t)e * kEdgeWords + kEEs + k];
  double tot[6];
  for (int k = 0; k < 6; ++k) tot[k] = block_sum(acc[k], sh);
  if (threadIdx.x == 0) {
    dst[0] = tot[0] + tot[1] + tot[2];
    dst[1] = tot[0];
    dst[2] = tot[1];
    dst[3] = tot[2];
    dst[4] = tot[3];
    dst[5] = tot[4];
    dst[6] = tot[5];
    dst[7] = 0.0;
  }
}

// Full H and g for export: every frame's diagonal block and gradient, every edge's
// off-diagonal block and its transpose.
__global__ void k_export_diag(const double* __restrict__ eb, const long long* __restrict__ iptr,
                              const long long* __restrict__ jptr, const long long* __restrict__ ej_sorted, int F,
                              double* __restrict__ H, double* __restrict__ g) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F * 42) return;
  int f = (int)(t / 42), l = (int)(t % 42);
  const int offH = l < 36 ? kEHii + l : kEGi + (l - 36);
  const int offHj = l < 36 ? kEHjj + l : kEGj + (l - 36);
  double s = 0.0;
  for (long long k = iptr[f]; k < iptr[f + 1]; ++k) s += eb[(size_t)k * kEdgeWords + offH];
  for (long long k = jptr[f]; k < jptr[f + 1]; ++k) s += eb[(size_t)ej_sorted[k] * kEdgeWords + offHj];
  const long long N = 6LL * F;
  if (l < 36) {
    if (H) H[(6LL * f + l / 6) * N + 6LL * f + l % 6] = s;
  } else if (g) {
    g[6LL * f + (l - 36)] = s;
  }
}

__global__ void k_export_off(const double* __restrict__ eb, const int* __restrict__ eij, long long E, int F,
                             double* __restrict__ H) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * 36) return;
  long long e = t / 36;
  int l = (int)(t % 36), a = l / 6, b = l % 6;
  int i = eij[2 * e], j = eij[2 * e + 1];
  const long long N = 6LL * F;
  double v = eb[(size_t)e * kEdgeWords + kEHij + l];
  H[(6LL * i + a) * N + 6LL * j + b] = v;
  H[(6LL * j + b) * N + 6LL * i + a] = v;
}

}  // namespace

void launch_edge_blocks(Context& c, const double* poses, const bf_params& prm, bool with_jacobians) {
  const long long E = c.shape.E;
  if (E == 0) return;
  unsigned grid = (unsigned)((E + 63) / 64);
  if (c.pcg_storage == 1)
    hipLaunchKernelGGL(k_edge_blocks<double>, dim3(grid), dim3(64), 0, c.stream, c.edge_ij.as<int>(), E,
                       c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                       c.records.as<double>(), poses, prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                       c.eblocks.as<double>(), c.hij64.as<double>());
  else
    hipLaunchKernelGGL(k_edge_blocks<float>, dim3(grid), dim3(64), 0, c.stream, c.edge_ij.as<int>(), E,
                       c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                       c.records.as<double>(), poses, prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                       c.eblocks.as<double>(), c.hij32.as<float>());
}

void launch_assemble(Context& c) {
  const long long nf = c.shape.nfree;
  if (nf == 0) return;
  if (c.pcg_storage == 1)
    hipLaunchKernelGGL(k_assemble<double>, dim3((unsigned)nf), dim3(64), 0, c.stream, c.eblocks.as<double>(),
                       c.iptr.as<long long>(), c.jptr.as<long long>(), c.ej_sorted.as<long long>(),
                       c.frame_of_var.as<int>(), nf, c.diag64.as<double>(), c.minv64.as<double>(),
                       c.rhs.as<double>(), c.flags.as<int>());
  else
    hipLaunchKernelGGL(k_assemble<float>, dim3((unsigned)nf), dim3(64), 0, c.stream, c.eblocks.as<double>(),
                       c.iptr.as<long long>(), c.jptr.as<long long>(), c.ej_sorted.as<long long>(),
                       c.frame_of_var.as<int>(), nf, c.diag32.as<float>(), c.minv32.as<float>(),
                       c.rhs.as<float>(), c.flags.as<int>());
}

void launch_pcg(Context& c, int iters, double* delta_out, double* poses_inout, double* stats, bool update_poses) {
  const long long nf = c.shape.nfree;
  const long long n = 6 * nf;
  if (c.pcg_storage == 1) {
    double* v = c.pcg_vec.as<double>();
    hipLaunchKernelGGL(k_pcg_single<double>, dim3(1), dim3(1024), 0, c.stream, nf, c.shape.F, iters,
                       c.diag64.as<double>(), c.minv64.as<double>(), c.rhs.as<double>(), c.hij64.as<double>(),
                       c.edge_ij.as<int>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                       c.ej_sorted.as<long long>(), c.frame_of_var.as<int>(), c.var_of.as<int>(), v, v + n, v + 2 * n,
                       v + 3 * n, v + 4 * n, delta_out, poses_inout, update_poses ? 1 : 0, stats, c.flags.as<int>());
  } else {
    float* v = c.pcg_vec.as<float>();
    hipLaunchKernelGGL(k_pcg_single<float>, dim3(1), dim3(1024), 0, c.stream, nf, c.shape.F, iters,
                       c.diag32.as<float>(), c.minv32.as<float>(), c.rhs.as<float>(), c.hij32.as<float>(),
                       c.edge_ij.as<int>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                       c.ej_sorted.as<long long>(), c.frame_of_var.as<int>(), c.var_of.as<int>(), v, v + n, v + 2 * n,
                       v + 3 * n, v + 4 * n, delta_out, poses_inout, update_poses ? 1 : 0, stats, c.flags.as<int>());
  }
}

void launch_energy(Context& c, double* dst8) {
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, c.stream, c.eblocks.as<double>(), (long long)c.shape.E, dst8);
}

void launch_export_dense(Context& c, double* H, double* g) {
  const int F = c.shape.F;
  const long long N = 6LL * F;
  if (H) check_hip(hipMemsetAsync(H, 0, sizeof(double) * N * N, c.stream), "memset H");
  long long nt = (long long)F * 42;
  hipLaunchKernelGGL(k_export_diag, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c.stream,
                     c.eblocks.as<double>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                     c.ej_sorted.as<long long>(), F, H, g);
  if (H && c.shape.E > 0) {
    long long ne = c.shape.E * 36;
    hipLaunchKernelGGL(k_export_off, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c.stream,
                       c.eblocks.as<double>(), c.edge_ij.as<int>(), (long long)c.shape.E, F, H);
  }
}

}  // namespace bf
