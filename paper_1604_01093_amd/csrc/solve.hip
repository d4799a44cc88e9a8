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
#include <algorithm>
#include <atomic>
#include <mutex>

#include <type_traits>

#include "internal.h"

namespace bf {

namespace {

// Edge blocks, one lane per edge (used when there are enough edges to fill the
// GPU one lane each; the wavefront-per-edge kernel below serves fewer edges):
// the same quantities, each lane reading its edge's records and moments and
// forming the 6x6 products in registers.
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
__global__ void __launch_bounds__(64) k_edge_blocks_lane(const int* __restrict__ eij, long long E,
                                                    const long long* __restrict__ edense,
                                                    const long long* __restrict__ esparse,
                                                    const double* __restrict__ mom, const double* __restrict__ rec,
                                                    long long P, int bidir, int tiles,
                                                    const double* __restrict__ poses, double w_sparse, int jac,
                                                    double* __restrict__ eb, T* __restrict__ hij_store,
                                                    double* __restrict__ ediag_dense) {
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
  // a pair job's record is the sum of its `tiles` partial records, in tile order
  if (d >= 0) {
    for (int tl = 0; tl < tiles; ++tl) {
      const double* r = rec + ((size_t)d * tiles + tl) * kRecWords;
      if (jac) {
        int k = 0;
        for (int a = 0; a < 6; ++a)
          for (int b = a; b < 6; ++b) {
            Hjj_d[6 * a + b] += r[k];
            ++k;
          }
        for (int a = 0; a < 6; ++a) gj_d[a] += r[kRecG + a];
      }
      Eg += r[kRecEg];
      Ep += r[kRecEp];
      ng += r[kRecNg];
      np += r[kRecNp];
    }
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < a; ++b) Hjj_d[6 * a + b] = Hjj_d[6 * b + a];
  }
  // the reverse job (j -> i, record P + d): its block is the one of frame i
  double Hii_r[36], gi_r[6];
  const bool has_rev = bidir && d >= 0;
  for (int k = 0; k < 36; ++k) Hii_r[k] = 0.0;
  for (int k = 0; k < 6; ++k) gi_r[k] = 0.0;
  if (has_rev) {
    for (int tl = 0; tl < tiles; ++tl) {
      const double* r = rec + ((size_t)(P + d) * tiles + tl) * kRecWords;
      if (jac) {
        int k = 0;
        for (int a = 0; a < 6; ++a)
          for (int b = a; b < 6; ++b) {
            Hii_r[6 * a + b] += r[k];
            ++k;
          }
        for (int a = 0; a < 6; ++a) gi_r[a] += r[kRecG + a];
      }
      Eg += r[kRecEg];
      Ep += r[kRecEp];
      ng += r[kRecNg];
      np += r[kRecNp];
    }
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < a; ++b) Hii_r[6 * a + b] = Hii_r[6 * b + a];
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
    // reverse job: Ad(T_ij) = [[R^T, 0], [[t2]x R^T, R^T]] with t2 = -R^T t;
    // H_jj += Ad2^T Hii_r Ad2 (symmetrised), H_ij -= Hii_r Ad2, g_j -= Ad2^T gi_r
    double Y2[36], R2[9], TR2[9];
    if (has_rev) {
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R2[3 * a + b] = R[3 * b + a];
      double t2[3], Tx2[9];
      for (int a = 0; a < 3; ++a) t2[a] = -(R2[3 * a] * t[0] + R2[3 * a + 1] * t[1] + R2[3 * a + 2] * t[2]);
      skew(t2, Tx2);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          TR2[3 * a + b] = Tx2[3 * a] * R2[b] + Tx2[3 * a + 1] * R2[3 + b] + Tx2[3 * a + 2] * R2[6 + b];
    }
    auto ad2 = [&](int r, int c) -> double {
      if (r < 3) return c < 3 ? R2[3 * r + c] : 0.0;
      return c < 3 ? TR2[3 * (r - 3) + c] : R2[3 * (r - 3) + (c - 3)];
    };
    double Z2[36];
    if (has_rev) {
      // Y2 = Hii_r Ad2
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
          double v = 0.0;
          for (int k = 0; k < 6; ++k) v += Hii_r[6 * a + k] * ad2(k, b);
          Y2[6 * a + b] = v;
        }
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
          double v = 0.0;
          for (int k = 0; k < 6; ++k) v += ad2(k, a) * Y2[6 * k + b];
          Z2[6 * a + b] = v;
        }
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) out[kEHjj + 6 * a + b] += 0.5 * (Z2[6 * a + b] + Z2[6 * b + a]);
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
        Hii[6 * a + b] += v + Hii_r[6 * a + b];
        // the dense term's part alone (matrix-free sparse mode: the product takes the
        // sparse part per correspondence)
        if (ediag_dense) ediag_dense[(size_t)e * 72 + 6 * a + b] = v + Hii_r[6 * a + b];
      }
    if (ediag_dense) {
      double* dd = ediag_dense + (size_t)e * 72;
      for (int a = 0; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b) {
          const double v = 0.5 * (dd[6 * a + b] + dd[6 * b + a]);
          dd[6 * a + b] = v;
          dd[6 * b + a] = v;
        }
      // H_jj of the dense term: the forward job's block and the reverse job's, as above
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
          double v = Hjj_d[6 * a + b];
          if (has_rev) v += 0.5 * (Z2[6 * a + b] + Z2[6 * b + a]);
          dd[36 + 6 * a + b] = v;
        }
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
      const double vd = -Y[k] - (has_rev ? Y2[k] : 0.0);
      double v = Hij[k] - Y[k] - (has_rev ? Y2[k] : 0.0);
      out[kEHij + k] = v;
      // the PCG's copy: the dense term's block alone in matrix-free sparse mode
      hij_store[(size_t)e * 36 + k] = (T)(ediag_dense ? vd : v);
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
      double v = 0.0, v2 = 0.0;
      for (int k = 0; k < 6; ++k) v += ad(k, a) * gj_d[k];
      if (has_rev)
        for (int k = 0; k < 6; ++k) v2 += ad2(k, a) * gi_r[k];
      out[kEGi + a] = gi[a] - v + gi_r[a];
      out[kEGj + a] = gj[a] + gj_d[a] - v2;
    }
  }
  out[kEEs] = Es;
  out[kEEg] = Eg;
  out[kEEp] = Ep;
  out[kENs] = ns;
  out[kENg] = ng;
  out[kENp] = np;
}

// Edge blocks: one wavefront per edge, four edges per workgroup.  The lanes load
// the pair job's records (tiles summed in order) and the sparse moments into LDS;
// then every 6x6 product and output entry is one lane's (entry (a, b) = lane
// 6a + b), with wavefront barriers between the stages.
constexpr int kEdgeThreads = 256;
// Above this many edges the lane-per-edge kernel is used: at 224,736 edges it took
// 121 us per launch against 268 us for a wavefront per edge, at 3789 edges 13.3 us
// against 10.0 us.
constexpr long long kEdgeLaneMin = 32768;
constexpr int kEdgeScratch = 32 + 32 + 36 * 10 + 24;  // doubles of LDS per wavefront

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// position of (a, b), a <= b, in a record's packed upper triangle (row by row)
__device__ __forceinline__ int packed_upper(int a, int b) { return a * (11 - a) / 2 + b; }

// entry (r, c) of the cross-product matrix [v]x
__device__ __forceinline__ double skew_at(const double* v, int r, int c) {
  if (r == c) return 0.0;
  const int k = 3 - r - c;  // the third index
  const double x = v[k];
  // [v]x = [[0, -v2, v1], [v2, 0, -v0], [-v1, v0, 0]]: +v_k where (r, c, k) is cyclic
  return ((c - r + 3) % 3 == 1) ? -x : x;
}

template <class T>
__global__ void __launch_bounds__(kEdgeThreads) k_edge_blocks(const int* __restrict__ eij, long long E,
                                                              const long long* __restrict__ edense,
                                                              const long long* __restrict__ esparse,
                                                              const double* __restrict__ mom,
                                                              const double* __restrict__ rec, long long P, int bidir,
                                                              int tiles, const double* __restrict__ poses,
                                                              double w_sparse, int jac, double* __restrict__ eb,
                                                              T* __restrict__ hij_store,
                                                              double* __restrict__ ediag_dense) {
  __shared__ double smem[kEdgeThreads / 64][kEdgeScratch];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e = (long long)blockIdx.x * (kEdgeThreads / 64) + wave;
  if (e >= E) return;  // whole wavefronts only: nothing below synchronises the workgroup
  double* Fw = smem[wave];     // forward job record, tiles summed [32]
  double* Rw = Fw + 32;        // reverse job record [32]
  double* Mw = Rw + 32;        // sparse moments [36]
  double* Hd = Mw + 36;        // forward job's frame-j block H_jj (full 6x6)
  double* Hr = Hd + 36;        // reverse job's frame-i block
  double* AD = Hr + 36;        // Ad(T_ji)
  double* AD2 = AD + 36;       // Ad(T_ij)
  double* Yw = AD2 + 36;       // Ad^T H_jj
  double* Y2w = Yw + 36;       // H_ii_r Ad2
  double* Pw = Y2w + 36;       // H_ii before symmetrising
  double* Dw = Pw + 36;        // the dense term's H_ii before symmetrising
  double* Zw = Dw + 36;        // Ad2^T H_ii_r Ad2
  double* Gw = Zw + 36;        // R (row-major) [9], t [3], R^T [9], t2 = -R^T t [3]
  const int i = eij[2 * e], j = eij[2 * e + 1];
  const long long s = esparse[e];
  const long long d = edense[e];
  const bool has_rev = bidir && d >= 0;
  double R[9], t[3];
  relative_pose_nc(poses + (size_t)i * 16, poses + (size_t)j * 16, R, t);
  double* out = eb + (size_t)e * kEdgeWords;

  // stage 1: records (a pair job's record is the sum of its `tiles` partial
  // records, in tile order) and moments
  if (lane < 32) {
    double v = 0.0;
    if (d >= 0)
      for (int tl = 0; tl < tiles; ++tl) v += rec[((size_t)d * tiles + tl) * kRecWords + lane];
    Fw[lane] = v;
  } else {
    double v = 0.0;
    if (has_rev)
      for (int tl = 0; tl < tiles; ++tl) v += rec[((size_t)(P + d) * tiles + tl) * kRecWords + lane - 32];
    Rw[lane - 32] = v;
  }
  if (lane < 36) Mw[lane] = s >= 0 ? mom[(size_t)s * kMomWords + lane] : 0.0;
  if (lane == 0) {
    for (int q = 0; q < 9; ++q) Gw[q] = R[q];
    for (int q = 0; q < 3; ++q) Gw[9 + q] = t[q];
    for (int q = 0; q < 3; ++q)
      for (int r2 = 0; r2 < 3; ++r2) Gw[12 + 3 * q + r2] = R[3 * r2 + q];
    for (int q = 0; q < 3; ++q) Gw[21 + q] = -(R[q] * t[0] + R[3 + q] * t[1] + R[6 + q] * t[2]);
  }
  wave_sync();
  // energies and counts (the forward job's, then the reverse job's; the sparse
  // term's from the moments)
  if (lane == 63) {
    double Es = 0, ns = 0;
    if (s >= 0) {
      const double* m = Mw;
      const double n = m[kMN];
      ns = n;
      // E = w [tr Spp + tr Sqq + n |t|^2 + 2 t^T R sp - 2 t^T sq - 2 sum_cd R_cd Spq[d][c]]
      double Rsp[3];
      for (int a2 = 0; a2 < 3; ++a2)
        Rsp[a2] = R[3 * a2] * m[kMP] + R[3 * a2 + 1] * m[kMP + 1] + R[3 * a2 + 2] * m[kMP + 2];
      double qRp = 0.0;
      for (int c2 = 0; c2 < 3; ++c2)
        for (int d2 = 0; d2 < 3; ++d2) qRp += R[3 * c2 + d2] * m[kMPQ + 3 * d2 + c2];
      const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
      const double tRsp = t[0] * Rsp[0] + t[1] * Rsp[1] + t[2] * Rsp[2];
      const double tsq = t[0] * m[kMQ] + t[1] * m[kMQ + 1] + t[2] * m[kMQ + 2];
      Es = w_sparse * ((m[kMPP] + m[kMPP + 4] + m[kMPP + 8]) + (m[kMQQ] + m[kMQQ + 4] + m[kMQQ + 8]) + n * tt +
                       2.0 * tRsp - 2.0 * tsq - 2.0 * qRp);
    }
    out[kEEs] = Es;
    out[kEEg] = Fw[kRecEg] + Rw[kRecEg];
    out[kEEp] = Fw[kRecEp] + Rw[kRecEp];
    out[kENs] = ns;
    out[kENg] = Fw[kRecNg] + Rw[kRecNg];
    out[kENp] = Fw[kRecNp] + Rw[kRecNp];
  }
  if (!jac) return;

  const double w = w_sparse;
  const int a = lane / 6, b = lane - 6 * (lane / 6);  // entry of lanes 0..35
  // stage 2: full blocks from the packed records; the two adjoints
  //   Ad(T_ji) = [[R, 0], [[t]x R, R]],  Ad(T_ij) = [[R^T, 0], [[t2]x R^T, R^T]], t2 = -R^T t
  if (lane < 36) {
    const int k = a <= b ? packed_upper(a, b) : packed_upper(b, a);
    Hd[lane] = Fw[k];
    Hr[lane] = Rw[k];
    const double* Rg = Gw;        // R
    const double* tg = Gw + 9;    // t
    const double* R2g = Gw + 12;  // R^T
    const double* t2g = Gw + 21;  // -R^T t
    const int ra = a % 3, cb = b % 3;
    double adv, ad2v;
    if (a < 3) {
      adv = b < 3 ? Rg[3 * ra + cb] : 0.0;
      ad2v = b < 3 ? R2g[3 * ra + cb] : 0.0;
    } else if (b < 3) {
      adv = skew_at(tg, ra, 0) * Rg[cb] + skew_at(tg, ra, 1) * Rg[3 + cb] + skew_at(tg, ra, 2) * Rg[6 + cb];
      ad2v = skew_at(t2g, ra, 0) * R2g[cb] + skew_at(t2g, ra, 1) * R2g[3 + cb] + skew_at(t2g, ra, 2) * R2g[6 + cb];
    } else {
      adv = Rg[3 * ra + cb];
      ad2v = R2g[3 * ra + cb];
    }
    AD[lane] = adv;
    AD2[lane] = ad2v;
  }
  wave_sync();
  // stage 3: Y = Ad^T H_jj, Y2 = H_ii_r Ad2
  if (lane < 36) {
    double v = 0.0;
    for (int k = 0; k < 6; ++k) v += AD[6 * k + a] * Hd[6 * k + b];
    Yw[lane] = v;
    double v2 = 0.0;
    if (has_rev)
      for (int k = 0; k < 6; ++k) v2 += Hr[6 * a + k] * AD2[6 * k + b];
    Y2w[lane] = v2;
  }
  wave_sync();
  // stage 4: the dense term's H_ii = Y Ad + H_ii_r and Z2 = Ad2^T Y2; the sparse
  // H_ii (the moments: H_ii = sum A_p^T A_p with A_p = [-[p]x | I])
  const double n = Mw[kMN];
  if (lane < 36) {
    double v = 0.0;
    for (int k = 0; k < 6; ++k) v += Yw[6 * a + k] * AD[6 * k + b];
    double z = 0.0;
    if (has_rev)
      for (int k = 0; k < 6; ++k) z += AD2[6 * k + a] * Y2w[6 * k + b];
    Zw[lane] = z;
    const double* sp = Mw + kMP;
    const double* Spp = Mw + kMPP;
    const int ra = a % 3, cb = b % 3;
    const double trp = Spp[0] + Spp[4] + Spp[8];
    double hs;
    if (a < 3) hs = b < 3 ? w * ((a == b ? trp : 0.0) - Spp[3 * a + b]) : w * skew_at(sp, ra, cb);
    else hs = b < 3 ? -w * skew_at(sp, ra, cb) : (ra == cb ? w * n : 0.0);
    const double dv = v + Hr[lane];
    Pw[lane] = hs + dv;
    Dw[lane] = dv;
  }
  wave_sync();
  // stage 5: outputs
  if (lane < 36) {
    const int ra = a % 3, cb = b % 3;
    const double* sp = Mw + kMP;
    const double* sq = Mw + kMQ;
    const double* Sqq = Mw + kMQQ;
    const double* Spq = Mw + kMPQ;
    // H_jj: the forward job's block, the sparse part, then the reverse job's lifted
    // block (symmetrised)
    {
      const double trq = Sqq[0] + Sqq[4] + Sqq[8];
      double v;
      if (a < 3)
        v = b < 3 ? Hd[lane] + w * ((a == b ? trq : 0.0) - Sqq[3 * a + b]) : Hd[lane] + w * skew_at(sq, ra, cb);
      else v = b < 3 ? Hd[lane] - w * skew_at(sq, ra, cb) : Hd[lane] + (ra == cb ? w * n : 0.0);
      if (has_rev) v += 0.5 * (Zw[6 * a + b] + Zw[6 * b + a]);
      out[kEHjj + lane] = v;
    }
    // H_ii, symmetrised: both triangles from the same sums
    out[kEHii + lane] = a == b ? Pw[lane] : 0.5 * (Pw[6 * a + b] + Pw[6 * b + a]);
    if (ediag_dense) {
      double* dd = ediag_dense + (size_t)e * 72;
      dd[lane] = a == b ? Dw[lane] : 0.5 * (Dw[6 * a + b] + Dw[6 * b + a]);
      double v = Hd[lane];
      if (has_rev) v += 0.5 * (Zw[6 * a + b] + Zw[6 * b + a]);
      dd[36 + lane] = v;
    }
    // H_ij: sparse = -sum A_p^T R^T A_q = [[sum [p]x R^T [q]x, -[sp]x R^T], [R^T [sq]x, -n R^T]];
    // dense = -Y (and -Y2 for the reverse job)
    double hs;
    {
      const double* Rt = Gw + 12;  // R^T
      const int r = ra, c2 = cb;
      if (a < 3 && b < 3) {
        // sum_k [p_k]x Rt [q_k]x = sum eps(r,k,m) eps(l,c,n) Rt[k][l] Spq[m][n]: four
        // nonzero terms, (k, m) and (l, n) the two orders of the indices other than
        // r and c; summed with k, then l ascending
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;    // eps(r, r1, r2) = +1
        const int c1 = (c2 + 1) % 3, c3 = (c2 + 2) % 3;  // eps(c3, c, c1) = +1
        const int kA = r1 < r2 ? r1 : r2, kB = r1 < r2 ? r2 : r1;
        const int lA = c1 < c3 ? c1 : c3, lB = c1 < c3 ? c3 : c1;
        const double sk[2] = {kA == r1 ? 1.0 : -1.0, kB == r1 ? 1.0 : -1.0};  // eps(r, k, m)
        const double sl[2] = {lA == c3 ? 1.0 : -1.0, lB == c3 ? 1.0 : -1.0};  // eps(l, c, n)
        const int mk[2] = {kA == r1 ? r2 : r1, kB == r1 ? r2 : r1};
        const int nl[2] = {lA == c3 ? c1 : c3, lB == c3 ? c1 : c3};
        const int kk[2] = {kA, kB}, ll[2] = {lA, lB};
        double tl = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int q = 0; q < 2; ++q) tl += (sk[u] * sl[q]) * Rt[3 * kk[u] + ll[q]] * Spq[3 * mk[u] + nl[q]];
        hs = w * tl;
      } else if (a < 3) {
        double tr = 0.0;
        for (int k = 0; k < 3; ++k) tr -= skew_at(sp, r, k) * Rt[3 * k + c2];
        hs = w * tr;
      } else if (b < 3) {
        double bl = 0.0;
        for (int k = 0; k < 3; ++k) bl += Rt[3 * r + k] * skew_at(sq, k, c2);
        hs = w * bl;
      } else {
        hs = -w * n * Rt[3 * r + c2];
      }
    }
    const double y2 = has_rev ? Y2w[lane] : 0.0;
    const double vd = -Yw[lane] - y2;
    const double v = hs - Yw[lane] - y2;
    out[kEHij + lane] = v;
    // the PCG's copy: the dense term's block alone in matrix-free sparse mode
    hij_store[(size_t)e * 36 + lane] = (T)(ediag_dense ? vd : v);
  } else if (lane < 42) {
    // gradients, lane 36 + a2 for a2 = 0..5: g_i sparse = w [sp x (R^T t) - sum p x (R^T q);
    // sp + n R^T t - R^T sq], g_j sparse = -w [sum q x (R p) + sq x t; R sp + n t - sq];
    // dense: g_j += gj_d, g_i -= Ad^T gj_d (and the reverse job's, lifted with Ad2)
    const int a2 = lane - 36;
    const double* sp = Mw + kMP;
    const double* sq = Mw + kMQ;
    const double* Spq = Mw + kMPQ;
    const double* Rg = Gw;      // R
    const double* tg = Gw + 9;  // t
    double gi, gj;
    const int c3 = a2 % 3;
    auto Rtt = [&](int q) { return Rg[q] * tg[0] + Rg[3 + q] * tg[1] + Rg[6 + q] * tg[2]; };
    if (a2 < 3) {
      const int bb0 = (c3 + 1) % 3, cc0 = (c3 + 2) % 3;
      const double sx = sp[bb0] * Rtt(cc0) - sp[cc0] * Rtt(bb0);
      // the two nonzero eps(c3, bb, cc), bb ascending
      const int bA = bb0 < cc0 ? bb0 : cc0, bB = bb0 < cc0 ? cc0 : bb0;
      const int bbs[2] = {bA, bB}, ccs[2] = {bA == bb0 ? cc0 : bb0, bB == bb0 ? cc0 : bb0};
      const double eps[2] = {bA == bb0 ? 1.0 : -1.0, bB == bb0 ? 1.0 : -1.0};
      double pxRq = 0.0, qxRp = 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
          pxRq += eps[u] * Rg[3 * dd + ccs[u]] * Spq[3 * bbs[u] + dd];  // sum p_b (R^T q)_c
          qxRp += eps[u] * Rg[3 * ccs[u] + dd] * Spq[3 * dd + bbs[u]];  // sum q_b (R p)_c
        }
      const double sqxt = sq[bb0] * tg[cc0] - sq[cc0] * tg[bb0];
      gi = w * (sx - pxRq);
      gj = -w * (qxRp + sqxt);
    } else {
      const double Rtsq = Rg[c3] * sq[0] + Rg[3 + c3] * sq[1] + Rg[6 + c3] * sq[2];
      const double Rsp = Rg[3 * c3] * sp[0] + Rg[3 * c3 + 1] * sp[1] + Rg[3 * c3 + 2] * sp[2];
      gi = w * (sp[c3] + n * Rtt(c3) - Rtsq);
      gj = -w * (Rsp + n * tg[c3] - sq[c3]);
    }
    double v = 0.0, v2 = 0.0;
    for (int k = 0; k < 6; ++k) v += AD[6 * k + a2] * Fw[kRecG + k];
    if (has_rev)
      for (int k = 0; k < 6; ++k) v2 += AD2[6 * k + a2] * Rw[kRecG + k];
    out[kEGi + a2] = gi - v + Rw[kRecG + a2];
    out[kEGj + a2] = gj + Fw[kRecG + a2] - v2;
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

// ---------------------------------------------------------------- persistent solve

// Every wait for other workgroups polls at most `spin_limit` times (a launch
// argument; 2^26, about two seconds, unless the caller sets another): a barrier
// that never completes raises an error instead of hanging.
constexpr int kSolveThreads = 1024;          // 16 wavefronts, one matrix row per wavefront at a time
constexpr int kSolveWaves = kSolveThreads / 64;
constexpr int kParts = 8;                     // doubles per workgroup in a grid reduction
constexpr int kMaxSolveGroups = 512;          // workgroups of a cooperative solve

// Data shared between workgroups is written and read with agent-scope relaxed
// atomics (coherent across the XCDs without L2 write-back fences); a barrier
// waits for the wavefront's memory operations to complete, then arrives.
template <class T>
__device__ __forceinline__ T ld_shared(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_shared(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false if the spin limit was hit (then every later barrier is skipped).
__device__ __forceinline__ bool grid_sync(unsigned* ctr, unsigned target, int* flags, int* sh_ok,
                                          unsigned spin_limit) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = *sh_ok;
    if (ok) {
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
          atomicOr(flags, kFlagTimeout);
          ok = 0;
          break;
        }
      }
    }
    *sh_ok = ok;
  }
  __syncthreads();
  return *sh_ok != 0;
}

// Grid-wide sums of K <= kParts doubles per thread, identical in every workgroup
// (fixed trees: lanes, then wavefronts in order, then workgroups in order).
template <int K, int NW = kSolveWaves>
__device__ void grid_sums(double (&v)[K], double* parts, unsigned* bar, unsigned& nbar, int* flags, double* sh,
                          int* sh_ok, unsigned spin_limit, unsigned bar_base = 0u) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = v[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) sh[wave * kParts + k] = t;
  }
  __syncthreads();
  // two partial buffers alternating with the barrier count: a workgroup can only
  // overwrite a buffer after every workgroup has passed the next barrier, i.e.
  // after all of them have read it
  double* pb = parts + (size_t)(nbar & 1) * kParts * kMaxSolveGroups;
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += sh[w * kParts + threadIdx.x];
    st_shared(&pb[blockIdx.x * kParts + threadIdx.x], t);
  }
  ++nbar;
  grid_sync(bar, bar_base + nbar * gridDim.x, flags, sh_ok, spin_limit);
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int g = lane; g < (int)gridDim.x; g += 64) t += ld_shared(&pb[g * kParts + k]);
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
      if (lane == 0) sh[NW * kParts + k] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = sh[NW * kParts + k];
  __syncthreads();
}

// Assembly + block-Jacobi PCG + pose update in one cooperative launch.
//  prologue: each wavefront assembles the diagonal block and gradient of its rows
//            from the incident edges (fixed order), inverts the diagonal block
//            (6x6 Cholesky, FP64), sets x = 0, r = -g, z = M^-1 r, p = z; the
//            energy over all edges is reduced alongside r.z.
//  per iteration, two barriers:
//   A: p_v = z_v + beta p_v(prev) for own rows (into the other p buffer), and
//      Ap_v = D_v p_v + sum_w H_vw p_w with partners' p_w formed on the fly from
//      their z_w and previous p_w;  barrier (p.Ap)
//   B: x += alpha p, r -= alpha Ap, z = M^-1 r for own rows;  barrier (r.z)
//  epilogue: owners write dx and/or apply T_f <- T_f Exp(x_f).
template <class T>
__global__ void __launch_bounds__(kSolveThreads) k_solve_coop(
    long long nfree, int F, long long E, int iters, const double* __restrict__ eb, const T* __restrict__ hij,
    const long long* __restrict__ iptr, const long long* __restrict__ jptr, const long long* __restrict__ ej_sorted,
    const long long* __restrict__ row_ptr, const int2* __restrict__ entries, const int* __restrict__ frame_of_var,
    const int* __restrict__ var_of, T* __restrict__ diag, T* __restrict__ minv, T* __restrict__ x,
    T* __restrict__ r, T* __restrict__ Ap, T* z, T* pb0, T* pb1, double* parts, unsigned* bar,
    double* __restrict__ trace_slot, double* __restrict__ delta_out, double* __restrict__ poses, int update,
    double* __restrict__ stats, int* flags, int precond, unsigned spin_limit) {
  __shared__ double sh[(kSolveWaves + 1) * kParts];
  __shared__ double red[kSolveWaves][64];
  __shared__ double blk[kSolveWaves][48];
  __shared__ int sh_ok;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long gw = (long long)blockIdx.x * kSolveWaves + wave, nw = (long long)gridDim.x * kSolveWaves;
  const int grp = lane / 6, a = lane % 6;
  unsigned nbar = 0;
  if (threadIdx.x == 0) sh_ok = 1;
  __syncthreads();

  // ---- prologue: assembly, preconditioner, initial residual
  double pro[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // r.z, not-PD count, Es, Eg, Ep, ns, ng, np
  for (long long v = gw; v < nfree; v += nw) {
    const int f = frame_of_var[v];
    if (lane < 42) {
      const int offI = lane < 36 ? kEHii + lane : kEGi + (lane - 36);
      const int offJ = lane < 36 ? kEHjj + lane : kEGj + (lane - 36);
      double s0 = 0.0, s1 = 0.0;
      const long long i0 = iptr[f], i1 = iptr[f + 1];
      long long k = i0;
      for (; k + 1 < i1; k += 2) {
        s0 += eb[(size_t)k * kEdgeWords + offI];
        s1 += eb[(size_t)(k + 1) * kEdgeWords + offI];
      }
      if (k < i1) s0 += eb[(size_t)k * kEdgeWords + offI];
      const long long j0 = jptr[f], j1 = jptr[f + 1];
      for (k = j0; k + 1 < j1; k += 2) {
        s0 += eb[(size_t)ej_sorted[k] * kEdgeWords + offJ];
        s1 += eb[(size_t)ej_sorted[k + 1] * kEdgeWords + offJ];
      }
      if (k < j1) s0 += eb[(size_t)ej_sorted[k] * kEdgeWords + offJ];
      blk[wave][lane] = s0 + s1;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 36) diag[v * 36 + lane] = (T)blk[wave][lane];
    if (lane == 0) {
      double A[36];
      for (int q = 0; q < 36; ++q) A[q] = blk[wave][q];
      bool ok = block_jacobi_inverse6(A, precond) >= 0;
      if (!ok) {
        pro[1] += 1.0;
        for (int q = 0; q < 36; ++q) A[q] = (q % 7 == 0) ? 1.0 : 0.0;
      }
      for (int q = 0; q < 36; ++q) minv[v * 36 + q] = (T)A[q];
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (lane < 6) {
      const T rv = (T)(-blk[wave][36 + a]);
      double s = 0.0;
      for (int b = 0; b < 6; ++b) s += (double)minv[v * 36 + 6 * a + b] * (double)(T)(-blk[wave][36 + b]);
      const T zt = (T)s;
      x[6 * v + a] = (T)0;
      r[6 * v + a] = rv;
      st_shared(&z[6 * v + a], zt);
      st_shared(&pb0[6 * v + a], zt);
      pro[0] += (double)rv * (double)zt;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (trace_slot) {
    for (long long e = (long long)blockIdx.x * kSolveThreads + threadIdx.x; e < E;
         e += (long long)gridDim.x * kSolveThreads)
      for (int q = 0; q < 6; ++q) pro[2 + q] += eb[(size_t)e * kEdgeWords + kEEs + q];
  }
  grid_sums<8>(pro, parts, bar, nbar, flags, sh, &sh_ok, spin_limit);
  double rz = pro[0];
  const bool bad = pro[1] > 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (bad && sh_ok) atomicOr(flags, kFlagNotPD);  // the sums are only whole if the barrier completed
    if (trace_slot) {
      trace_slot[0] = pro[2] + pro[3] + pro[4];
      for (int q = 0; q < 6; ++q) trace_slot[1 + q] = pro[2 + q];
      trace_slot[7] = 0.0;
    }
  }
  const double rz0 = rz;
  double beta = 0.0;
  int done = 0;
  for (int k = 0; k < iters && !bad && sh_ok; ++k) {
    if (rz <= 1e-30) break;
    T* pold = (k & 1) ? pb0 : pb1;  // p^{k-1}
    T* pnew = (k & 1) ? pb1 : pb0;  // p^k (for k = 0 it already holds z^0)
    const T tb = (T)beta;
    double part[1] = {0.0};
    for (long long v = gw; v < nfree; v += nw) {
      double acc = 0.0;
      if (grp < 10) {
        if (grp == 0) {
          for (int b = 0; b < 6; ++b) {
            const T pv = (k == 0) ? ld_shared(&pnew[6 * v + b])
                                  : (T)(ld_shared(&z[6 * v + b]) + tb * ld_shared(&pold[6 * v + b]));
            acc += (double)(diag[v * 36 + 6 * a + b] * pv);
          }
        }
        const long long q1 = row_ptr[v + 1];
#pragma unroll 2
        for (long long q = row_ptr[v] + grp; q < q1; q += 10) {
          const int2 en = entries[q];
          const long long w = en.x;
          const T* B = hij + (size_t)(en.y >> 1) * 36;
          const bool tr = en.y & 1;
          T sacc = (T)0;
          for (int b = 0; b < 6; ++b) {
            const T pw = (k == 0) ? ld_shared(&pnew[6 * w + b])
                                  : (T)(ld_shared(&z[6 * w + b]) + tb * ld_shared(&pold[6 * w + b]));
            sacc += (tr ? B[6 * b + a] : B[6 * a + b]) * pw;
          }
          acc += (double)sacc;
        }
      }
      red[wave][lane] = acc;
      __builtin_amdgcn_wave_barrier();
      if (lane < 6) {
        double t = 0.0;
        for (int g = 0; g < 10; ++g) t += red[wave][a + 6 * g];
        const T apv = (T)t;
        Ap[6 * v + a] = apv;
        const T pv = (k == 0) ? ld_shared(&pnew[6 * v + a])
                              : (T)(ld_shared(&z[6 * v + a]) + tb * ld_shared(&pold[6 * v + a]));
        if (k > 0) st_shared(&pnew[6 * v + a], pv);
        part[0] += (double)pv * (double)apv;
      }
      __builtin_amdgcn_wave_barrier();
    }
    grid_sums<1>(part, parts, bar, nbar, flags, sh, &sh_ok, spin_limit);
    const double alpha = rz / part[0];
    double part2[1] = {0.0};
    for (long long v = gw; v < nfree; v += nw) {
      double rv = 0.0;
      if (lane < 6) {
        const T pv = ld_shared(&pnew[6 * v + a]);
        x[6 * v + a] = (T)((double)x[6 * v + a] + alpha * (double)pv);
        rv = (double)(T)((double)r[6 * v + a] - alpha * (double)Ap[6 * v + a]);
        r[6 * v + a] = (T)rv;
      }
      double s = 0.0;
      for (int b = 0; b < 6; ++b) {
        const double rb = __shfl(rv, b);
        if (lane < 6) s += (double)minv[v * 36 + 6 * a + b] * rb;
      }
      if (lane < 6) {
        const T zt = (T)s;
        st_shared(&z[6 * v + a], zt);
        part2[0] += rv * (double)zt;
      }
    }
    grid_sums<1>(part2, parts, bar, nbar, flags, sh, &sh_ok, spin_limit);
    beta = part2[0] / rz;
    rz = part2[0];
    ++done;
  }
  if (delta_out) {
    // owners write their own rows (x never crosses workgroups); frames that are not
    // variables get zeros
    for (long long v = gw; v < nfree; v += nw)
      if (lane < 6) delta_out[6LL * frame_of_var[v] + a] = bad ? 0.0 : (double)x[6 * v + a];
    for (long long o = (long long)blockIdx.x * kSolveThreads + threadIdx.x; o < 6LL * F;
         o += (long long)gridDim.x * kSolveThreads)
      if (var_of[o / 6] < 0) delta_out[o] = 0.0;
  }
  if (update && !bad && sh_ok) {
    for (long long v = gw; v < nfree; v += nw) {
      if (lane != 0) continue;
      const int f = frame_of_var[v];
      double xi[6];
      for (int q = 0; q < 6; ++q) xi[q] = (double)x[6 * v + q];
      double dR[9], dt[3];
      exp_se3(xi, dR, dt);
      double* T4 = poses + (size_t)f * 16;
      double Rn[9], tn[3];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          Rn[3 * i + j] = T4[4 * i] * dR[j] + T4[4 * i + 1] * dR[3 + j] + T4[4 * i + 2] * dR[6 + j];
        tn[i] = T4[4 * i] * dt[0] + T4[4 * i + 1] * dt[1] + T4[4 * i + 2] * dt[2] + T4[4 * i + 3];
      }
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T4[4 * i + j] = Rn[3 * i + j];
        T4[4 * i + 3] = tn[i];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && stats) {
    stats[0] = rz0;
    stats[1] = rz;
    stats[2] = done;
  }
}

// Deterministic sum over a workgroup of NT threads (fixed tree through LDS).
template <int NT>
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum1024(double v, double* red1024) { return block_sum<1024>(v, red1024); }

// Sum over the 64 lanes of a wavefront in FP64, returned to every lane: four DPP
// steps inside each row of 16 lanes (swap neighbours, swap pairs, mirror within
// 8, mirror within 16; each lane adds the same two values in the other order as
// its partner, so all lanes agree), then two exchanges across rows.  Fixed order.
__device__ __forceinline__ double dpp_d(double v, int ctrl_id) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  switch (ctrl_id) {
    case 0:
      lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d(v, 0);
  v += dpp_d(v, 1);
  v += dpp_d(v, 2);
  v += dpp_d(v, 3);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Deterministic workgroup sum: fixed butterfly per wavefront (lane 0's result),
// then the NW wavefront sums in order; every thread returns the same value.
template <int NW>
__device__ __forceinline__ double block_sum_dpp(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_d(v);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NW; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// As block_sum_dpp with one barrier: `sh` must not be written again before every
// thread of the workgroup has passed another barrier (callers alternate slots).
template <int NW>
__device__ __forceinline__ double block_sum_dpp_1(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_d(v);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NW; ++w) t += sh[w];
  return t;
}

// Two sums behind one barrier (same slot rule as block_sum_dpp_1; `sh` holds 2 NW).
// Inside a wavefront the halves exchange first (lanes 0..31 keep a, 32..63 keep b),
// then each half sums its 32 values: one exchange across rows of 16 and the DPP
// steps within a row (every lane of a half ends with its sum).  Fixed order.
template <int NW>
__device__ __forceinline__ void block_sum2_dpp(double a, double b, double* sh, double out[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool hi = (lane & 32) != 0;
  double k = (hi ? b : a) + __shfl_xor(hi ? a : b, 32);
  k += __shfl_xor(k, 16);
  k += dpp_d(k, 0);
  k += dpp_d(k, 1);
  k += dpp_d(k, 2);
  k += dpp_d(k, 3);
  if (lane == 0) sh[wave] = k;
  if (lane == 32) sh[NW + wave] = k;
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int w = 0; w < NW; ++w) {
    ta += sh[w];
    tb += sh[NW + w];
  }
  out[0] = ta;
  out[1] = tb;
}

template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NW; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Six sums over the 64 lanes at once (transpose-reduce, fixed order): values 6
// and 7 are zero; lanes 32 apart exchange half of their eight values and each
// keeps the sum of the half it owns (bit 5 of the lane picks the half), then lanes
// 16 apart halve the four, lanes 8 apart the two, and the eight lanes of each group
// add their one value (DPP: swap neighbours, swap pairs, mirror within 8).  Value
// b ends in lanes 8b .. 8b + 7: seven exchanges instead of six full sums' 36.
__device__ __forceinline__ double wave_sum6_d(const double (&v)[6]) {
  const int lane = threadIdx.x & 63;
  const double x8[8] = {v[0], v[1], v[2], v[3], v[4], v[5], 0.0, 0.0};
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
  double k4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = h5 ? x8[i] : x8[4 + i];
    const double keep = h5 ? x8[4 + i] : x8[i];
    k4[i] = keep + __shfl_xor(send, 32);
  }
  double k2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = h4 ? k4[i] : k4[2 + i];
    const double keep = h4 ? k4[2 + i] : k4[i];
    k2[i] = keep + __shfl_xor(send, 16);
  }
  double k1 = (h3 ? k2[1] : k2[0]) + __shfl_xor(h3 ? k2[0] : k2[1], 8);
  k1 += dpp_d(k1, 0);
  k1 += dpp_d(k1, 1);
  k1 += dpp_d(k1, 2);
  return k1;
}

// y = B p (or B^T p) for one 6x6 block, 16-byte loads, FP32 or FP64 arithmetic.
template <class T>
__device__ __forceinline__ void block_mv(const T* __restrict__ B, const T* pw, bool tr, T y[6]) {
  T m[36];
#pragma unroll
  for (int q = 0; q < 36; ++q) m[q] = B[q];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T s = (T)0;
#pragma unroll
    for (int j = 0; j < 6; ++j) s += (tr ? m[6 * j + i] : m[6 * i + j]) * pw[j];
    y[i] = s;
  }
}

// Assembly + block-Jacobi PCG + pose update, one workgroup of NT threads per
// problem (segment b = blockIdx.x of consecutive frames, variables and edges), no
// grid barriers.  LDS holds x, r, z, p, Ap of the problem (and M^-1 when it fits);
// the off-diagonal blocks are streamed from L2 every iteration, one block per
// lane.  Every sum has a fixed order, so a problem's result does not depend on the
// other problems launched with it.  trace_slot, stats: 8 and 4 words per problem.
template <class T, int NT>
__global__ void __launch_bounds__(NT) k_solve_single(
    const long long* __restrict__ seg_var_ptr, const long long* __restrict__ seg_edge_ptr,
    const int* __restrict__ seg_start, int iters, const double* __restrict__ eb, const T* __restrict__ hij,
    const long long* __restrict__ iptr, const long long* __restrict__ jptr, const long long* __restrict__ ej_sorted,
    const long long* __restrict__ row_ptr, const int2* __restrict__ entries, const int* __restrict__ frame_of_var,
    const int* __restrict__ var_of, T* __restrict__ diag_all, T* __restrict__ minv_all, int minv_in_lds,
    double* __restrict__ trace_all, double* __restrict__ delta_out, double* __restrict__ poses, int update,
    double* __restrict__ stats_all, int* __restrict__ flags, int precond) {
  constexpr int NW = NT / 64;
  extern __shared__ double dyn[];
  __shared__ double red1024[NT];
  __shared__ double blk[NW][48];
  __shared__ int bad_sh;
  const int seg = blockIdx.x;
  const long long v0 = seg_var_ptr[seg];
  const long long nfree = seg_var_ptr[seg + 1] - v0;
  const long long E0 = seg_edge_ptr[seg], E = seg_edge_ptr[seg + 1];
  const int F0 = seg_start[seg], F = seg_start[seg + 1];
  double* trace_slot = trace_all ? trace_all + 8 * seg : nullptr;
  double* stats = stats_all ? stats_all + 4 * seg : nullptr;
  T* diag_g = diag_all + 36 * v0;
  const long long n = 6 * nfree;
  T* x = reinterpret_cast<T*>(dyn);
  T* r = x + n;
  T* z = r + n;
  T* p = z + n;
  T* Ap = p + n;
  T* minv = minv_in_lds ? Ap + n : minv_all + 36 * v0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) bad_sh = 0;
  __syncthreads();

  // prologue: per-row assembly and preconditioner (one wavefront per row)
  for (long long v = wave; v < nfree; v += NW) {
    const int f = frame_of_var[v0 + v];
    if (lane < 42) {
      const int offI = lane < 36 ? kEHii + lane : kEGi + (lane - 36);
      const int offJ = lane < 36 ? kEHjj + lane : kEGj + (lane - 36);
      double s0 = 0.0, s1 = 0.0;
      const long long i0 = iptr[f], i1 = iptr[f + 1];
      long long k = i0;
      for (; k + 1 < i1; k += 2) {
        s0 += eb[(size_t)k * kEdgeWords + offI];
        s1 += eb[(size_t)(k + 1) * kEdgeWords + offI];
      }
      if (k < i1) s0 += eb[(size_t)k * kEdgeWords + offI];
      const long long j0 = jptr[f], j1 = jptr[f + 1];
      for (k = j0; k + 1 < j1; k += 2) {
        s0 += eb[(size_t)ej_sorted[k] * kEdgeWords + offJ];
        s1 += eb[(size_t)ej_sorted[k + 1] * kEdgeWords + offJ];
      }
      if (k < j1) s0 += eb[(size_t)ej_sorted[k] * kEdgeWords + offJ];
      blk[wave][lane] = s0 + s1;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 36) diag_g[v * 36 + lane] = (T)blk[wave][lane];
    if (lane == 0) {
      double A[36];
      for (int q = 0; q < 36; ++q) A[q] = blk[wave][q];
      if (block_jacobi_inverse6(A, precond) < 0) {
        bad_sh = 1;
        for (int q = 0; q < 36; ++q) A[q] = (q % 7 == 0) ? 1.0 : 0.0;
      }
      for (int q = 0; q < 36; ++q) blk[wave][q] = A[q];
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 36) minv[v * 36 + lane] = (T)blk[wave][lane];
    if (lane < 6) {
      x[6 * v + lane] = (T)0;
      r[6 * v + lane] = (T)(-blk[wave][36 + lane]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // energy over the problem's edges
  double en[6] = {0, 0, 0, 0, 0, 0};
  if (trace_slot)
    for (long long e = E0 + tid; e < E; e += NT)
      for (int q = 0; q < 6; ++q) en[q] += eb[(size_t)e * kEdgeWords + kEEs + q];
  __syncthreads();
  if (trace_slot) {
    double tot[6];
    for (int q = 0; q < 6; ++q) tot[q] = block_sum<NT>(en[q], red1024);
    if (tid == 0) {
      trace_slot[0] = tot[0] + tot[1] + tot[2];
      for (int q = 0; q < 6; ++q) trace_slot[1 + q] = tot[q];
      trace_slot[7] = 0.0;
    }
  }
  const bool bad = bad_sh != 0;
  if (bad && tid == 0) atomicOr(flags, kFlagNotPD);
  // z = M^-1 r, p = z
  double part = 0.0;
  for (long long o = tid; o < n; o += NT) {
    const long long v = o / 6;
    const int a = (int)(o % 6);
    double s = 0.0;
    for (int b = 0; b < 6; ++b) s += (double)minv[v * 36 + 6 * a + b] * (double)r[6 * v + b];
    z[o] = (T)s;
    p[o] = (T)s;
    part += (double)r[o] * (double)(T)s;
  }
  double rz = block_sum<NT>(part, red1024);
  const double rz0 = rz;
  int done = 0;
  for (int it = 0; it < iters && !bad; ++it) {
    if (rz <= 1e-30) break;
    // Ap = H p: one wavefront per row, one block per lane
    part = 0.0;
    for (long long v = wave; v < nfree; v += NW) {
      const long long q0 = row_ptr[v0 + v], q1 = row_ptr[v0 + v + 1];
      T acc[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
      for (long long qb = q0; qb < q1; qb += 64) {
        const long long q = qb + lane;
        if (q < q1) {
          const int2 en2 = entries[q];
          T pw[6], y[6];
#pragma unroll
          for (int b = 0; b < 6; ++b) pw[b] = p[6 * ((long long)en2.x - v0) + b];
          block_mv<T>(hij + (size_t)(en2.y >> 1) * 36, pw, en2.y & 1, y);
#pragma unroll
          for (int b = 0; b < 6; ++b) acc[b] += y[b];
        }
      }
      if (lane == 63) {
        T pv[6], y[6];
#pragma unroll
        for (int b = 0; b < 6; ++b) pv[b] = p[6 * v + b];
        block_mv<T>(diag_g + v * 36, pv, false, y);
#pragma unroll
        for (int b = 0; b < 6; ++b) acc[b] += y[b];
      }
      // fixed butterfly over the 64 lanes (lane 0 holds the result)
      double tot[6];
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        double t = (double)acc[b];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        tot[b] = t;
      }
      if (lane == 0) {
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          const T apv = (T)tot[b];
          Ap[6 * v + b] = apv;
          part += (double)p[6 * v + b] * (double)apv;
        }
      }
    }
    // p.Ap and r.z reduce into separate slots, each behind one barrier: a slot is
    // written again only after the barriers that follow its reads
    const double pAp = block_sum_dpp_1<NT / 64>(part, red1024);
    const double alpha = rz / pAp;
    for (long long o = tid; o < n; o += NT) {
      x[o] = (T)((double)x[o] + alpha * (double)p[o]);
      r[o] = (T)((double)r[o] - alpha * (double)Ap[o]);
    }
    __syncthreads();
    part = 0.0;
    for (long long o = tid; o < n; o += NT) {
      const long long v = o / 6;
      const int a = (int)(o % 6);
      double s = 0.0;
      for (int b = 0; b < 6; ++b) s += (double)minv[v * 36 + 6 * a + b] * (double)r[6 * v + b];
      z[o] = (T)s;
      part += (double)r[o] * (double)(T)s;
    }
    const double rz_new = block_sum_dpp_1<NT / 64>(part, red1024 + NT / 64);
    const double beta = rz_new / rz;
    rz = rz_new;
    ++done;
    for (long long o = tid; o < n; o += NT) p[o] = (T)((double)z[o] + beta * (double)p[o]);
    __syncthreads();
  }
  if (delta_out)
    for (long long o = 6LL * F0 + tid; o < 6LL * F; o += NT) {
      const int w = var_of[o / 6];
      delta_out[o] = (w >= 0 && !bad) ? (double)x[6LL * (w - v0) + (o % 6)] : 0.0;
    }
  if (update && !bad)
    for (long long v = tid; v < nfree; v += NT) {
      const int f = frame_of_var[v0 + v];
      double xi[6];
      for (int q = 0; q < 6; ++q) xi[q] = (double)x[6 * v + q];
      double dR[9], dt[3];
      exp_se3(xi, dR, dt);
      double* T4 = poses + (size_t)f * 16;
      double Rn[9], tn[3];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          Rn[3 * i + j] = T4[4 * i] * dR[j] + T4[4 * i + 1] * dR[3 + j] + T4[4 * i + 2] * dR[6 + j];
        tn[i] = T4[4 * i] * dt[0] + T4[4 * i + 1] * dt[1] + T4[4 * i + 2] * dt[2] + T4[4 * i + 3];
      }
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T4[4 * i + j] = Rn[3 * i + j];
        T4[4 * i + 3] = tn[i];
      }
    }
  if (tid == 0 && stats) {
    stats[0] = rz0;
    stats[1] = rz;
    stats[2] = done;
  }
}

// Row assembly for the replicated-vector PCG, one workgroup of 256 per free frame
// (row v): the diagonal block and gradient are the sums of the frame's incident
// edge blocks (its "i" edges, then its "j" edges); the four wavefronts take every
// fourth edge of that list, sixteen loads in flight per lane (one lane per word),
// and the partial sums are combined in a fixed order.  Wavefront 0 then inverts
// the diagonal block (6x6 Cholesky, FP64; a block that is not positive definite
// raises the flag and is replaced by the identity) and stores, in the PCG's
// storage type, the diagonal block, its inverse and r0 = -g.  One more workgroup
// (the last) sums the energies and counts over all edges for the trace.
constexpr int kAsmThreads = 256;

template <class T>
__global__ void __launch_bounds__(kAsmThreads) k_row_assemble(
    long long nfree, long long E, const double* __restrict__ eb, const long long* __restrict__ iptr,
    const long long* __restrict__ jptr, const long long* __restrict__ ej_sorted, const int* __restrict__ frame_of_var,
    int precond, T* __restrict__ diag_t, T* __restrict__ minv_g, T* __restrict__ r0, double* __restrict__ trace_slot,
    int* flags) {
  __shared__ double part[kAsmThreads / 64][48];
  __shared__ double red6s[6][kAsmThreads];  // energy workgroup: six sums at once
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = kAsmThreads / 64;
  const long long v = blockIdx.x;
  if (v == nfree) {
    if (!trace_slot) return;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (long long e = tid; e < E; e += kAsmThreads)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[q] += eb[(size_t)e * kEdgeWords + kEEs + q];
    // the six sums share one tree (the same order per value as a single-value tree)
#pragma unroll
    for (int q = 0; q < 6; ++q) red6s[q][tid] = acc[q];
    __syncthreads();
    for (int o = kAsmThreads / 2; o > 0; o >>= 1) {
      if (tid < o)
#pragma unroll
        for (int q = 0; q < 6; ++q) red6s[q][tid] += red6s[q][tid + o];
      __syncthreads();
    }
    if (tid == 0) {
      trace_slot[0] = red6s[0][0] + red6s[1][0] + red6s[2][0];
      for (int q = 0; q < 6; ++q) trace_slot[1 + q] = red6s[q][0];
      trace_slot[7] = 0.0;
    }
    return;
  }
  const int f = frame_of_var[v];
  const long long i0 = iptr[f], ni = iptr[f + 1] - i0;
  const long long j0 = jptr[f], cnt = ni + (jptr[f + 1] - j0);
  if (lane < 42) {
    const int offI = lane < 36 ? kEHii + lane : kEGi + (lane - 36);
    const int offJ = lane < 36 ? kEHjj + lane : kEGj + (lane - 36);
    constexpr int kDepth = 16;
    double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long q0 = wave; q0 < cnt; q0 += (long long)NW * kDepth) {
      long long off[kDepth];
#pragma unroll
      for (int u = 0; u < kDepth; ++u) {
        const long long q = q0 + (long long)NW * u;
        off[u] = q >= cnt ? -1
                 : q < ni ? (long long)(i0 + q) * kEdgeWords + offI
                          : (long long)ej_sorted[j0 + q - ni] * kEdgeWords + offJ;
      }
      double t[kDepth];
#pragma unroll
      for (int u = 0; u < kDepth; ++u) t[u] = off[u] >= 0 ? eb[off[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < kDepth; ++u) s8[u & 7] += t[u];
    }
    part[wave][lane] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  }
  __syncthreads();
  if (tid < 42) part[0][tid] = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
  __syncthreads();
  if (tid < 36) diag_t[v * 36 + tid] = (T)part[0][tid];
  else if (tid < 42) r0[6 * v + tid - 36] = (T)(-part[0][tid]);
  if (tid == 0) {
    double A[36];
    for (int q = 0; q < 36; ++q) A[q] = part[0][q];
    if (block_jacobi_inverse6(A, precond) < 0) {
      atomicOr(flags, kFlagNotPD);
      for (int q = 0; q < 36; ++q) A[q] = (q % 7 == 0) ? 1.0 : 0.0;
    }
    for (int q = 0; q < 36; ++q) part[1][q] = A[q];
  }
  __syncthreads();
  if (tid < 36) minv_g[v * 36 + tid] = (T)part[1][tid];
}

// Replicated-vector PCG in one launch of resident workgroups (at most what the
// device holds at once; every wait is bounded).  Every workgroup keeps the full
// vectors and all block-Jacobi inverses in LDS and updates them redundantly, in
// the same fixed order, so all copies stay bit-identical; each wavefront owns one
// matrix row and keeps that row's blocks in registers (one block per lane) for
// the whole solve.
//
// The recurrence is the single-reduction form of preconditioned CG (Chronopoulos
// and Gear, 1989): with u = M^-1 r and w = A u,
//   gamma_k = (r_k, u_k), delta_k = (w_k, u_k), beta_k = gamma_k / gamma_{k-1},
//   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1}),
//   p_k = u_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}  (s = A p),
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k,
// the same iterates as the two-reduction form in exact arithmetic.  Per iteration
// one product w = A u crosses workgroups (the owners publish their rows as tagged
// words; every workgroup polls until it holds all of w).  beta needs gamma alone,
// so p = u + beta p runs while the words travel and s = w + beta s as they arrive;
// delta = (w, u) then reduces behind one barrier, and gamma of the next iterate
// behind the barrier that ends the r and u updates.
constexpr int kRepThreads = 512;
constexpr int kRepWaves = kRepThreads / 64;

// MLDS: the block-Jacobi inverses are copied into LDS (else read from memory,
// for problems whose vectors fit in LDS but not together with the inverses).
template <class T, bool MLDS>
__global__ void __launch_bounds__(kRepThreads) k_solve_rep(
    long long nfree, int F, int iters, const T* __restrict__ hij, const long long* __restrict__ row_ptr,
    const int2* __restrict__ entries, const int* __restrict__ frame_of_var, const int* __restrict__ var_of,
    const T* __restrict__ diag_t, const T* __restrict__ minv_g, const T* __restrict__ r0,
    unsigned long long* ap_words, double* __restrict__ delta_out, double* __restrict__ poses, int update,
    double* __restrict__ stats, int* flags, unsigned tag_base, unsigned spin_limit) {
  extern __shared__ double lds_dyn[];
  __shared__ double sh[(kRepWaves + 1) * kParts];
  __shared__ double blk[kRepWaves][36];
  __shared__ int sh_ok;
  const long long n = 6 * nfree;
  T* r = reinterpret_cast<T*>(lds_dyn);
  T* u = r + n;      // M^-1 r
  T* p = u + n;
  T* sv = p + n;     // A p, by recurrence
  T* wvec = sv + n;  // A u, gathered
  T* minv_l = wvec + n;
  const T* minv = MLDS ? minv_l : minv_g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long wg = blockIdx.x, ngroups = gridDim.x;
  const long long v = wg * kRepWaves + wave;  // owned row (if < nfree)
  const bool owner = v < nfree;
  if (tid == 0) sh_ok = 1;
  __syncthreads();

  // ---- prologue (rows assembled and inverted by k_row_assemble): owners load
  // their row's blocks into registers, every workgroup loads r and M^-1 into LDS
  const bool bad = (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagNotPD) != 0;
  // NB register blocks per lane: rows of up to 64 NB - 1 off-diagonal blocks keep
  // every block in registers (two per lane in FP32; FP64 holds one)
  constexpr int NB = sizeof(T) == 4 ? 2 : 1;
  T blockreg[NB][36];
  int partner[NB];
  bool tr[NB];
  long long ne = 0;
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    partner[s] = -1;
    tr[s] = false;
  }
  if (owner) {
    if (lane < 36) blk[wave][lane] = (double)diag_t[v * 36 + lane];
    __builtin_amdgcn_wave_barrier();
    // virtual entries 0..ne-1 are the off-diagonal blocks, ne the diagonal; lane l
    // holds entries l, l + 64, ...
    ne = row_ptr[v + 1] - row_ptr[v];
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const long long q = lane + 64 * s;
      if (q < ne) {
        const int2 en = entries[row_ptr[v] + q];
        partner[s] = en.x;
        tr[s] = en.y & 1;
        const T* B = hij + (size_t)(en.y >> 1) * 36;
#pragma unroll
        for (int e = 0; e < 36; ++e) blockreg[s][e] = B[e];
      } else if (q == ne) {
        partner[s] = (int)v;
#pragma unroll
        for (int e = 0; e < 36; ++e) blockreg[s][e] = (T)blk[wave][e];
      }
    }
  }
  for (long long o = tid; o < n; o += kRepThreads) {
    r[o] = r0[o];
    p[o] = (T)0;
    sv[o] = (T)0;
  }
  if constexpr (MLDS)
    for (long long o = tid; o < 36 * nfree; o += kRepThreads) minv_l[o] = minv_g[o];
  __syncthreads();
  // u = M^-1 r and (r, u) partials, one block row per thread
  double part_ru = 0.0;
  for (long long w = tid; w < nfree; w += kRepThreads) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double s2 = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) s2 += (double)minv[w * 36 + 6 * a + b] * (double)r[6 * w + b];
      const T ut = (T)s2;
      u[6 * w + a] = ut;
      part_ru += (double)r[6 * w + a] * (double)ut;
    }
  }
  // gamma_0 = (r_0, u_0); its barrier also completes u.  The two sums of an
  // iteration use their own slots (delta at sh[0..], gamma at sh[2 NW..]): a slot is
  // written again only after the barrier of the other sum, which every thread
  // passes after its reads.
  double* const sh_delta = sh;
  double* const sh_gamma = sh + 2 * kRepWaves;
  double gamma = block_sum_dpp_1<kRepWaves>(part_ru, sh_gamma);
  const int rr = lane / 6, a6 = lane - 6 * (lane / 6);  // update pass: row, element
  T xo = (T)0;  // owner lanes 0..5: x of the owned row
  int done = 0;
  const double rz0 = bad ? 0.0 : gamma;
  double gamma_prev = 1.0, alpha_prev = 1.0;
  constexpr int WPV = sizeof(T) / 4;  // 32-bit halves per value, each published with the tag
  for (int k = 0; k < iters && !bad && sh_ok && gamma > 1e-30; ++k) {
    const double beta = k == 0 ? 0.0 : gamma / gamma_prev;
    const float beta_f = (float)beta;
    const unsigned tag = tag_base + (unsigned)k + 1u;
    unsigned long long* apw = ap_words + (size_t)(k & 1) * n * WPV;
    // ---- w = A u (exchange k): owners compute (A u)_v from register blocks and
    // the LDS copy of u, and publish it
    if (owner) {
      T acc[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        if (partner[s] >= 0) {
          T uw[6];
#pragma unroll
          for (int b = 0; b < 6; ++b) uw[b] = u[6 * (long long)partner[s] + b];
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            T s2 = (T)0;
#pragma unroll
            for (int j = 0; j < 6; ++j) s2 += (tr[s] ? blockreg[s][6 * j + i] : blockreg[s][6 * i + j]) * uw[j];
            acc[i] += s2;
          }
        }
      }
      // rows with more entries than the registers hold take the rest from memory
      for (long long q = 64 * NB + lane; q <= ne; q += 64) {
        T uw[6], y[6];
        if (q < ne) {
          const int2 en = entries[row_ptr[v] + q];
#pragma unroll
          for (int b = 0; b < 6; ++b) uw[b] = u[6 * (long long)en.x + b];
          block_mv<T>(hij + (size_t)(en.y >> 1) * 36, uw, en.y & 1, y);
        } else {
          T dg[36];
#pragma unroll
          for (int q2 = 0; q2 < 36; ++q2) dg[q2] = (T)blk[wave][q2];
#pragma unroll
          for (int b = 0; b < 6; ++b) uw[b] = u[6 * v + b];
          block_mv<T>(dg, uw, false, y);
        }
#pragma unroll
        for (int b = 0; b < 6; ++b) acc[b] += y[b];
      }
      double accd[6];
#pragma unroll
      for (int b = 0; b < 6; ++b) accd[b] = (double)acc[b];
      const double tb = wave_sum6_d(accd);  // value lane / 8
      if ((lane >> 3) < 6 && (lane & 7) < WPV) {
        // lane 8b + h publishes half h of value b: (tag << 32) | bits
        const int b = lane >> 3, h = lane & 7;
        unsigned bits;
        if constexpr (WPV == 1) {
          bits = __float_as_uint((float)tb);
        } else {
          const unsigned long long d = (unsigned long long)__double_as_longlong(tb);
          bits = h ? (unsigned)(d >> 32) : (unsigned)(d & 0xffffffffull);
        }
        st_shared(&apw[(6 * v + b) * WPV + h], ((unsigned long long)tag << 32) | bits);
      }
    }
    // ---- p = u + beta p over the whole vector (beta needs gamma only), while the
    // other owners' words are on their way
    for (long long o = tid; o < n; o += kRepThreads) {
      if constexpr (sizeof(T) == 4)
        p[o] = __builtin_fmaf(beta_f, p[o], u[o]);
      else
        p[o] = (T)((double)u[o] + beta * (double)p[o]);
    }
    // ---- every workgroup gathers all of w (polling the tagged words); the thread
    // that gathers a value forms s = w + beta s and the (w, u) partial of it
    double part_wu = 0.0;
    constexpr int kMaxPer = 8;  // values per thread gathered at once
    const long long nw = n * WPV;
    for (long long o0 = tid; o0 < nw; o0 += (long long)kRepThreads * kMaxPer) {
      unsigned long long wv[kMaxPer];
      const unsigned long long filler = (unsigned long long)tag << 32;  // past the end: ready
      unsigned spins = 0;
      for (;;) {
        // all loads of a poll are issued before any is tested
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) {
          const long long o = o0 + (long long)q * kRepThreads;
          wv[q] = o < nw ? ld_shared(&apw[o]) : filler;
        }
        bool ready = true;
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) ready = ready & ((unsigned)(wv[q] >> 32) == tag);
        if (ready) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
          atomicOr(flags, kFlagTimeout);
          sh_ok = 0;
          break;
        }
      }
      if constexpr (WPV == 1) {
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) {
          const long long o = o0 + (long long)q * kRepThreads;
          if (o < nw) {
            const float wq = __uint_as_float((unsigned)(wv[q] & 0xffffffffull));
            sv[o] = __builtin_fmaf(beta_f, sv[o], wq);
            part_wu += (double)wq * (double)u[o];
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) {
          const long long o = o0 + (long long)q * kRepThreads;
          if (o < nw) reinterpret_cast<unsigned*>(wvec)[o] = (unsigned)(wv[q] & 0xffffffffull);
        }
      }
    }
    if constexpr (WPV == 2) {
      __syncthreads();  // both halves of a value gathered
      for (long long o = tid; o < n; o += kRepThreads) {
        sv[o] = (T)((double)wvec[o] + beta * (double)sv[o]);
        part_wu += (double)wvec[o] * (double)u[o];
      }
    }
    // ---- delta = (w, u) behind one barrier (which also completes p and s)
    const double delta = block_sum_dpp_1<kRepWaves>(part_wu, sh_delta);
    if (!sh_ok) break;
    const double alpha = gamma / (delta - (k == 0 ? 0.0 : beta * gamma / alpha_prev));
    const float alpha_f = (float)alpha;
    if (owner && lane < 6) xo = (T)((double)xo + alpha * (double)p[6 * v + lane]);
    // ---- r -= alpha s element by element, then u = M^-1 r and the (r, u) partials
    // per block row: each wavefront takes ten block rows at a time, six lanes per
    // row (lanes 60..63 idle), so consecutive lanes touch consecutive values; a
    // row's six new r values are read back from LDS after a wavefront barrier (the
    // same wavefront wrote them).  FP32 storage updates in FP32; FP64 stays with the
    // dot products and alpha, beta.
    part_ru = 0.0;
    for (long long w0 = (long long)wave * 10; w0 < nfree; w0 += 10 * kRepWaves) {
      const long long w = w0 + rr;
      const bool act = lane < 60 && w < nfree;
      double rb = 0.0;
      if (act) {
        const long long o = 6 * w + a6;
        T rn;
        if constexpr (sizeof(T) == 4)
          rn = __builtin_fmaf(-alpha_f, sv[o], r[o]);
        else
          rn = (T)((double)r[o] - alpha * (double)sv[o]);
        r[o] = rn;
        rb = (double)rn;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (act) {
        const T* mr = minv + w * 36 + 6 * a6;
        T ut;
        if constexpr (sizeof(T) == 4) {
          float s2 = 0.0f;
#pragma unroll
          for (int b = 0; b < 6; ++b) s2 = __builtin_fmaf(mr[b], r[6 * w + b], s2);
          ut = s2;
        } else {
          double s2 = 0.0;
#pragma unroll
          for (int b = 0; b < 6; ++b) s2 += (double)mr[b] * (double)r[6 * w + b];
          ut = (T)s2;
        }
        u[6 * w + a6] = ut;
        part_ru += rb * (double)ut;
      }
    }
    gamma_prev = gamma;
    alpha_prev = alpha;
    // ---- gamma = (r, u) of the new iterate; its barrier also completes u
    gamma = block_sum_dpp_1<kRepWaves>(part_ru, sh_gamma);
    ++done;
  }
  const double rz = bad ? 0.0 : gamma;
  // epilogue: owners publish dx and update their poses
  if (owner && lane < 6 && delta_out) delta_out[6LL * frame_of_var[v] + lane] = bad ? 0.0 : (double)xo;
  if (delta_out)
    for (long long o = wg * kRepThreads + tid; o < 6LL * F; o += ngroups * kRepThreads)
      if (var_of[o / 6] < 0) delta_out[o] = 0.0;
  if (owner && update && !bad && sh_ok) {
    double xi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) xi[q] = (double)__shfl(xo, q);
    if (lane == 0) {
      double dR[9], dt[3];
      exp_se3(xi, dR, dt);
      double* T4 = poses + (size_t)frame_of_var[v] * 16;
      double Rn[9], tn[3];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          Rn[3 * i + j] = T4[4 * i] * dR[j] + T4[4 * i + 1] * dR[3 + j] + T4[4 * i + 2] * dR[6 + j];
        tn[i] = T4[4 * i] * dt[0] + T4[4 * i + 1] * dt[1] + T4[4 * i + 2] * dt[2] + T4[4 * i + 3];
      }
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T4[4 * i + j] = Rn[3 * i + j];
        T4[4 * i + 3] = tn[i];
      }
    }
  }
  if (wg == 0 && tid == 0 && stats) {
    stats[0] = rz0;
    stats[1] = rz;
    stats[2] = done;
  }
}

// The sparse term applied matrix-free inside the distributed PCG (Sec. 4.4): per
// sparse frame pair g = (a, b), sorted correspondence positions [ptr[g], ptr[g+1])
// with points pts[m] = (P in frame a, Q in frame b), and y_g = w J^T J p over them,
// 12 values per pair (frame a's six, then frame b's).
struct MfArgs {
  const float* pts;
  const long long* ptr;
  const int* ij;
  long long S;
  const long long* edge_sparse;
  const long long* iptr;       // edges of frame f as their lower frame: [iptr[f], iptr[f+1])
  const long long* jptr;       // ... as their upper frame: ej_sorted[jptr[f] ..]
  const long long* ej_sorted;
  double w;
  double* y;
};

// Correspondence points in sorted position order, oriented as their pair (a < b).
__global__ void k_mf_points(const int* __restrict__ fi, const int* __restrict__ fj, const float* __restrict__ pi,
                            const float* __restrict__ pj, const long long* __restrict__ perm, long long M,
                            float* __restrict__ pts) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const long long c = perm[m];
  const bool sw = fi[c] > fj[c];
  const float* P = sw ? pj : pi;
  const float* Q = sw ? pi : pj;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pts[6 * m + k] = P[3 * c + k];
    pts[6 * m + 3 + k] = Q[3 * c + k];
  }
}

// Diagonal blocks of the dense term alone per free frame (one wavefront per row,
// the frame's edges in list order), for the product in matrix-free sparse mode.
template <class T>
__global__ void __launch_bounds__(64) k_row_dense_diag(const double* __restrict__ ediag,
                                                       const long long* __restrict__ iptr,
                                                       const long long* __restrict__ jptr,
                                                       const long long* __restrict__ ej_sorted,
                                                       const int* __restrict__ frame_of_var, T* __restrict__ diag_t) {
  const long long v = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane >= 36) return;
  const int f = frame_of_var[v];
  double s = 0.0;
  for (long long k = iptr[f]; k < iptr[f + 1]; ++k) s += ediag[(size_t)k * 72 + lane];
  for (long long k = jptr[f]; k < jptr[f + 1]; ++k) s += ediag[(size_t)ej_sorted[k] * 72 + 36 + lane];
  diag_t[v * 36 + lane] = (T)s;
}

// Distributed-vector PCG (the two-reduction block-Jacobi recurrence of the
// cooperative kernel) for problems whose vectors do not fit in LDS five times
// over but whose search direction fits once.  Rows are assembled and inverted by
// k_row_assemble before it.
//
// Work split: each workgroup owns the contiguous range of rows whose start falls
// in its share of the total row weight (a row weighs its entries, the diagonal
// block counted, plus kDistRowWeight), so the block products are shared evenly
// however uneven the rows are.  Inside a workgroup the rows are cut into segments
// of at most c consecutive entries, one per thread (c chosen so that the segments
// fit the threads); a thread sums its segment's block products, streamed from
// memory every iteration, and each row's segment sums are added in order by its
// owner (row r of the range: wavefront r mod 8, lanes 0..5), which keeps x, r and
// A p of the row to itself.  z is published by the owners, and after each
// reduction every workgroup rebuilds the full search direction p = z + beta p in
// its LDS, so the products read partner values from LDS.  Reductions are
// all-gathers without atomics: each workgroup publishes its partial sums as tagged
// 32-bit halves into its own slot (slot buffers alternate with the parity of the
// reduction count: a workgroup can be at most one reduction ahead of the slowest),
// and every workgroup reads all slots, one thread per workgroup, and adds them in
// one fixed tree, so all workgroups hold the same sums.  Per iteration: rebuild p,
// A p, reduce (p.Ap), update x, r, z, reduce (r.z).
constexpr int kDistThreads = 512;
constexpr int kDistWaves = kDistThreads / 64;
constexpr int kDistMaxRows = kDistThreads - 64;  // rows of one workgroup's range
constexpr long long kDistRowWeight = 8;
constexpr size_t kDistSegBytes = sizeof(double) * 6 * kDistThreads;  // segment sums, dynamic LDS
constexpr size_t kDistLdsMax = 128 * 1024;

// Sum over all workgroups of K doubles per thread (see above); false if a wait gave
// up.  `sh`: kDistWaves * K doubles.
template <int K>
__device__ bool dist_reduce(double (&v)[K], unsigned long long* slots, long long G, unsigned tag, unsigned parity,
                            double* sh, int* sh_ok, int* flags, unsigned spin_limit) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = wave_sum_d(v[k]);
    if (lane == 0) sh[wave * K + k] = t;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's earlier stores have landed
  __syncthreads();
  if (tid < 2 * K) {
    const int k = tid >> 1, h = tid & 1;
    double t = 0.0;
    for (int w = 0; w < kDistWaves; ++w) t += sh[w * K + k];
    const unsigned long long d = (unsigned long long)__double_as_longlong(t);
    const unsigned bits = h ? (unsigned)(d >> 32) : (unsigned)(d & 0xffffffffull);
    st_shared(&slots[((size_t)parity * G + blockIdx.x) * 2 * K + tid], ((unsigned long long)tag << 32) | bits);
  }
  double got[K];
#pragma unroll
  for (int k = 0; k < K; ++k) got[k] = 0.0;
  if (tid < G) {
    const unsigned long long* src = slots + ((size_t)parity * G + tid) * 2 * K;
    unsigned long long w[2 * K];
    unsigned spins = 0;
    for (;;) {
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) w[q] = ld_shared(&src[q]);
      bool ready = true;
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) ready = ready & ((unsigned)(w[q] >> 32) == tag);
      if (ready) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin_limit) {
        atomicOr(flags, kFlagTimeout);
        *sh_ok = 0;
        break;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      got[k] = __longlong_as_double((long long)(((w[2 * k + 1] & 0xffffffffull) << 32) | (w[2 * k] & 0xffffffffull)));
  }
  __syncthreads();  // sh was read for the publication
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = wave_sum_d(got[k]);
    if (lane == 0) sh[wave * K + k] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
    for (int w = 0; w < kDistWaves; ++w) t += sh[w * K + k];
    v[k] = t;
  }
  const bool ok = *sh_ok != 0;
  __syncthreads();  // sh and sh_ok read by every thread
  return ok;
}

template <class T, bool MF>
__global__ void __launch_bounds__(kDistThreads) k_solve_dist(
    long long nfree, int F, int iters, const T* __restrict__ hij, const long long* __restrict__ row_ptr,
    const int2* __restrict__ entries, const int* __restrict__ frame_of_var, const int* __restrict__ var_of,
    const T* __restrict__ diag_t, const T* __restrict__ minv_g, const T* __restrict__ r0, T* zpub,
    T* __restrict__ xv, T* __restrict__ rv, T* __restrict__ apv, unsigned long long* slots, unsigned tag_base,
    double* __restrict__ delta_out, double* __restrict__ poses, int update, double* __restrict__ stats, int* flags,
    unsigned spin_limit, MfArgs mf) {
  extern __shared__ double lds_dyn[];
  double* segsum = lds_dyn;                                 // [kDistThreads][6] segment sums
  T* p = reinterpret_cast<T*>(lds_dyn + 6 * kDistThreads);  // the full search direction
  __shared__ double sh[kDistWaves * 2];
  __shared__ int sh_ok;
  __shared__ long long sh_range[2];
  __shared__ int seg_first[kDistMaxRows + 1];
  __shared__ int sh_c;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long G = gridDim.x;
  const long long gw = (long long)blockIdx.x * kDistWaves + wave, nw = G * kDistWaves;
  const long long n = 6 * nfree;
  unsigned nred = 0;  // reductions so far: tag tag_base + nred + 1, slot parity nred & 1
  auto reduce1 = [&](double (&v)[1]) {
    const bool ok = dist_reduce<1>(v, slots, G, tag_base + nred + 1u, nred & 1u, sh, &sh_ok, flags, spin_limit);
    ++nred;
    return ok;
  };

  // ---- this workgroup's rows [rs, re) by weight, and their segments
  if (tid == 0) sh_ok = 1;
  const long long Wt = row_ptr[nfree] + (1 + kDistRowWeight) * nfree;
  if (tid < 2) {
    const long long target = ((long long)(blockIdx.x + tid) * Wt + G - 1) / G;
    long long lo = 0, hi = nfree;  // the first row whose weighted start reaches target
    while (lo < hi) {
      const long long mid = (lo + hi) / 2;
      if (row_ptr[mid] + (1 + kDistRowWeight) * mid >= target) hi = mid;
      else lo = mid + 1;
    }
    sh_range[tid] = lo;
  }
  __syncthreads();
  const long long rs = sh_range[0];
  long long re = sh_range[1];
  if (tid == 0) {
    long long R = re - rs;
    if (R > kDistMaxRows) {  // cannot be cut for the threads: flagged, its rows skipped
      atomicOr(flags, kFlagShape);
      R = 0;
    }
    const long long S = (row_ptr[rs + R] + rs + R) - (row_ptr[rs] + rs);  // entries of the range
    long long c = R > 0 ? (S + (kDistThreads - R) - 1) / (kDistThreads - R) : 1;
    if (c < 1) c = 1;
    int sgs = 0;
    for (long long r = 0; r < R; ++r) {
      seg_first[r] = sgs;
      const long long m = row_ptr[rs + r + 1] - row_ptr[rs + r] + 1;
      sgs += (int)((m + c - 1) / c);
    }
    seg_first[R] = sgs;
    sh_c = (int)c;
    sh_range[1] = rs + R;
  }
  __syncthreads();
  re = sh_range[1];
  const int R = (int)(re - rs);
  const int c = sh_c;
  // this thread's segment: row my_v, entries [q0, q1) (entry ne = the diagonal block)
  long long my_v = -1, q0 = 0, q1 = 0;
  if (tid < seg_first[R]) {
    int r = 0;
    while (seg_first[r + 1] <= tid) ++r;
    my_v = rs + r;
    q0 = (long long)(tid - seg_first[r]) * c;
    const long long m = row_ptr[my_v + 1] - row_ptr[my_v] + 1;
    q1 = q0 + c < m ? q0 + c : m;
  }
  const bool bad = (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagNotPD) != 0;

  // z = M^-1 r for an owned row (lanes 0..5), published; (r, z) partial
  auto precondition = [&](long long v, double rb, double& part) {
    double s2 = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const double rbb = __shfl(rb, b);
      if (lane < 6) s2 += (double)minv_g[v * 36 + 6 * lane + b] * rbb;
    }
    if (lane < 6) {
      const T zt = (T)s2;
      st_shared(&zpub[6 * v + lane], zt);
      part += rb * (double)zt;
    }
  };

  double rz = 0.0, rz0 = 0.0, beta = 0.0;
  int done = 0;
  if (!bad) {
    double part[1] = {0.0};
    for (long long v = rs + wave; v < re; v += kDistWaves) {
      const double rb = lane < 6 ? (double)r0[6 * v + lane] : 0.0;
      if (lane < 6) {
        xv[6 * v + lane] = (T)0;
        rv[6 * v + lane] = (T)rb;
      }
      precondition(v, rb, part[0]);
    }
    reduce1(part);
    rz = rz0 = part[0];
  }
  for (int k = 0; k < iters && !bad && sh_ok; ++k) {
    if (rz <= 1e-30) break;
    // p = z (first iteration) or z + beta p; z was published before the last reduction
    const T tb = (T)beta;
    for (long long o = tid; o < n; o += kDistThreads) {
      const T zo = ld_shared(&zpub[o]);
      p[o] = k == 0 ? zo : (T)(zo + tb * p[o]);
    }
    __syncthreads();
    if constexpr (MF) {
      // y_g = w sum_m J^T (J_a p_a + J_b p_b) per sparse pair, one wavefront per pair:
      // r = T_a P - T_b Q, J_a x = R_a (omega_a x P + v_a), J_b x = -R_b (omega_b x Q + v_b)
      for (long long g = gw; g < mf.S; g += nw) {
        const int fa = mf.ij[2 * g], fb = mf.ij[2 * g + 1];
        const int va = var_of[fa], vb = var_of[fb];
        double Ra[9], Rb[9], xa[6], xb[6];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          Ra[q] = poses[(size_t)fa * 16 + 4 * (q / 3) + q % 3];
          Rb[q] = poses[(size_t)fb * 16 + 4 * (q / 3) + q % 3];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          xa[q] = va >= 0 ? (double)p[6 * (long long)va + q] : 0.0;
          xb[q] = vb >= 0 ? (double)p[6 * (long long)vb + q] : 0.0;
        }
        double ya[6] = {0, 0, 0, 0, 0, 0}, yb[6] = {0, 0, 0, 0, 0, 0};
        for (long long m = mf.ptr[g] + lane; m < mf.ptr[g + 1]; m += 64) {
          const double P[3] = {mf.pts[6 * m], mf.pts[6 * m + 1], mf.pts[6 * m + 2]};
          const double Q[3] = {mf.pts[6 * m + 3], mf.pts[6 * m + 4], mf.pts[6 * m + 5]};
          const double la[3] = {xa[1] * P[2] - xa[2] * P[1] + xa[3], xa[2] * P[0] - xa[0] * P[2] + xa[4],
                                xa[0] * P[1] - xa[1] * P[0] + xa[5]};
          const double lb[3] = {xb[1] * Q[2] - xb[2] * Q[1] + xb[3], xb[2] * Q[0] - xb[0] * Q[2] + xb[4],
                                xb[0] * Q[1] - xb[1] * Q[0] + xb[5]};
          double u[3];
#pragma unroll
          for (int r = 0; r < 3; ++r)
            u[r] = (Ra[3 * r] * la[0] + Ra[3 * r + 1] * la[1] + Ra[3 * r + 2] * la[2]) -
                   (Rb[3 * r] * lb[0] + Rb[3 * r + 1] * lb[1] + Rb[3 * r + 2] * lb[2]);
          double aR[3], bR[3];  // R_a^T u, R_b^T u
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            aR[r] = Ra[r] * u[0] + Ra[3 + r] * u[1] + Ra[6 + r] * u[2];
            bR[r] = Rb[r] * u[0] + Rb[3 + r] * u[1] + Rb[6 + r] * u[2];
          }
          ya[0] += P[1] * aR[2] - P[2] * aR[1];
          ya[1] += P[2] * aR[0] - P[0] * aR[2];
          ya[2] += P[0] * aR[1] - P[1] * aR[0];
          yb[0] -= Q[1] * bR[2] - Q[2] * bR[1];
          yb[1] -= Q[2] * bR[0] - Q[0] * bR[2];
          yb[2] -= Q[0] * bR[1] - Q[1] * bR[0];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            ya[3 + r] += aR[r];
            yb[3 + r] -= bR[r];
          }
        }
        const double sa = wave_sum6_d(ya), sb = wave_sum6_d(yb);  // value lane / 8
        if ((lane & 7) == 0 && (lane >> 3) < 6) {
          st_shared(&mf.y[12 * g + (lane >> 3)], mf.w * sa);
          st_shared(&mf.y[12 * g + 6 + (lane >> 3)], mf.w * sb);
        }
      }
      double none[1] = {0.0};  // a reduction as the barrier after the pair sums
      if (!reduce1(none)) break;
    }
    // segment sums of the block products
    {
      double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (my_v >= 0) {
        const long long e0 = row_ptr[my_v], ne = row_ptr[my_v + 1] - e0;
        int2 en_next = q0 < ne ? entries[e0 + q0] : make_int2((int)my_v, -1);
        for (long long q = q0; q < q1; ++q) {
          const int2 en = en_next;
          if (q + 1 < q1) en_next = q + 1 < ne ? entries[e0 + q + 1] : make_int2((int)my_v, -1);
          const T* B = en.y >= 0 ? hij + (size_t)(en.y >> 1) * 36 : diag_t + (size_t)my_v * 36;
          T pw[6], y[6];
#pragma unroll
          for (int b = 0; b < 6; ++b) pw[b] = p[6 * (long long)en.x + b];
          block_mv<T>(B, pw, en.y >= 0 && (en.y & 1), y);
#pragma unroll
          for (int b = 0; b < 6; ++b) acc[b] += (double)y[b];
        }
      }
#pragma unroll
      for (int b = 0; b < 6; ++b) segsum[6 * tid + b] = acc[b];
    }
    __syncthreads();
    // owners: A p of their rows (segments in order), and the (p, A p) partial
    double part[1] = {0.0};
    for (int rl = wave; rl < R; rl += kDistWaves) {
      const long long v = rs + rl;
      double mfv = 0.0;
      if constexpr (MF) {
        // the sparse pairs' sums over every edge of the frame, also those whose other
        // frame is not a variable (the gauge frame, held frames): as frame a (lower)
        // of the edges it starts, as frame b of the others
        const int f = frame_of_var[v];
        const long long ni = mf.iptr[f + 1] - mf.iptr[f], nj = mf.jptr[f + 1] - mf.jptr[f];
        double ms[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (long long q = lane; q < ni + nj; q += 64) {
          const long long e = q < ni ? mf.iptr[f] + q : mf.ej_sorted[mf.jptr[f] + q - ni];
          const long long g = mf.edge_sparse[e];
          if (g >= 0) {
            const double* yg = mf.y + 12 * g + (q < ni ? 0 : 6);
#pragma unroll
            for (int b = 0; b < 6; ++b) ms[b] += ld_shared(&yg[b]);
          }
        }
        const double t = wave_sum6_d(ms);        // value lane / 8
        mfv = __shfl(t, 8 * (lane < 6 ? lane : 0));  // lane a < 6: value a
      }
      if (lane < 6) {
        double t = 0.0;
        for (int sg = seg_first[rl]; sg < seg_first[rl + 1]; ++sg) t += segsum[6 * sg + lane];
        const T ap = (T)(t + mfv);
        apv[6 * v + lane] = ap;
        part[0] += (double)p[6 * v + lane] * (double)ap;
      }
    }
    if (!reduce1(part)) break;
    const double alpha = rz / part[0];
    double part2[1] = {0.0};
    for (long long v = rs + wave; v < re; v += kDistWaves) {
      double rb = 0.0;
      if (lane < 6) {
        const long long o = 6 * v + lane;
        xv[o] = (T)((double)xv[o] + alpha * (double)p[o]);
        rb = (double)(T)((double)rv[o] - alpha * (double)apv[o]);
        rv[o] = (T)rb;
      }
      precondition(v, rb, part2[0]);
    }
    if (!reduce1(part2)) break;
    beta = part2[0] / rz;
    rz = part2[0];
    ++done;
  }
  if (delta_out) {
    for (long long v = rs + wave; v < re; v += kDistWaves)
      if (lane < 6) delta_out[6LL * frame_of_var[v] + lane] = bad ? 0.0 : (double)xv[6 * v + lane];
    for (long long o = (long long)blockIdx.x * kDistThreads + tid; o < 6LL * F; o += G * kDistThreads)
      if (var_of[o / 6] < 0) delta_out[o] = 0.0;
  }
  if (update && !bad && sh_ok) {
    for (long long v = rs + wave; v < re; v += kDistWaves) {
      if (lane != 0) continue;
      double xi[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) xi[q] = (double)xv[6 * v + q];
      double dR[9], dt[3];
      exp_se3(xi, dR, dt);
      double* T4 = poses + (size_t)frame_of_var[v] * 16;
      double Rn[9], tn[3];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          Rn[3 * i + j] = T4[4 * i] * dR[j] + T4[4 * i + 1] * dR[3 + j] + T4[4 * i + 2] * dR[6 + j];
        tn[i] = T4[4 * i] * dt[0] + T4[4 * i + 1] * dt[1] + T4[4 * i + 2] * dt[2] + T4[4 * i + 3];
      }
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T4[4 * i + j] = Rn[3 * i + j];
        T4[4 * i + 3] = tn[i];
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0 && stats) {
    stats[0] = rz0;
    stats[1] = rz;
    stats[2] = done;
  }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

__global__ void k_zero_tags(unsigned long long* tags, long long n, unsigned* bar) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) tags[k] = 0ull;
  if (k == 0) *bar = 0u;
}

// Energy and counts over each problem's edges, fixed order (one workgroup of 256
// per problem; 8 words per problem at dst).
__global__ void __launch_bounds__(256) k_energy(const double* __restrict__ eb,
                                                const long long* __restrict__ seg_edge_ptr,
                                                double* __restrict__ dst_all) {
  __shared__ double sh6[6][256];  // the six sums share one tree (per value the order of a single tree)
  const int tid = threadIdx.x;
  const long long E0 = seg_edge_ptr[blockIdx.x], E = seg_edge_ptr[blockIdx.x + 1];
  double* dst = dst_all + 8 * blockIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long e = E0 + tid; e < E; e += 256)
    for (int k = 0; k < 6; ++k) acc[k] += eb[(size_t)e * kEdgeWords + kEEs + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) sh6[k][tid] = acc[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
#pragma unroll
      for (int k = 0; k < 6; ++k) sh6[k][tid] += sh6[k][tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    dst[0] = sh6[0][0] + sh6[1][0] + sh6[2][0];
    for (int k = 0; k < 6; ++k) dst[1 + k] = sh6[k][0];
    dst[7] = 0.0;
  }
}

// Energy sums of a large single problem on several workgroups: workgroup q sums a
// contiguous range of edges with the tree of k_energy into parts[8q ..], then one
// workgroup adds the parts (one per thread, the same tree).  A fixed order for a
// given edge count; one workgroup over 225k edges took 0.6 ms.
constexpr long long kEnergySplit = 32768;  // edges above which the split is used
constexpr int kEnergyMaxParts = 256;

__global__ void __launch_bounds__(256) k_energy_parts(const double* __restrict__ eb, long long E, long long chunk,
                                                      double* __restrict__ parts) {
  __shared__ double sh6[6][256];
  const int tid = threadIdx.x;
  const long long e0 = (long long)blockIdx.x * chunk, e1 = e0 + chunk < E ? e0 + chunk : E;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long e = e0 + tid; e < e1; e += 256)
    for (int k = 0; k < 6; ++k) acc[k] += eb[(size_t)e * kEdgeWords + kEEs + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) sh6[k][tid] = acc[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
#pragma unroll
      for (int k = 0; k < 6; ++k) sh6[k][tid] += sh6[k][tid + o];
    __syncthreads();
  }
  if (tid < 6) parts[8 * (size_t)blockIdx.x + tid] = sh6[tid][0];
}

__global__ void __launch_bounds__(256) k_energy_final(const double* __restrict__ parts, int nparts,
                                                      double* __restrict__ dst) {
  __shared__ double sh6[6][256];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 6; ++k) sh6[k][tid] = tid < nparts ? parts[8 * (size_t)tid + k] : 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
#pragma unroll
      for (int k = 0; k < 6; ++k) sh6[k][tid] += sh6[k][tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    dst[0] = sh6[0][0] + sh6[1][0] + sh6[2][0];
    for (int k = 0; k < 6; ++k) dst[1 + k] = sh6[k][0];
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
  // matrix-free sparse mode: the PCG's blocks hold the dense term only, and the
  // dense term's diagonal parts go beside them
  double* ed = nullptr;
  if (prm.sparse_matrix_free && with_jacobians) {
    ensure(c.ediag_dense, sizeof(double) * 72 * (size_t)(c.shape.E + 1));
    ed = c.ediag_dense.as<double>();
  }
  const long long E = c.shape.E;
  if (E == 0) return;
  if (E > kEdgeLaneMin) {
    // enough edges to fill the GPU one lane each
    const unsigned grid = (unsigned)((E + 63) / 64);
    if (c.pcg_storage == 1)
      hipLaunchKernelGGL(k_edge_blocks_lane<double>, dim3(grid), dim3(64), 0, c.stream, c.edge_ij.as<int>(), E,
                         c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                         c.records.as<double>(), (long long)c.shape.P, c.bidir, c.dense_tiles, poses,
                         prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                         c.eblocks.as<double>(), c.hij64.as<double>(), ed);
    else
      hipLaunchKernelGGL(k_edge_blocks_lane<float>, dim3(grid), dim3(64), 0, c.stream, c.edge_ij.as<int>(), E,
                         c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                         c.records.as<double>(), (long long)c.shape.P, c.bidir, c.dense_tiles, poses,
                         prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                         c.eblocks.as<double>(), c.hij32.as<float>(), ed);
    return;
  }
  constexpr int per = kEdgeThreads / 64;
  unsigned grid = (unsigned)((E + per - 1) / per);
  if (c.pcg_storage == 1)
    hipLaunchKernelGGL(k_edge_blocks<double>, dim3(grid), dim3(kEdgeThreads), 0, c.stream, c.edge_ij.as<int>(), E,
                       c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                       c.records.as<double>(), (long long)c.shape.P, c.bidir, c.dense_tiles, poses,
                       prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                       c.eblocks.as<double>(), c.hij64.as<double>(), ed);
  else
    hipLaunchKernelGGL(k_edge_blocks<float>, dim3(grid), dim3(kEdgeThreads), 0, c.stream, c.edge_ij.as<int>(), E,
                       c.edge_dense.as<long long>(), c.edge_sparse.as<long long>(), c.moments.as<double>(),
                       c.records.as<double>(), (long long)c.shape.P, c.bidir, c.dense_tiles, poses,
                       prm.use_sparse ? prm.w_sparse : 0.0, with_jacobians ? 1 : 0,
                       c.eblocks.as<double>(), c.hij32.as<float>(), ed);
}

template <class T>
void launch_solve_coop(Context& c, int iters, double* trace_slot, double* delta_out, double* poses, double* stats,
                       bool update, T* diag, T* minv, T* hij, T* vec) {
  long long nf = c.shape.nfree;
  long long n = 6 * nf;
  long long E = c.shape.E;
  auto kern = k_solve_coop<T>;
  if (c.pcg_grid == 0) {
    int per_cu = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                           kSolveThreads, 0),
              "occupancy query");
    c.pcg_grid = std::max(1, per_cu) * c.num_cus;
  }
  int G = (int)std::min<long long>((nf + kSolveWaves - 1) / kSolveWaves, std::min(c.pcg_grid, kMaxSolveGroups));
  if (G < 1) G = 1;
  ensure(c.pcg_partials, sizeof(double) * 2 * kParts * kMaxSolveGroups);
  ensure(c.pcg_barrier, sizeof(unsigned) * 4);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c.stream, c.pcg_barrier.as<unsigned>());
  c.pcg_tags_dirty = true;  // the barrier counter no longer matches the replicated kernel's running count
  T* x = vec;
  T* r = vec + n;
  T* z = vec + 2 * n;
  T* pb0 = vec + 3 * n;
  T* pb1 = vec + 4 * n;
  T* Ap = vec + 5 * n;
  double* parts = c.pcg_partials.as<double>();
  unsigned* bar = c.pcg_barrier.as<unsigned>();
  int F = c.shape.F;
  int upd = update ? 1 : 0;
  const double* eb = c.eblocks.as<double>();
  const long long* ip = c.iptr.as<long long>();
  const long long* jp = c.jptr.as<long long>();
  const long long* ejs = c.ej_sorted.as<long long>();
  const long long* rp = c.row_ptr.as<long long>();
  const int2* en = c.row_entries.as<int2>();
  const int* fov = c.frame_of_var.as<int>();
  const int* vof = c.var_of.as<int>();
  int* fl = c.flags.as<int>();
  int pc = c.precond;
  unsigned spin = c.spin_limit;
  void* args[] = {&nf, &F, &E, &iters, &eb, &hij, &ip, &jp, &ejs, &rp, &en, &fov, &vof, &diag, &minv, &x, &r,
                  &Ap, &z, &pb0, &pb1, &parts, &bar, &trace_slot, &delta_out, &poses, &upd, &stats, &fl, &pc, &spin};
  check_hip(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(G), dim3(kSolveThreads), args, 0,
                                       c.stream),
            "cooperative solve launch");
}

// LDS budget of the single-workgroup solve (dynamic part).
constexpr size_t kSingleLdsMax = 64 * 1024;

// Raise the dynamic LDS limit of k_solve_single<T, NT> (once per process).
template <class T, int NT>
void set_single_lds_limit() {
  static std::atomic<bool> done{false};
  if (done.load()) return;
  check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_solve_single<T, NT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSingleLdsMax),
            "set LDS limit");  // idempotent: two threads may both set it
  done.store(true);
}

// One workgroup of NT threads per problem; LDS sized for the largest problem.
template <class T, int NT>
bool launch_solve_single(Context& c, int iters, double* trace_slot, double* delta_out, double* poses, double* stats,
                         bool update, T* diag, T* minv, T* hij) {
  const long long nf = c.shape.max_seg_free;
  const size_t vec_bytes = sizeof(T) * 5 * 6 * (size_t)nf;
  const size_t minv_bytes = sizeof(T) * 36 * (size_t)nf;
  if (vec_bytes > kSingleLdsMax) return false;
  const int minv_lds = (vec_bytes + minv_bytes <= kSingleLdsMax) ? 1 : 0;
  const size_t lds = vec_bytes + (minv_lds ? minv_bytes : 0);
  set_single_lds_limit<T, NT>();
  hipLaunchKernelGGL((k_solve_single<T, NT>), dim3(c.shape.nseg), dim3(NT), lds, c.stream,
                     c.seg_var_ptr.as<long long>(), c.seg_edge_ptr.as<long long>(), c.seg_start.as<int>(), iters,
                     c.eblocks.as<double>(), hij, c.iptr.as<long long>(), c.jptr.as<long long>(),
                     c.ej_sorted.as<long long>(), c.row_ptr.as<long long>(), c.row_entries.as<int2>(),
                     c.frame_of_var.as<int>(), c.var_of.as<int>(), diag, minv, minv_lds, trace_slot, delta_out, poses,
                     update ? 1 : 0, stats, c.flags.as<int>(), c.precond);
  return true;
}

// LDS budget of the replicated-vector solve (dynamic part).
constexpr size_t kRepLdsMax = 128 * 1024;

template <class T>
bool launch_solve_rep(Context& c, int iters, double* trace_slot, double* delta_out, double* poses, double* stats,
                      bool update, T* diag_t, T* minv_g, T* hij, T* vec) {
  long long nf = c.shape.nfree;
  long long n = 6 * nf;
  long long E = c.shape.E;
  // vectors and inverses in LDS if they fit, else the vectors only
  const bool mlds = sizeof(T) * (5 * (size_t)n + 36 * (size_t)nf) <= kRepLdsMax;
  const size_t lds = sizeof(T) * (5 * (size_t)n + (mlds ? 36 * (size_t)nf : 0));
  if (lds > kRepLdsMax) return false;
  auto kern = mlds ? k_solve_rep<T, true> : k_solve_rep<T, false>;
  // kernel attributes once per process; the occupancy for the last LDS size asked
  // (contexts on several threads share these, hence the lock)
  static std::mutex mu;
  static bool attr_set = false;
  static int cached_per_cu = -1;
  static size_t cached_lds = 0;
  static bool cached_mlds = false;
  int per_cu_at;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!attr_set) {
      for (auto kk : {k_solve_rep<T, true>, k_solve_rep<T, false>})
        check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(kk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kRepLdsMax),
                  "set LDS limit");
      attr_set = true;
    }
    if (cached_per_cu < 0 || cached_lds != lds || cached_mlds != mlds) {
      int per_cu = 0;
      check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             kRepThreads, lds),
                "occupancy query");
      cached_per_cu = per_cu;
      cached_lds = lds;
      cached_mlds = mlds;
    }
    per_cu_at = cached_per_cu;
  }
  // every workgroup waits for all others within an iteration: all must be resident
  const long long G = (nf + kRepWaves - 1) / kRepWaves;   // one row per wavefront
  if (per_cu_at < 1 || G > (long long)per_cu_at * c.num_cus || G > kMaxSolveGroups) return false;
  ensure(c.pcg_barrier, sizeof(unsigned) * 4);
  // Exchange words carry an iteration tag that grows across launches, so
  // consecutive launches need no clearing: the buffer is zeroed when it is
  // (re)allocated, after an error, or before a tag would wrap.
  const long long nwords = 2 * n * (long long)(sizeof(T) / 4);
  ensure(c.pcg_tags, sizeof(unsigned long long) * (size_t)(nwords + 1));
  unsigned long long* tags = c.pcg_tags.as<unsigned long long>();
  const unsigned long long tag_end = (unsigned long long)c.pcg_tag_base + (unsigned long long)iters + 1ull;
  if (c.pcg_tags_dirty || c.pcg_tags_ptr != c.pcg_tags.p || tag_end >= 0xffffffffull) {
    hipLaunchKernelGGL(k_zero_tags, dim3((unsigned)((c.pcg_tags.cap / 8 + 255) / 256)), dim3(256), 0, c.stream, tags,
                       (long long)(c.pcg_tags.cap / 8), c.pcg_barrier.as<unsigned>());
    c.pcg_tag_base = 0;
    c.pcg_tags_ptr = c.pcg_tags.p;
    c.pcg_tags_dirty = false;
  }
  const unsigned tag_base = c.pcg_tag_base;
  c.pcg_tag_base += (unsigned)iters + 1u;
  T* r0 = vec;
  const int F = c.shape.F;
  int* fl = c.flags.as<int>();
  if (trace_slot && E > kEnergySplit) {  // the trace energy on several workgroups
    launch_energy_split(c, trace_slot);
    trace_slot = nullptr;
  }
  hipLaunchKernelGGL(k_row_assemble<T>, dim3((unsigned)(nf + 1)), dim3(kAsmThreads), 0, c.stream, nf, E,
                     c.eblocks.as<double>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                     c.ej_sorted.as<long long>(), c.frame_of_var.as<int>(), c.precond, diag_t, minv_g, r0, trace_slot,
                     fl);
  // Every workgroup waits for the others: with one context in the process a plain
  // launch of a grid that fits the occupancy is resident as a whole (nothing else
  // that waits runs beside it); with several, another context's kernels may hold
  // CUs, and a cooperative launch guarantees co-residency (about 16 us more per
  // launch).
  if (live_contexts() > 1) {
    const T* hij_c = hij;
    const long long* rp = c.row_ptr.as<long long>();
    const int2* en = c.row_entries.as<int2>();
    const int* fov = c.frame_of_var.as<int>();
    const int* vof = c.var_of.as<int>();
    const T* dg = diag_t;
    const T* mi = minv_g;
    const T* r0c = r0;
    int upd = update ? 1 : 0;
    unsigned spin = c.spin_limit;
    int itv = iters;
    void* args[] = {&nf, const_cast<int*>(&F), &itv, &hij_c, &rp, &en, &fov, &vof, &dg, &mi, &r0c, &tags,
                    &delta_out, &poses, &upd, &stats, &fl, const_cast<unsigned*>(&tag_base), &spin};
    check_hip(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)G), dim3(kRepThreads),
                                         args, lds, c.stream),
              "cooperative replicated solve launch");
  } else {
    hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(kRepThreads), lds, c.stream, nf, F, iters, (const T*)hij,
                       c.row_ptr.as<long long>(), c.row_entries.as<int2>(), c.frame_of_var.as<int>(),
                       c.var_of.as<int>(), (const T*)diag_t, (const T*)minv_g, (const T*)r0, tags, delta_out, poses,
                       update ? 1 : 0, stats, fl, tag_base, c.spin_limit);
  }
  return true;
}

// Occupancy of k_solve_dist<T, MF> at a dynamic LDS size (attributes set once per
// process; contexts on several threads share them, hence the lock).
template <class T, bool MF>
int dist_blocks_per_cu(size_t lds) {
  static std::mutex mu;
  static bool attr_set = false;
  static int cached = -1;
  static size_t cached_lds = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (!attr_set) {
    check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_solve_dist<T, MF>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDistLdsMax),
              "set LDS limit");
    attr_set = true;
  }
  if (cached < 0 || cached_lds != lds) {
    int q = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, reinterpret_cast<const void*>(k_solve_dist<T, MF>),
                                                           kDistThreads, lds),
              "occupancy query");
    cached = q;
    cached_lds = lds;
  }
  return cached;
}

template <class T, bool MF>
bool launch_solve_dist(Context& c, int iters, double* trace_slot, double* delta_out, double* poses, double* stats,
                       bool update, T* diag_t, T* minv_g, T* hij, T* vec) {
  long long nf = c.shape.nfree;
  long long n = 6 * nf;
  long long E = c.shape.E;
  const size_t lds = kDistSegBytes + sizeof(T) * (size_t)n;
  if (lds > kDistLdsMax) return false;
  const int per_cu = dist_blocks_per_cu<T, MF>(lds);
  if (per_cu < 1) return false;
  // every resident workgroup takes a share of the rows (the matrix-free product also
  // spreads its sparse pairs over all of them)
  long long G = std::min<long long>((long long)per_cu * c.num_cus, kMaxSolveGroups);
  if (!MF) G = std::min<long long>(G, std::max<long long>(1, (nf + 1) / 2));
  // a workgroup's rows must fit its threads: at most (2 E + 9 nfree) / (9 G) + 2 rows
  // start in one share of the weight (the kernel flags a range that does not fit)
  if ((2 * E + (1 + kDistRowWeight) * nf) / ((1 + kDistRowWeight) * G) + 2 > kDistMaxRows) return false;
  MfArgs mf{nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr};
  if (MF) {
    ensure(c.mf_y, sizeof(double) * 12 * (size_t)(c.shape.S + 1));
    mf = MfArgs{c.mf_pts.as<float>(), c.sparse_ptr.as<long long>(), c.sparse_ij.as<int>(), (long long)c.shape.S,
                c.edge_sparse.as<long long>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                c.ej_sorted.as<long long>(), c.mf_w_sparse, c.mf_y.as<double>()};
  }
  // reduction slots: [2 parities][workgroups][2 tagged halves]; tags grow across
  // launches, so the slots are cleared only when (re)allocated or before a tag wraps
  ensure(c.pcg_barrier, sizeof(unsigned) * 4);
  ensure(c.dist_slots, sizeof(unsigned long long) * 4 * kMaxSolveGroups);
  const unsigned long long nred = 1ull + (unsigned long long)iters * (MF ? 3ull : 2ull);
  if (c.dist_slots_ptr != c.dist_slots.p || (unsigned long long)c.dist_tag_base + nred + 1ull >= 0xffffffffull) {
    hipLaunchKernelGGL(k_zero_tags, dim3((4 * kMaxSolveGroups + 255) / 256), dim3(256), 0, c.stream,
                       c.dist_slots.as<unsigned long long>(), (long long)(4 * kMaxSolveGroups),
                       c.pcg_barrier.as<unsigned>());
    c.dist_tag_base = 0;
    c.dist_slots_ptr = c.dist_slots.p;
  }
  unsigned tag_base = c.dist_tag_base;
  c.dist_tag_base += (unsigned)nred;
  T* r0 = vec;
  T* z = vec + n;
  T* xv = vec + 2 * n;
  T* rv = vec + 3 * n;
  T* apv = vec + 4 * n;
  int* fl = c.flags.as<int>();
  if (trace_slot && E > kEnergySplit) {  // the trace energy on several workgroups
    launch_energy_split(c, trace_slot);
    trace_slot = nullptr;
  }
  hipLaunchKernelGGL(k_row_assemble<T>, dim3((unsigned)(nf + 1)), dim3(kAsmThreads), 0, c.stream, nf, E,
                     c.eblocks.as<double>(), c.iptr.as<long long>(), c.jptr.as<long long>(),
                     c.ej_sorted.as<long long>(), c.frame_of_var.as<int>(), c.precond, diag_t, minv_g, r0, trace_slot,
                     fl);
  // matrix-free sparse term: the product's diagonal blocks hold the dense term only
  // (the preconditioner above keeps the full blocks)
  if (MF)
    hipLaunchKernelGGL(k_row_dense_diag<T>, dim3((unsigned)nf), dim3(64), 0, c.stream, c.ediag_dense.as<double>(),
                       c.iptr.as<long long>(), c.jptr.as<long long>(), c.ej_sorted.as<long long>(),
                       c.frame_of_var.as<int>(), diag_t);
  const T* hij_c = hij;
  const long long* rp = c.row_ptr.as<long long>();
  const int2* en = c.row_entries.as<int2>();
  const int* fov = c.frame_of_var.as<int>();
  const int* vof = c.var_of.as<int>();
  const T* dg = diag_t;
  const T* mi = minv_g;
  const T* r0c = r0;
  unsigned long long* slots = c.dist_slots.as<unsigned long long>();
  int F = c.shape.F;
  int upd = update ? 1 : 0;
  unsigned spin = c.spin_limit;
  int itv = iters;
  // all workgroups wait for each other: a plain launch when this context is the
  // only one in the process (the grid fits the occupancy), else a cooperative one
  if (live_contexts() > 1) {
    void* args[] = {&nf, &F, &itv, &hij_c, &rp, &en, &fov, &vof, &dg, &mi, &r0c, &z, &xv, &rv, &apv, &slots,
                    &tag_base, &delta_out, &poses, &upd, &stats, &fl, &spin, &mf};
    check_hip(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_solve_dist<T, MF>), dim3((unsigned)G),
                                         dim3(kDistThreads), args, lds, c.stream),
              "cooperative distributed solve launch");
  } else {
    hipLaunchKernelGGL((k_solve_dist<T, MF>), dim3((unsigned)G), dim3(kDistThreads), lds, c.stream, nf, F, itv,
                       hij_c, rp, en, fov, vof, dg, mi, r0c, z, xv, rv, apv, slots, tag_base, delta_out, poses, upd,
                       stats, fl, spin, mf);
  }
  return true;
}

template <class T>
bool launch_solve_dist_any(Context& c, bool mf, int iters, double* trace_slot, double* delta_out, double* poses,
                           double* stats, bool update, T* diag_t, T* minv_g, T* hij, T* vec) {
  return mf ? launch_solve_dist<T, true>(c, iters, trace_slot, delta_out, poses, stats, update, diag_t, minv_g, hij,
                                         vec)
            : launch_solve_dist<T, false>(c, iters, trace_slot, delta_out, poses, stats, update, diag_t, minv_g, hij,
                                          vec);
}

void launch_mf_points(Context& c, const bf_corrs* co) {
  const long long M = c.shape.M;
  ensure(c.mf_pts, sizeof(float) * 6 * (size_t)(M + 1));
  if (M == 0 || !co) return;
  hipLaunchKernelGGL(k_mf_points, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, c.stream, co->frame_i, co->frame_j,
                     co->p_i, co->p_j, c.corr_perm.as<long long>(), M, c.mf_pts.as<float>());
}

// Largest problem (free frames) solved by the per-problem workgroup kernel when the
// kernel is chosen automatically.
constexpr long long kPerProblemMaxFree = 64;

bool solve_per_problem(const Context& c) {
  const bool many = c.shape.nseg > 1;
  return c.solve_mode == 4 || (c.solve_mode == 0 && (many || c.shape.max_seg_free <= kPerProblemMaxFree));
}

void prepare_solve(Context& c) {
  if (c.pcg_storage == 1) {
    set_single_lds_limit<double, 64>();
    set_single_lds_limit<double, 128>();
    set_single_lds_limit<double, 256>();
    set_single_lds_limit<double, 1024>();
  } else {
    set_single_lds_limit<float, 64>();
    set_single_lds_limit<float, 128>();
    set_single_lds_limit<float, 256>();
    set_single_lds_limit<float, 1024>();
  }
}

namespace {

// The per-problem kernel with workgroups of nt threads (64, 128, 256 or 1024).
bool launch_per_problem(Context& c, int nt, int iters, double* trace_slot, double* delta_out, double* poses,
                        double* stats, bool update) {
  auto go = [&](auto ntc) {
    constexpr int NT = decltype(ntc)::value;
    return c.pcg_storage == 1
               ? launch_solve_single<double, NT>(c, iters, trace_slot, delta_out, poses, stats, update,
                                                 c.diag64.as<double>(), c.minv64.as<double>(), c.hij64.as<double>())
               : launch_solve_single<float, NT>(c, iters, trace_slot, delta_out, poses, stats, update,
                                                c.diag32.as<float>(), c.minv32.as<float>(), c.hij32.as<float>());
  };
  switch (nt) {
    case 64: return go(std::integral_constant<int, 64>{});
    case 128: return go(std::integral_constant<int, 128>{});
    case 1024: return go(std::integral_constant<int, 1024>{});
    default: return go(std::integral_constant<int, 256>{});
  }
}

}  // namespace

// params.pcg_threads: 0 = 256, a size, or -1 = the fastest size for this (storage,
// problem count range, largest problem), timed once on the current system: each
// candidate launched once, then three times between two events, with no pose
// update, increment, statistics or trace written (only the flags the real solve
// would raise as well).  No timing while a graph is being captured.
int per_problem_pcg_threads(Context& c, bool may_time, int iters) {
  if (c.pcg_threads > 0) return c.pcg_threads;
  if (c.pcg_threads == 0) return 256;
  int bucket = 0;
  while (bucket < 40 && (1LL << bucket) < c.shape.nseg) ++bucket;
  const long long key = ((long long)c.shape.max_seg_free * 64 + bucket) * 2 + c.pcg_storage;
  auto it = c.pcg_threads_timed.find(key);
  if (it != c.pcg_threads_timed.end()) return it->second;
  if (!may_time || c.in_capture || iters <= 0) return 256;
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  int best = 256;
  float best_ms = 1e30f;
  for (int nt : {64, 128, 256, 1024}) {
    if (!launch_per_problem(c, nt, iters, nullptr, nullptr, nullptr, nullptr, false)) continue;  // warm-up
    check_hip(hipEventRecord(e0, c.stream), "hipEventRecord");
    for (int r = 0; r < 3; ++r) launch_per_problem(c, nt, iters, nullptr, nullptr, nullptr, nullptr, false);
    check_hip(hipEventRecord(e1, c.stream), "hipEventRecord");
    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (ms < best_ms) {
      best_ms = ms;
      best = nt;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.pcg_threads_timed[key] = best;
  return best;
}

void launch_solve(Context& c, int iters, double* trace_slot, double* delta_out, double* poses_inout, double* stats,
                  bool update_poses, bool sparse_matrix_free) {
  if (c.shape.nfree == 0) return;
  auto dist = [&](bool mf) {
    return c.pcg_storage == 1
               ? launch_solve_dist_any<double>(c, mf, iters, trace_slot, delta_out, poses_inout, stats, update_poses,
                                               c.diag64.as<double>(), c.minv64.as<double>(), c.hij64.as<double>(),
                                               c.pcg_vec.as<double>())
               : launch_solve_dist_any<float>(c, mf, iters, trace_slot, delta_out, poses_inout, stats, update_poses,
                                              c.diag32.as<float>(), c.minv32.as<float>(), c.hij32.as<float>(),
                                              c.pcg_vec.as<float>());
  };
  if (sparse_matrix_free) {
    if (c.solve_mode != 0 && c.solve_mode != 5)
      fail(BF_ERR_UNSUPPORTED, "the matrix-free sparse term runs in the distributed-vector PCG (solve_kernel 0 or 5)");
    if (c.shape.nseg > 1) fail(BF_ERR_UNSUPPORTED, "the matrix-free sparse term solves one problem at a time");
    if (!dist(true)) fail(BF_ERR_UNSUPPORTED, "the search direction does not fit in one workgroup's LDS");
    return;
  }
  const bool many = c.shape.nseg > 1;
  if (many && c.solve_mode != 0 && c.solve_mode != 4)
    fail(BF_ERR_UNSUPPORTED, "several problems are solved by the per-problem kernel (solve_kernel 0 or 4)");
  if (solve_per_problem(c)) {
    const int nt = per_problem_pcg_threads(c, true, iters);
    if (launch_per_problem(c, nt, iters, trace_slot, delta_out, poses_inout, stats, update_poses)) {
      c.pcg_threads_last = nt;
      return;
    }
    fail(BF_ERR_UNSUPPORTED, "a problem's PCG vectors do not fit in one workgroup's LDS");
  }
  if (c.solve_mode == 0 || c.solve_mode == 3) {
    bool ok = c.pcg_storage == 1
                  ? launch_solve_rep<double>(c, iters, trace_slot, delta_out, poses_inout, stats, update_poses,
                                             c.diag64.as<double>(), c.minv64.as<double>(), c.hij64.as<double>(),
                                             c.pcg_vec.as<double>())
                  : launch_solve_rep<float>(c, iters, trace_slot, delta_out, poses_inout, stats, update_poses,
                                            c.diag32.as<float>(), c.minv32.as<float>(), c.hij32.as<float>(),
                                            c.pcg_vec.as<float>());
    if (ok) return;
    if (c.solve_mode == 3) fail(BF_ERR_UNSUPPORTED, "replicated-vector solve does not fit");
  }
  if (c.solve_mode == 0 || c.solve_mode == 5) {
    if (dist(false)) return;
    if (c.solve_mode == 5) fail(BF_ERR_UNSUPPORTED, "the search direction does not fit in one workgroup's LDS");
  }
  if (c.solve_mode == 1) {
    bool ok = c.pcg_storage == 1
                  ? launch_solve_single<double, 1024>(c, iters, trace_slot, delta_out, poses_inout, stats,
                                                      update_poses, c.diag64.as<double>(), c.minv64.as<double>(),
                                                      c.hij64.as<double>())
                  : launch_solve_single<float, 1024>(c, iters, trace_slot, delta_out, poses_inout, stats,
                                                     update_poses, c.diag32.as<float>(), c.minv32.as<float>(),
                                                     c.hij32.as<float>());
    if (ok) return;
    if (c.solve_mode == 1) fail(BF_ERR_UNSUPPORTED, "PCG vectors do not fit in one workgroup's LDS");
  }
  if (c.pcg_storage == 1)
    launch_solve_coop<double>(c, iters, trace_slot, delta_out, poses_inout, stats, update_poses,
                              c.diag64.as<double>(), c.minv64.as<double>(), c.hij64.as<double>(),
                              c.pcg_vec.as<double>());
  else
    launch_solve_coop<float>(c, iters, trace_slot, delta_out, poses_inout, stats, update_poses, c.diag32.as<float>(),
                             c.minv32.as<float>(), c.hij32.as<float>(), c.pcg_vec.as<float>());
}

// The eight energy words of a single problem with more than kEnergySplit edges.
void launch_energy_split(Context& c, double* dst8) {
  const long long E = c.shape.E;
  long long chunk = (E + kEnergyMaxParts - 1) / kEnergyMaxParts;
  if (chunk < 2048) chunk = 2048;
  const int nparts = (int)((E + chunk - 1) / chunk);
  ensure(c.energy_parts, sizeof(double) * 8 * kEnergyMaxParts);
  hipLaunchKernelGGL(k_energy_parts, dim3((unsigned)nparts), dim3(256), 0, c.stream, c.eblocks.as<double>(), E, chunk,
                     c.energy_parts.as<double>());
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, c.stream, c.energy_parts.as<double>(), nparts, dst8);
}

void launch_energy(Context& c, double* dst8) {
  if (c.shape.nseg == 1 && c.shape.E > kEnergySplit) {
    launch_energy_split(c, dst8);
    return;
  }
  hipLaunchKernelGGL(k_energy, dim3(c.shape.nseg), dim3(256), 0, c.stream, c.eblocks.as<double>(),
                     c.seg_edge_ptr.as<long long>(), dst8);
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
