// Key-point correspondence filter and surface-area filter (paper Sec. 4.1.1).
//
// One wavefront per frame pair, the pair's correspondences in input order (the
// order of match distance).  Candidates are added one at a time; after each
// addition, while the current set has at least three members, the rigid
// transform q = R p + t of least RMSD over the set is computed (Kabsch: SVD of
// the cross-covariance through the eigen-decomposition of H^T H), and the set
// passes when its largest residual |R p + t - q| is at most max_res and the
// transform is well determined: the ratio of the largest to the second largest
// eigenvalue of the covariance of the p's and of the q's, and of the largest to
// the second largest singular value of the cross-covariance, are at most
// max_cond.  While it fails, the member with the largest residual is removed
// (ties: the earliest).  The pair keeps its final set only if that passed and
// has at least max(min_count, 3) members, and if the p's and the q's each span
// at least min_area along their two principal axes (extent x extent).
//
// All sums are FP64 in a fixed order (lanes striding over the candidates, then
// a butterfly); every lane computes the 3x3 algebra redundantly.
#include "internal.h"

namespace bf {

namespace {

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Eigen-decomposition of a symmetric 3x3 matrix (row-major) by cyclic Jacobi
// rotations: eigenvalues w descending, eigenvectors as the columns of V.
__device__ void sym_eig3(const double* A, double* w, double* V) {
  double a[9];
  for (int k = 0; k < 9; ++k) a[k] = A[k];
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
    const double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
    if (!(off > 1e-32 * dia)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = a[3 * p + q];
      if (apq == 0.0) continue;
      const double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) {  // columns p, q
        const double akp = a[3 * k + p], akq = a[3 * k + q];
        a[3 * k + p] = c * akp - s * akq;
        a[3 * k + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {  // rows p, q
        const double apk = a[3 * p + k], aqk = a[3 * q + k];
        a[3 * p + k] = c * apk - s * aqk;
        a[3 * q + k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[3 * k + p], vkq = V[3 * k + q];
        V[3 * k + p] = c * vkp - s * vkq;
        V[3 * k + q] = s * vkp + c * vkq;
      }
    }
  }
  w[0] = a[0];
  w[1] = a[4];
  w[2] = a[8];
  for (int i = 0; i < 2; ++i)  // sort descending, columns along
    for (int j = 0; j < 2 - i; ++j)
      if (w[j] < w[j + 1]) {
        const double tw = w[j];
        w[j] = w[j + 1];
        w[j + 1] = tw;
        for (int k = 0; k < 3; ++k) {
          const double tv = V[3 * k + j];
          V[3 * k + j] = V[3 * k + j + 1];
          V[3 * k + j + 1] = tv;
        }
      }
}

__device__ __forceinline__ double ratio(double a, double b) { return b > 0.0 ? a / b : __builtin_inf(); }

struct PairPts {
  const int* fi;
  const int* fj;
  const float* pi;
  const float* pj;
  const long long* perm;
  long long base;
  __device__ void get(long long k, double* p, double* q) const {
    const long long c = perm[base + k];
    const bool sw = fi[c] > fj[c];
    const float* P = sw ? pj : pi;
    const float* Q = sw ? pi : pj;
    for (int a = 0; a < 3; ++a) {
      p[a] = P[3 * c + a];
      q[a] = Q[3 * c + a];
    }
  }
};

__global__ void __launch_bounds__(64) k_keypoint_filter(const int* __restrict__ fi, const int* __restrict__ fj,
                                                        const float* __restrict__ pi, const float* __restrict__ pj,
                                                        const long long* __restrict__ perm,
                                                        const long long* __restrict__ ptr, long long S,
                                                        double max_res, double max_cond, int min_count,
                                                        double min_area, int cond_mode, uint8_t* keep) {
  const long long g = blockIdx.x;
  if (g >= S) return;
  const int lane = threadIdx.x;
  const PairPts pts{fi, fj, pi, pj, perm, ptr[g]};
  const long long n = ptr[g + 1] - ptr[g];
  for (long long k = lane; k < n; k += 64) keep[perm[pts.base + k]] = 0;
  __syncthreads();
  long long cnt = 0;
  bool ok = false;
  double Vp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Vq[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double pm[3] = {0, 0, 0}, qm[3] = {0, 0, 0};
  for (long long cand = 0; cand < n; ++cand) {
    if (lane == 0) keep[perm[pts.base + cand]] = 1;
    ++cnt;
    __syncthreads();
    ok = false;
    while (cnt >= 3) {
      // means over the members among candidates 0..cand
      double s[6] = {0, 0, 0, 0, 0, 0};
      for (long long k = lane; k <= cand; k += 64) {
        if (!keep[perm[pts.base + k]]) continue;
        double p[3], q[3];
        pts.get(k, p, q);
        for (int a = 0; a < 3; ++a) {
          s[a] += p[a];
          s[3 + a] += q[a];
        }
      }
      for (int a = 0; a < 3; ++a) {
        pm[a] = wsum(s[a]) / (double)cnt;
        qm[a] = wsum(s[3 + a]) / (double)cnt;
      }
      // centered second moments
      double m[21];
      for (int k = 0; k < 21; ++k) m[k] = 0.0;
      for (long long k = lane; k <= cand; k += 64) {
        if (!keep[perm[pts.base + k]]) continue;
        double p[3], q[3];
        pts.get(k, p, q);
        for (int a = 0; a < 3; ++a) {
          p[a] -= pm[a];
          q[a] -= qm[a];
        }
        int o = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) {
            m[o] += p[a] * p[b];
            m[6 + o] += q[a] * q[b];
            ++o;
          }
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) m[12 + 3 * a + b] += p[a] * q[b];
      }
      for (int k = 0; k < 21; ++k) m[k] = wsum(m[k]);
      const double inv = 1.0 / (double)cnt;
      double Cp[9], Cq[9], H[9];
      {
        int o = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) {
            Cp[3 * a + b] = Cp[3 * b + a] = m[o] * inv;
            Cq[3 * a + b] = Cq[3 * b + a] = m[6 + o] * inv;
            ++o;
          }
        for (int k = 0; k < 9; ++k) H[k] = m[12 + k];
      }
      double wp[3], wq[3];
      sym_eig3(Cp, wp, Vp);
      sym_eig3(Cq, wq, Vq);
      // Kabsch: H = U S V^T from the eigen-decomposition of H^T H
      double HtH[9], ws[3], V[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) HtH[3 * a + b] = H[a] * H[b] + H[3 + a] * H[3 + b] + H[6 + a] * H[6 + b];
      sym_eig3(HtH, ws, V);
      const double s0 = sqrt(fmax(ws[0], 0.0)), s1 = sqrt(fmax(ws[1], 0.0)), s2 = sqrt(fmax(ws[2], 0.0));
      // condition number: largest over second largest value (cond_mode 0), or over
      // the smallest (cond_mode 1, the plain definition)
      const int lo = cond_mode ? 2 : 1;
      const double cond = fmax(fmax(ratio(wp[0], wp[lo]), ratio(wq[0], wq[lo])), ratio(s0, cond_mode ? s2 : s1));
      double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      if (s1 > 0.0) {
        double U[9];
        for (int k = 0; k < 2; ++k) {
          const double sk = k == 0 ? s0 : s1;
          for (int a = 0; a < 3; ++a)
            U[3 * a + k] = (H[3 * a] * V[k] + H[3 * a + 1] * V[3 + k] + H[3 * a + 2] * V[6 + k]) / sk;
        }
        // orthonormalise the second column against the first, third = first x second
        double d01 = U[0] * U[1] + U[3] * U[4] + U[6] * U[7];
        for (int a = 0; a < 3; ++a) U[3 * a + 1] -= d01 * U[3 * a];
        double nn = sqrt(U[1] * U[1] + U[4] * U[4] + U[7] * U[7]);
        for (int a = 0; a < 3; ++a) U[3 * a + 1] /= nn;
        U[2] = U[3] * U[7] - U[6] * U[4];
        U[5] = U[6] * U[1] - U[0] * U[7];
        U[8] = U[0] * U[4] - U[3] * U[1];
        const double detV = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                            V[2] * (V[3] * V[7] - V[4] * V[6]);
        const double D[3] = {1.0, 1.0, detV >= 0.0 ? 1.0 : -1.0};
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            double r = 0.0;
            for (int k = 0; k < 3; ++k) r += V[3 * a + k] * D[k] * U[3 * b + k];
            R[3 * a + b] = r;
          }
      }
      double t[3];
      for (int a = 0; a < 3; ++a) t[a] = qm[a] - (R[3 * a] * pm[0] + R[3 * a + 1] * pm[1] + R[3 * a + 2] * pm[2]);
      // largest residual and its (earliest) member
      double best = -1.0;
      long long bk = -1;
      for (long long k = lane; k <= cand; k += 64) {
        if (!keep[perm[pts.base + k]]) continue;
        double p[3], q[3];
        pts.get(k, p, q);
        double e2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          const double d = R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2] + t[a] - q[a];
          e2 += d * d;
        }
        const double r = sqrt(e2);
        if (r > best) {
          best = r;
          bk = k;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const long long ok2 = __shfl_xor(bk, o);
        if (ob > best || (ob == best && ok2 >= 0 && (bk < 0 || ok2 < bk))) {
          best = ob;
          bk = ok2;
        }
      }
      if (best <= max_res && cond <= max_cond) {
        ok = true;
        break;
      }
      if (lane == 0) keep[perm[pts.base + bk]] = 0;
      --cnt;
      __syncthreads();
    }
  }
  bool pass = ok && cnt >= (min_count > 3 ? min_count : 3);
  if (pass) {
    // area of the p's and of the q's along their two principal axes
    double lo[4] = {1e300, 1e300, 1e300, 1e300}, hi[4] = {-1e300, -1e300, -1e300, -1e300};
    for (long long k = lane; k < n; k += 64) {
      if (!keep[perm[pts.base + k]]) continue;
      double p[3], q[3];
      pts.get(k, p, q);
      for (int ax = 0; ax < 2; ++ax) {
        const double up = (p[0] - pm[0]) * Vp[ax] + (p[1] - pm[1]) * Vp[3 + ax] + (p[2] - pm[2]) * Vp[6 + ax];
        const double uq = (q[0] - qm[0]) * Vq[ax] + (q[1] - qm[1]) * Vq[3 + ax] + (q[2] - qm[2]) * Vq[6 + ax];
        lo[ax] = fmin(lo[ax], up);
        hi[ax] = fmax(hi[ax], up);
        lo[2 + ax] = fmin(lo[2 + ax], uq);
        hi[2 + ax] = fmax(hi[2 + ax], uq);
      }
    }
    for (int k = 0; k < 4; ++k)
      for (int o = 32; o > 0; o >>= 1) {
        lo[k] = fmin(lo[k], __shfl_xor(lo[k], o));
        hi[k] = fmax(hi[k], __shfl_xor(hi[k], o));
      }
    const double ap = (hi[0] - lo[0]) * (hi[1] - lo[1]), aq = (hi[2] - lo[2]) * (hi[3] - lo[3]);
    pass = ap >= min_area && aq >= min_area;
  }
  if (!pass) {
    __syncthreads();
    for (long long k = lane; k < n; k += 64) keep[perm[pts.base + k]] = 0;
  }
}

}  // namespace

void launch_filters(Context& c, const bf_corrs& co, long long S, double max_res, double max_cond, int min_count,
                    double min_area, int cond_mode, uint8_t* keep) {
  if (S == 0) return;
  hipLaunchKernelGGL(k_keypoint_filter, dim3((unsigned)S), dim3(64), 0, c.stream, co.frame_i, co.frame_j, co.p_i,
                     co.p_j, c.corr_perm.as<long long>(), c.sparse_ptr.as<long long>(), S, max_res, max_cond,
                     min_count, min_area, cond_mode, keep);
}

}  // namespace bf
