// Device-side helpers shared by the kernels of libbf.
//
// Decision arithmetic (which pixels associate, which frame pairs exist) is
// written as a fixed operation sequence, so that it is reproducible bit for bit
// from run to run: FP32 with explicit fused multiply-adds (and no other
// contraction) for the per-pixel association, FP64 without contraction for the
// pair test and the relative poses.  Everything else may use fused multiply-add.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bf.h"

namespace bf {

constexpr int kRecWords = 32;     // per dense pair job record (doubles)
constexpr int kRecG = 21;         // offset of J^T r in a record
constexpr int kRecEg = 27, kRecEp = 28, kRecNg = 29, kRecNp = 30;
constexpr int kEdgeWords = 128;   // per edge block record (doubles)
constexpr int kEHii = 0, kEHjj = 36, kEHij = 72, kEGi = 108, kEGj = 114;
constexpr int kEEs = 120, kEEg = 121, kEEp = 122, kENs = 123, kENg = 124, kENp = 125;
constexpr int kMomWords = 36;     // per sparse pair moments (doubles)
// moments layout: n, sum p (3), sum q (3), sum p p^T (9), sum q q^T (9), sum p q^T (9)
constexpr int kMN = 0, kMP = 1, kMQ = 4, kMPP = 7, kMQQ = 16, kMPQ = 25;

// Error flags raised by kernels, read back at the next synchronisation.
enum DeviceFlag : int {
  kFlagBadIndex = 1,
  kFlagNonFinite = 2,
  kFlagNotPD = 4,
  kFlagUnsorted = 8,
  kFlagTimeout = 16,
  kFlagShape = 32  // a problem the chosen PCG kernel cannot split (its launch then computes nothing usable)
};

struct Intr32 {
  float fx, fy, cx, cy;
  int W, H;
};

// T_ji = T_j^-1 T_i for row-major 4x4 camera-to-world poses, FP64, fixed order:
//   R[a][b] = (Rj[0][a]*Ri[0][b] + Rj[1][a]*Ri[1][b]) + Rj[2][a]*Ri[2][b]
//   d = t_i - t_j,  t[a] = (Rj[0][a]*d0 + Rj[1][a]*d1) + Rj[2][a]*d2
__device__ __forceinline__ void relative_pose_nc(const double* __restrict__ Ti, const double* __restrict__ Tj,
                                                 double R[9], double t[3]) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      R[3 * a + b] = (Tj[0 * 4 + a] * Ti[0 * 4 + b] + Tj[1 * 4 + a] * Ti[1 * 4 + b]) + Tj[2 * 4 + a] * Ti[2 * 4 + b];
  double d0 = Ti[3] - Tj[3], d1 = Ti[7] - Tj[7], d2 = Ti[11] - Tj[11];
  for (int a = 0; a < 3; ++a) t[a] = (Tj[0 * 4 + a] * d0 + Tj[1 * 4 + a] * d1) + Tj[2 * 4 + a] * d2;
}

// FP32 association arithmetic, a fixed sequence of fused multiply-adds (each
// a*b + c rounded once; plain products and sums are never contracted):
// c = R d + t row-wise, c_a = fma(R_a0, d.x, fma(R_a1, d.y, fma(R_a2, d.z, t_a))).
__device__ __forceinline__ float3 xform32(const float* R, const float* t, float3 d) {
  float3 c;
  c.x = __builtin_fmaf(R[0], d.x, __builtin_fmaf(R[1], d.y, __builtin_fmaf(R[2], d.z, t[0])));
  c.y = __builtin_fmaf(R[3], d.x, __builtin_fmaf(R[4], d.y, __builtin_fmaf(R[5], d.z, t[1])));
  c.z = __builtin_fmaf(R[6], d.x, __builtin_fmaf(R[7], d.y, __builtin_fmaf(R[8], d.z, t[2])));
  return c;
}

// m = R n, m_a = fma(R_a0, n.x, fma(R_a1, n.y, R_a2 * n.z))
__device__ __forceinline__ float3 rotate32(const float* R, float3 n) {
#pragma clang fp contract(off)
  float3 m;
  m.x = __builtin_fmaf(R[0], n.x, __builtin_fmaf(R[1], n.y, R[2] * n.z));
  m.y = __builtin_fmaf(R[3], n.x, __builtin_fmaf(R[4], n.y, R[5] * n.z));
  m.z = __builtin_fmaf(R[6], n.x, __builtin_fmaf(R[7], n.y, R[8] * n.z));
  return m;
}

// a.b = fma(a.x, b.x, fma(a.y, b.y, a.z * b.z))
__device__ __forceinline__ float dot32(float3 a, float3 b) {
#pragma clang fp contract(off)
  return __builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, a.z * b.z));
}

// u = fma(f * c, iz, cc)
__device__ __forceinline__ float project32(float f, float c, float iz, float cc) {
#pragma clang fp contract(off)
  return __builtin_fmaf(f * c, iz, cc);
}

__device__ __forceinline__ float mul_nc(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}

__device__ __forceinline__ bool is_nan(float x) { return !(x == x); }

// SE(3) exponential of xi = (omega, v): Rodrigues' formula and the matching V
// matrix, Taylor series through theta^6 below theta = 1e-2.  Out: row-major 3x4.
__device__ inline void exp_se3(const double xi[6], double R[9], double tv[3]) {
  double wx = xi[0], wy = xi[1], wz = xi[2];
  double th2 = wx * wx + wy * wy + wz * wz;
  double A, B, C;
  if (th2 < 1e-4) {
    double t4 = th2 * th2;
    A = 1.0 - th2 / 6.0 + t4 / 120.0 - t4 * th2 / 5040.0;
    B = 0.5 - th2 / 24.0 + t4 / 720.0 - t4 * th2 / 40320.0;
    C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t4 * th2 / 362880.0;
  } else {
    double th = sqrt(th2);
    double s = sin(th), c = cos(th);
    A = s / th;
    B = (1.0 - c) / th2;
    C = (th - s) / (th2 * th);
  }
  // W = [w]x, W2 = W W = w w^T - th2 I
  double W[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
  double W2[9] = {wx * wx - th2, wx * wy, wx * wz, wy * wx, wy * wy - th2, wy * wz, wz * wx, wz * wy, wz * wz - th2};
  double V[9];
  for (int k = 0; k < 9; ++k) {
    double I = (k % 4 == 0) ? 1.0 : 0.0;
    R[k] = I + A * W[k] + B * W2[k];
    V[k] = I + B * W[k] + C * W2[k];
  }
  for (int a = 0; a < 3; ++a) tv[a] = V[3 * a] * xi[3] + V[3 * a + 1] * xi[4] + V[3 * a + 2] * xi[5];
}

// Preconditioner block of a frame's 6x6 diagonal block, in place: 1 = inverted;
// 0 = the block is identically zero (no residual touches the frame at these poses),
// A stays zero so the frame is inert in the PCG (its gradient is zero too, so its
// increment stays zero); -1 = not positive definite.
// With `scalar` the preconditioner is the paper's Jacobi one (Sec. 4.4): only the
// diagonal entries, inverted one by one (a non-positive one is -1).
__device__ inline bool spd_inverse6(double* A);
__device__ inline int block_jacobi_inverse6(double* A, int scalar) {
  bool zero = true;
  for (int q = 0; q < 36; ++q) zero = zero && A[q] == 0.0;
  if (zero) return 0;
  if (scalar) {
    for (int q = 0; q < 36; ++q) {
      if (q % 7 == 0) {
        if (!(A[q] > 0.0)) return -1;
        A[q] = 1.0 / A[q];
      } else {
        A[q] = 0.0;
      }
    }
    return 1;
  }
  return spd_inverse6(A) ? 1 : -1;
}

// In-place 6x6 Cholesky inverse of a symmetric positive definite matrix (row-major).
// Returns false if a pivot is not positive.  One reciprocal per pivot, used as a
// multiplier wherever the factorisation and the triangular inverse divide by it.
__device__ inline bool spd_inverse6(double* A) {
  double L[36], inv_d[6];
  for (int k = 0; k < 36; ++k) L[k] = 0.0;
  for (int j = 0; j < 6; ++j) {
    double s = A[6 * j + j];
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 0.0)) return false;
    const double d = sqrt(s);
    L[6 * j + j] = d;
    inv_d[j] = 1.0 / d;
    for (int i = j + 1; i < 6; ++i) {
      double v = A[6 * i + j];
      for (int k = 0; k < j; ++k) v -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = v * inv_d[j];
    }
  }
  // Li = L^-1 (lower), A^-1 = Li^T Li
  double Li[36];
  for (int k = 0; k < 36; ++k) Li[k] = 0.0;
  for (int i = 0; i < 6; ++i) {
    Li[6 * i + i] = inv_d[i];
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[6 * i + k] * Li[6 * k + j];
      Li[6 * i + j] = -s * inv_d[i];
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
      for (int k = (i > j ? i : j); k < 6; ++k) s += Li[6 * k + i] * Li[6 * k + j];
      A[6 * i + j] = s;
    }
  return true;
}

__device__ __forceinline__ void raise_flag(int* flags, int f) { atomicOr(flags, f); }

}  // namespace bf
