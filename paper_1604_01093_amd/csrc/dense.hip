// Dense pair jobs (paper Sec. 4.3, E_geo and E_photo; Sec. 4.4: the dense part of
// J^T J is reduced locally and written once per pair).
//
// One workgroup per pair job (i -> j, source = lower index), one source pixel per
// lane per step.  For each pixel with a valid normal:
//   d = P_i(x,y), c = T_ji d, m = R_ji n                       (FP32, fixed order)
//   nearest pixel (floor(u+1/2), floor(v+1/2)) of pi(c) in frame j with a valid
//   normal, |c - q|^2 < tau_d^2 and m.N_j > tau_n               (FP32, fixed order)
//   r_g = m.(c - q),            J_g = [(m x q)^T, -m^T]
//   r_p = G_i(x,y) - G_j(pi(c)) (bilinear, photometric only where the geometric
//   association holds and the four taps and G_i are valid),
//   J_p = [(c x a)^T, a^T],  a = Jpi(c)^T grad G_j
// where J_g, J_p are the Jacobians with respect to the right perturbation of
// frame j.  The frame-i blocks follow per pair in FP64 from the adjoint
// (J_i = -J_j Ad(T_ji)), so each pixel feeds one 6x6 block: 21 + 6 + 4 values.
// Lane sums are FP32 (optionally two-sum compensated), combined across the
// workgroup in FP64 in a fixed order: the record is deterministic.
#include "internal.h"

namespace bf {

namespace {

struct Acc31 {
  float v[31];
};

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

template <bool JAC, bool KAHAN>
struct LaneAcc {
  static constexpr int N = JAC ? 31 : 4;
  float s[N];
  float c[KAHAN ? N : 1];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < (KAHAN ? N : 1); ++k) c[k] = 0.0f;
  }
  __device__ __forceinline__ void add(int k, float x) {
    if constexpr (KAHAN) kahan_add(s[k], c[k], x);
    else s[k] += x;
  }
  __device__ __forceinline__ double value(int k) const {
    if constexpr (KAHAN) return (double)s[k] - (double)c[k];
    else return (double)s[k];
  }
};

// Accumulate the outer products of the geometric and photometric Jacobians (both
// already scaled by the square root of their weights).
template <bool KAHAN>
__device__ __forceinline__ void accumulate_jac(LaneAcc<true, KAHAN>& A, const float* jg, float rg, const float* jp,
                                               float rp, float ph) {
  int k = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
#pragma unroll
    for (int b = a; b < 6; ++b) {
      A.add(k, jg[a] * jg[b] + jp[a] * jp[b]);
      ++k;
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) A.add(21 + a, jg[a] * rg + jp[a] * rp);
  A.add(27, rg * rg);
  A.add(28, rp * rp);
  A.add(29, 1.0f);
  A.add(30, ph);
}

template <bool JAC, bool KAHAN>
__global__ void __launch_bounds__(256) k_dense(const int* __restrict__ pairs, long long P,
                                               const float4* __restrict__ nd, const float* __restrict__ grad,
                                               const float* __restrict__ kx, const float* __restrict__ ky,
                                               const double* __restrict__ poses, Intr32 in, float tau_d2,
                                               float tau_n, float swg, float swp, double* __restrict__ records) {
  // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs, so give
  // each XCD a contiguous block of pair jobs (neighbouring jobs share frames and
  // stay in that XCD's L2).  The grid is a multiple of 8.
  const long long per = gridDim.x / 8;
  const long long p = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (p >= P) return;
  const int tid = threadIdx.x;
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const int W = in.W, H = in.H, HW = W * H;

  float R[9], t[3];
  {
    double Rd[9], td[3];
    relative_pose_nc(poses + (size_t)i * 16, poses + (size_t)j * 16, Rd, td);
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = (float)td[k];
  }
  const float4* __restrict__ ndi = nd + (size_t)i * HW;
  const float4* __restrict__ ndj = nd + (size_t)j * HW;
  const float* __restrict__ gi = grad + (size_t)i * HW;
  const float* __restrict__ gj = grad + (size_t)j * HW;
  const float fWm1 = (float)(W - 1), fHm1 = (float)(H - 1), fWm2 = (float)(W - 2), fHm2 = (float)(H - 2);

  LaneAcc<JAC, KAHAN> A;
  A.zero();

  int x = tid % W, y = tid / W;
  const int sx = blockDim.x % W, sy = blockDim.x / W;
  for (int pix = tid; pix < HW; pix += blockDim.x) {
    const int px = x, py = y;
    x += sx;
    y += sy;
    if (x >= W) {
      x -= W;
      y += 1;
    }
    const float4 s = ndi[pix];
    if (is_nan(s.x)) continue;
    const float D = s.w;
    const float3 d = make_float3(mul_nc(kx[px], D), mul_nc(ky[py], D), D);
    const float3 c = xform_nc(R, t, d);
    if (!(c.z > 0.0f)) continue;
    const float iz = 1.0f / c.z;
    const float u = project_nc(in.fx, c.x, iz, in.cx);
    const float v = project_nc(in.fy, c.y, iz, in.cy);
    const float xf = floorf(u + 0.5f), yf = floorf(v + 0.5f);
    if (!(xf >= 0.0f && xf <= fWm1 && yf >= 0.0f && yf <= fHm1)) continue;
    const int xh = (int)xf, yh = (int)yf;
    const float4 tq = ndj[yh * W + xh];
    if (is_nan(tq.x)) continue;
    const float3 q = make_float3(mul_nc(kx[xh], tq.w), mul_nc(ky[yh], tq.w), tq.w);
    const float3 e = make_float3(c.x - q.x, c.y - q.y, c.z - q.z);
    if (!(dot_nc(e, e) < tau_d2)) continue;
    const float3 n = make_float3(s.x, s.y, s.z);
    const float3 m = rotate_nc(R, n);
    if (!(dot_nc(m, make_float3(tq.x, tq.y, tq.z)) > tau_n)) continue;

    // geometric term
    const float rg = (m.x * e.x + m.y * e.y + m.z * e.z) * swg;
    // photometric term
    const float x0f = floorf(u), y0f = floorf(v);
    bool ph = x0f >= 0.0f && x0f <= fWm2 && y0f >= 0.0f && y0f <= fHm2;
    const float Gi = gi[pix];
    ph = ph && !is_nan(Gi);
    float g00 = 0.f, g10 = 0.f, g01 = 0.f, g11 = 0.f;
    if (ph) {
      const int t0 = (int)y0f * W + (int)x0f;
      g00 = gj[t0];
      g10 = gj[t0 + 1];
      g01 = gj[t0 + W];
      g11 = gj[t0 + W + 1];
      ph = !(is_nan(g00) || is_nan(g10) || is_nan(g01) || is_nan(g11));
    }
    float rp = 0.0f;
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (ph) {
      const float al = u - x0f, be = v - y0f;
      const float Gj = (1.0f - al) * ((1.0f - be) * g00 + be * g01) + al * ((1.0f - be) * g10 + be * g11);
      const float gu = ((1.0f - be) * (g10 - g00) + be * (g11 - g01)) * swp;
      const float gv = ((1.0f - al) * (g01 - g00) + al * (g11 - g10)) * swp;
      rp = (Gi - Gj) * swp;
      ax = gu * in.fx * iz;
      ay = gv * in.fy * iz;
      az = -(ax * c.x + ay * c.y) * iz;
    }
    if constexpr (JAC) {
      const float mx = m.x * swg, my = m.y * swg, mz = m.z * swg;
      const float jg[6] = {my * q.z - mz * q.y, mz * q.x - mx * q.z, mx * q.y - my * q.x, -mx, -my, -mz};
      const float jp[6] = {c.y * az - c.z * ay, c.z * ax - c.x * az, c.x * ay - c.y * ax, ax, ay, az};
      accumulate_jac<KAHAN>(A, jg, rg, jp, rp, ph ? 1.0f : 0.0f);
    } else {
      A.add(0, rg * rg);
      A.add(1, rp * rp);
      A.add(2, 1.0f);
      A.add(3, ph ? 1.0f : 0.0f);
    }
  }

  // Workgroup reduction in FP64, fixed order: 16 values at a time through LDS.
  __shared__ double red[16][256];
  __shared__ double part[16][16];
  __shared__ double out[32];
  constexpr int NV = LaneAcc<JAC, KAHAN>::N;
#pragma unroll
  for (int base = 0; base < 32; base += 16) {
    if (base < NV) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (base + k < NV) red[k][tid] = A.value(base + k);
      __syncthreads();
      const int k = tid >> 4, ch = tid & 15;
      if (base + k < NV) {
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l) sum += red[k][ch * 16 + l];
        part[k][ch] = sum;
      }
      __syncthreads();
      if (tid < 16 && base + tid < NV) {
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l) sum += part[tid][l];
        out[base + tid] = sum;
      }
      __syncthreads();
    }
  }
  if (tid < kRecWords) {
    double val = 0.0;
    if constexpr (JAC) {
      if (tid < 31) val = out[tid];
    } else {
      if (tid >= kRecEg && tid <= kRecNp) val = out[tid - kRecEg];
    }
    records[(size_t)p * kRecWords + tid] = val;
  }
}

}  // namespace

void launch_dense(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                  bool with_jacobians) {
  const long long P = c.shape.P;
  if (P == 0) return;
  Intr32 i32{(float)in.fx, (float)in.fy, (float)in.cx, (float)in.cy, in.width, in.height};
  float tau_d2 = (float)(prm.tau_dist * prm.tau_dist);
  float tau_n = (float)prm.tau_normal;
  float swg = (float)sqrt(wd * prm.w_geo);
  float swp = (float)sqrt(wd * prm.w_photo);
  unsigned grid = (unsigned)(8 * ((P + 7) / 8));
  const int* pr = c.pairs.as<int>();
  const float4* nd = c.nd.as<float4>();
  const float* g = c.grad.as<float>();
  double* rec = c.records.as<double>();
  const float* kx = c.kx.as<float>();
  const float* ky = c.ky.as<float>();
  if (with_jacobians) {
    if (prm.accumulate == 1)
      hipLaunchKernelGGL((k_dense<true, true>), dim3(grid), dim3(256), 0, c.stream, pr, P, nd, g, kx, ky, poses, i32,
                         tau_d2, tau_n, swg, swp, rec);
    else
      hipLaunchKernelGGL((k_dense<true, false>), dim3(grid), dim3(256), 0, c.stream, pr, P, nd, g, kx, ky, poses, i32,
                         tau_d2, tau_n, swg, swp, rec);
  } else {
    hipLaunchKernelGGL((k_dense<false, false>), dim3(grid), dim3(256), 0, c.stream, pr, P, nd, g, kx, ky, poses, i32,
                       tau_d2, tau_n, swg, swp, rec);
  }
}

}  // namespace bf
