// Dense pair jobs (paper Sec. 4.3, E_geo and E_photo; Sec. 4.4: the dense part of
// J^T J is reduced locally and written once per pair).
//
// One workgroup per pair job (i -> j, source = lower index), one source pixel per
// lane per step.  For each pixel with a valid normal:
//   d = P_i(x,y), c = T_ji d, m = R_ji n
//   nearest pixel (floor(u+1/2), floor(v+1/2)) of pi(c) in frame j with a valid
//   normal, |c - q|^2 < tau_d^2 and m.N_j > tau_n
//   r_g = m.(c - q),            J_g = [(m x q)^T, -m^T]
//   r_p = G_i(x,y) - G_j(pi(c)) (bilinear, photometric only where the geometric
//   association holds and the four taps and G_i are valid),
//   J_p = [(c x a)^T, a^T],  a = Jpi(c)^T grad G_j
// where J_g, J_p are the Jacobians with respect to the right perturbation of
// frame j.  The frame-i blocks follow per pair in FP64 from the adjoint
// (J_i = -J_j Ad(T_ji)), so each pixel feeds one 6x6 block: 21 + 6 + 4 values.
//
// The association decisions are always taken in FP32 with a fixed operation
// order and no contraction (reproducible bit for bit).  The residual/Jacobian
// values and their accumulation come in three precisions:
//   mode 0: FP32 values, FP32 lane sums;
//   mode 1: FP32 values, two-sum compensated FP32 lane sums;
//   mode 2: FP64 values (c, q, r, pi(c), Jacobians) and FP64 lane sums -- on
//           MI355X FP64 FMAs issue at the rate of unpacked FP32 FMAs.
// Lane sums are combined across the workgroup in FP64 in a fixed order through
// LDS: the record is deterministic for a given workgroup size.  The workgroup size (threads per pair
// job, 64..512) is a launch parameter; when the caller leaves it open it is chosen
// by timing the candidates once per image size, precision mode and job-count range.
#include <type_traits>

#include "internal.h"

namespace bf {

namespace {

__device__ __forceinline__ void two_sum_add(float& s, float& c, float x) {
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

template <int MODE, int N>
struct LaneAcc {
  using V = typename std::conditional<MODE == 2, double, float>::type;
  V s[N];
  V c[MODE == 1 ? N : 1];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] = (V)0;
#pragma unroll
    for (int k = 0; k < (MODE == 1 ? N : 1); ++k) c[k] = (V)0;
  }
  __device__ __forceinline__ void add(int k, V x) {
    if constexpr (MODE == 1) two_sum_add(s[k], c[k], x);
    else s[k] += x;
  }
  __device__ __forceinline__ double value(int k) const {
    if constexpr (MODE == 1) return (double)s[k] - (double)c[k];
    else return (double)s[k];
  }
};

template <int MODE, class V>
__device__ __forceinline__ void accumulate_jac(LaneAcc<MODE, 31>& A, const V* jg, V rg, const V* jp, V rp, V ph) {
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
  A.add(29, (V)1);
  A.add(30, ph);
}

__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int MODE, bool JAC, int NT>
__global__ void __launch_bounds__(NT) k_dense(const int* __restrict__ pairs, long long P,
                                               const float4* __restrict__ nd, const float* __restrict__ grad,
                                               const float* __restrict__ kx, const float* __restrict__ ky,
                                               const double* __restrict__ kx64, const double* __restrict__ ky64,
                                               const double* __restrict__ poses, Intr32 in, double fx64, double fy64,
                                               double cx64, double cy64, float tau_d2, float tau_n, double swg,
                                               double swp, double* __restrict__ records) {
  // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs, so give
  // each XCD a contiguous block of pair jobs (neighbouring jobs share frames and
  // stay in that XCD's L2).  The grid is a multiple of 8.
  const long long per = gridDim.x / 8;
  const long long p = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (p >= P) return;
  const int tid = threadIdx.x;
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const int W = in.W, H = in.H, HW = W * H;

  // relative pose: FP64 (fixed order), FP32 copy for the decisions; wave-uniform
  float R[9], t[3];
  double Rd[9], td[3];
  relative_pose_nc(poses + (size_t)i * 16, poses + (size_t)j * 16, Rd, td);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R[k] = uniform_f((float)Rd[k]);
    Rd[k] = uniform_d(Rd[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    t[k] = uniform_f((float)td[k]);
    td[k] = uniform_d(td[k]);
  }
  const float4* __restrict__ ndi = nd + (size_t)i * HW;
  const float4* __restrict__ ndj = nd + (size_t)j * HW;
  const float* __restrict__ gi = grad + (size_t)i * HW;
  const float* __restrict__ gj = grad + (size_t)j * HW;
  const float fWm1 = (float)(W - 1), fHm1 = (float)(H - 1), fWm2 = (float)(W - 2), fHm2 = (float)(H - 2);

  constexpr int NV = JAC ? 31 : 4;
  LaneAcc<MODE, NV> A;
  A.zero();
  using V = typename LaneAcc<MODE, NV>::V;

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
    // ---- FP32 association decisions (fixed operation order)
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

    // ---- residuals and Jacobians w.r.t. frame j
    V rg, rp = (V)0, jg[6], jp[6] = {(V)0, (V)0, (V)0, (V)0, (V)0, (V)0};
    if constexpr (MODE == 2) {
      const double D64 = (double)D, Dj = (double)tq.w;
      const double dx = kx64[px] * D64, dy = ky64[py] * D64;
      const double cx_ = Rd[0] * dx + Rd[1] * dy + Rd[2] * D64 + td[0];
      const double cy_ = Rd[3] * dx + Rd[4] * dy + Rd[5] * D64 + td[1];
      const double cz_ = Rd[6] * dx + Rd[7] * dy + Rd[8] * D64 + td[2];
      const double qx = kx64[xh] * Dj, qy = ky64[yh] * Dj, qz = Dj;
      const double nx = n.x, ny = n.y, nz = n.z;
      const double mx = Rd[0] * nx + Rd[1] * ny + Rd[2] * nz;
      const double my = Rd[3] * nx + Rd[4] * ny + Rd[5] * nz;
      const double mz = Rd[6] * nx + Rd[7] * ny + Rd[8] * nz;
      rg = (mx * (cx_ - qx) + my * (cy_ - qy) + mz * (cz_ - qz)) * swg;
      const double sx_ = mx * swg, sy_ = my * swg, sz_ = mz * swg;
      jg[0] = sy_ * qz - sz_ * qy;
      jg[1] = sz_ * qx - sx_ * qz;
      jg[2] = sx_ * qy - sy_ * qx;
      jg[3] = -sx_;
      jg[4] = -sy_;
      jg[5] = -sz_;
      if (ph) {
        const double iz64 = 1.0 / cz_;
        const double u64 = fx64 * cx_ * iz64 + cx64;
        const double v64 = fy64 * cy_ * iz64 + cy64;
        const double al = u64 - (double)x0f, be = v64 - (double)y0f;
        const double G00 = g00, G10 = g10, G01 = g01, G11 = g11;
        const double Gj = (1.0 - al) * ((1.0 - be) * G00 + be * G01) + al * ((1.0 - be) * G10 + be * G11);
        const double gu = ((1.0 - be) * (G10 - G00) + be * (G11 - G01)) * swp;
        const double gv = ((1.0 - al) * (G01 - G00) + al * (G11 - G10)) * swp;
        rp = ((double)Gi - Gj) * swp;
        const double ax = gu * fx64 * iz64, ay = gv * fy64 * iz64;
        const double az = -(ax * cx_ + ay * cy_) * iz64;
        jp[0] = cy_ * az - cz_ * ay;
        jp[1] = cz_ * ax - cx_ * az;
        jp[2] = cx_ * ay - cy_ * ax;
        jp[3] = ax;
        jp[4] = ay;
        jp[5] = az;
      }
    } else {
      const float fswg = (float)swg, fswp = (float)swp;
      rg = (m.x * e.x + m.y * e.y + m.z * e.z) * fswg;
      const float mx = m.x * fswg, my = m.y * fswg, mz = m.z * fswg;
      jg[0] = my * q.z - mz * q.y;
      jg[1] = mz * q.x - mx * q.z;
      jg[2] = mx * q.y - my * q.x;
      jg[3] = -mx;
      jg[4] = -my;
      jg[5] = -mz;
      if (ph) {
        const float al = u - x0f, be = v - y0f;
        const float Gj = (1.0f - al) * ((1.0f - be) * g00 + be * g01) + al * ((1.0f - be) * g10 + be * g11);
        const float gu = ((1.0f - be) * (g10 - g00) + be * (g11 - g01)) * fswp;
        const float gv = ((1.0f - al) * (g01 - g00) + al * (g11 - g10)) * fswp;
        rp = (Gi - Gj) * fswp;
        const float ax = gu * in.fx * iz, ay = gv * in.fy * iz;
        const float az = -(ax * c.x + ay * c.y) * iz;
        jp[0] = c.y * az - c.z * ay;
        jp[1] = c.z * ax - c.x * az;
        jp[2] = c.x * ay - c.y * ax;
        jp[3] = ax;
        jp[4] = ay;
        jp[5] = az;
      }
    }
    if constexpr (JAC) {
      accumulate_jac<MODE, V>(A, jg, rg, jp, rp, ph ? (V)1 : (V)0);
    } else {
      A.add(0, rg * rg);
      A.add(1, rp * rp);
      A.add(2, (V)1);
      A.add(3, ph ? (V)1 : (V)0);
    }
  }

  // Workgroup reduction in FP64, fixed order, 16 values at a time through LDS: with
  // 512 threads the upper half first adds onto the lower half; then each value's
  // RL lane sums are added in chunks of 16 lanes, and the chunk sums in order.
  constexpr int RL = NT < 256 ? NT : 256;
  constexpr int NCH = RL / 16;
  __shared__ double red[16][RL];
  __shared__ double part[16][NCH];
  __shared__ double out[32];
#pragma unroll
  for (int base = 0; base < 32; base += 16) {
    if (base < NV) {
      if constexpr (NT > RL) {
        if (tid >= RL)
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (base + k < NV) red[k][tid - RL] = A.value(base + k);
        __syncthreads();
        if (tid < RL)
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (base + k < NV) red[k][tid] = A.value(base + k) + red[k][tid];
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (base + k < NV) red[k][tid] = A.value(base + k);
      }
      __syncthreads();
      if (tid < RL) {
        const int k = tid / NCH, ch = tid % NCH;
        if (base + k < NV) {
          double sum = 0.0;
#pragma unroll
          for (int l = 0; l < 16; ++l) sum += red[k][ch * 16 + l];
          part[k][ch] = sum;
        }
      }
      __syncthreads();
      if (tid < 16 && base + tid < NV) {
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < NCH; ++l) sum += part[tid][l];
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

template <int MODE, bool JAC, int NT>
void launch_nt(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd) {
  const long long P = c.shape.P;
  Intr32 i32{(float)in.fx, (float)in.fy, (float)in.cx, (float)in.cy, in.width, in.height};
  float tau_d2 = (float)(prm.tau_dist * prm.tau_dist);
  float tau_n = (float)prm.tau_normal;
  double swg = sqrt(wd * prm.w_geo);
  double swp = sqrt(wd * prm.w_photo);
  unsigned grid = (unsigned)(8 * ((P + 7) / 8));
  hipLaunchKernelGGL((k_dense<MODE, JAC, NT>), dim3(grid), dim3(NT), 0, c.stream, c.pairs.as<int>(), P,
                     c.nd.as<float4>(), c.grad.as<float>(), c.kx.as<float>(), c.ky.as<float>(), c.kx64.as<double>(),
                     c.ky64.as<double>(), poses, i32, in.fx, in.fy, in.cx, in.cy, tau_d2, tau_n, swg, swp,
                     c.records.as<double>());
}

template <int MODE, bool JAC>
void launch_mode(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd, int nt) {
  switch (nt) {
    case 64: launch_nt<MODE, JAC, 64>(c, in, poses, prm, wd); break;
    case 128: launch_nt<MODE, JAC, 128>(c, in, poses, prm, wd); break;
    case 512: launch_nt<MODE, JAC, 512>(c, in, poses, prm, wd); break;
    default: launch_nt<MODE, JAC, 256>(c, in, poses, prm, wd); break;
  }
}

void launch_any(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                bool jac, int nt) {
  const int mode = prm.accumulate;
  if (jac) {
    if (mode == 2) launch_mode<2, true>(c, in, poses, prm, wd, nt);
    else if (mode == 1) launch_mode<1, true>(c, in, poses, prm, wd, nt);
    else launch_mode<0, true>(c, in, poses, prm, wd, nt);
  } else {
    if (mode == 2) launch_mode<2, false>(c, in, poses, prm, wd, nt);
    else launch_mode<0, false>(c, in, poses, prm, wd, nt);
  }
}

// Threads per pair job for this launch: the caller's choice, or the fastest of the
// candidates, timed once per (pixels per frame, precision mode, Jacobians, range of
// job counts) in this context.  Timing runs the real launch (it only rewrites the
// records) and synchronises the stream once.
int choose_threads(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                   bool jac) {
  if (prm.dense_threads != 0) return prm.dense_threads;
  int bucket = 0;
  while (bucket < 40 && (1LL << bucket) < c.shape.P) ++bucket;
  const long long key = (((long long)in.width * in.height * 4 + prm.accumulate) * 2 + (jac ? 1 : 0)) * 64 + bucket;
  auto it = c.dense_threads.find(key);
  if (it != c.dense_threads.end()) return it->second;
  static const int cand[4] = {64, 128, 256, 512};
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  int best = 256;
  float best_ms = 1e30f;
  for (int nt : cand) {
    launch_any(c, in, poses, prm, wd, jac, nt);  // warm-up
    check_hip(hipEventRecord(e0, c.stream), "hipEventRecord");
    for (int r = 0; r < 3; ++r) launch_any(c, in, poses, prm, wd, jac, nt);
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
  c.dense_threads[key] = best;
  return best;
}

}  // namespace

void launch_dense(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                  bool with_jacobians) {
  if (c.shape.P == 0) return;
  const int nt = choose_threads(c, in, poses, prm, wd, with_jacobians);
  launch_any(c, in, poses, prm, wd, with_jacobians, nt);
}

}  // namespace bf
