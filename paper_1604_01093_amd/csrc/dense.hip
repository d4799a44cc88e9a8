// Dense pair jobs (paper Sec. 4.3, E_geo and E_photo; Sec. 4.4: the dense part of
// J^T J is reduced locally and written once per pair).
//
// One workgroup per pair job (i -> j, source = lower index; with both directions
// per pair a second job j -> i), one source pixel per
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
// The association decisions are always taken in FP32 with a fixed sequence of
// fused multiply-adds (reproducible bit for bit); they agree with the rule
// evaluated exactly except where a tested quantity lies within its FP32 rounding
// error of the threshold (a pixel within ~1e-5 px of a rounding tie, a distance
// within ~1e-6 m of tau_d, ...).  The decisions can be written out per pixel for
// inspection.  The residual/Jacobian values and their accumulation come in three
// precisions:
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

// Load base[i] with a 32-bit byte offset from a wavefront-uniform base (one
// scalar base plus a vector offset: no 64-bit address arithmetic per lane).
template <class T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
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

// Per-lane accumulation of one associated pixel's residuals and Jacobians.
template <int MODE, bool JAC, class Acc>
__device__ __forceinline__ void pixel_terms(Acc& A, const float* w, const float* R, const float* t,
                                            const double* Rd, const double* td, const double* __restrict__ kx64,
                                            const double* __restrict__ ky64, const Intr32& in, double fx64,
                                            double fy64, double cx64, double cy64, double swg, double swp) {
  using V = typename Acc::V;
  V rg, rp = (V)0, jg[6], jp[6] = {(V)0, (V)0, (V)0, (V)0, (V)0, (V)0};
  bool ph;
  if constexpr (MODE == 2) {
    // payload: D, Dj, n(3), px, py, xh, yh, x0, y0, Gi, taps(4)
    const double D64 = (double)w[0], Dj = (double)w[1];
    const int px = (int)w[5], py = (int)w[6], xh = (int)w[7], yh = (int)w[8];
    const double x0f = (double)w[9], y0f = (double)w[10];
    const float Gi = w[11];
    ph = !is_nan(Gi);
    const double dx = kx64[px] * D64, dy = ky64[py] * D64;
    const double cx_ = Rd[0] * dx + Rd[1] * dy + Rd[2] * D64 + td[0];
    const double cy_ = Rd[3] * dx + Rd[4] * dy + Rd[5] * D64 + td[1];
    const double cz_ = Rd[6] * dx + Rd[7] * dy + Rd[8] * D64 + td[2];
    const double qx = kx64[xh] * Dj, qy = ky64[yh] * Dj, qz = Dj;
    const double nx = w[2], ny = w[3], nz = w[4];
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
      const double al = u64 - x0f, be = v64 - y0f;
      const double G00 = w[12], G10 = w[13], G01 = w[14], G11 = w[15];
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
    // payload: c(3), m(3), q(3), bilinear weights (u - x0, v - y0), Gi, taps(4)
    const float cx = w[0], cy = w[1], cz = w[2], mx0 = w[3], my0 = w[4], mz0 = w[5];
    const float qx = w[6], qy = w[7], qz = w[8], al = w[9], be = w[10], Gi = w[11];
    ph = !is_nan(Gi);
    const float fswg = (float)swg, fswp = (float)swp;
    rg = (mx0 * (cx - qx) + my0 * (cy - qy) + mz0 * (cz - qz)) * fswg;
    const float mx = mx0 * fswg, my = my0 * fswg, mz = mz0 * fswg;
    jg[0] = my * qz - mz * qy;
    jg[1] = mz * qx - mx * qz;
    jg[2] = mx * qy - my * qx;
    jg[3] = -mx;
    jg[4] = -my;
    jg[5] = -mz;
    if (ph) {
      const float iz = 1.0f / cz;
      const float g00 = w[12], g10 = w[13], g01 = w[14], g11 = w[15];
      const float Gj = (1.0f - al) * ((1.0f - be) * g00 + be * g01) + al * ((1.0f - be) * g10 + be * g11);
      const float gu = ((1.0f - be) * (g10 - g00) + be * (g11 - g01)) * fswp;
      const float gv = ((1.0f - al) * (g01 - g00) + al * (g11 - g10)) * fswp;
      rp = (Gi - Gj) * fswp;
      const float ax = gu * in.fx * iz, ay = gv * in.fy * iz;
      const float az = -(ax * cx + ay * cy) * iz;
      jp[0] = cy * az - cz * ay;
      jp[1] = cz * ax - cx * az;
      jp[2] = cx * ay - cy * ax;
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

// Payload words per queued pixel and queue slots per wavefront.
constexpr int kPayload = 16;
constexpr int kQueue = 128;

template <int MODE, bool JAC, int NT>
__global__ void __launch_bounds__(NT) k_dense(const int* __restrict__ pairs, long long P, int bidir, int tiles,
                                              const float4* __restrict__ nd, const float* __restrict__ grad,
                                              const float* __restrict__ kx, const float* __restrict__ ky,
                                              const double* __restrict__ kx64, const double* __restrict__ ky64,
                                              const double* __restrict__ poses, Intr32 in, double fx64, double fy64,
                                              double cx64, double cy64, float tau_d2, float tau_n, double swg,
                                              double swp, double* __restrict__ records,
                                              const unsigned* __restrict__ fixed,
                                              unsigned* __restrict__ assoc_out) {
  constexpr int NW = NT / 64;
  constexpr int RL = NT < 256 ? NT : 256;
  constexpr int NCH = RL / 16;
  constexpr size_t kQueueBytes = sizeof(float) * NW * kPayload * kQueue;
  constexpr size_t kRedBytes = sizeof(double) * (16 * RL + 16 * NCH + 32);
  // the per-wavefront queues and the final reduction share the workgroup's LDS
  __shared__ double smem[(kQueueBytes > kRedBytes ? kQueueBytes : kRedBytes) / sizeof(double)];

  // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs, so give
  // each XCD a contiguous block of pair jobs (neighbouring jobs share frames and
  // stay in that XCD's L2).  The grid is a multiple of 8.
  const long long per = gridDim.x / 8;
  const long long pt = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;  // tile of a pair job
  // jobs [0, P): pair p as (i -> j); with both directions, jobs [P, 2P): (j -> i);
  // job p's pixels are split into `tiles` contiguous tiles pt = p * tiles + tile
  const long long p = pt / tiles;
  if (p >= (bidir ? 2 * P : P)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rev = p >= P ? 1 : 0;
  const long long pp = p - (rev ? P : 0);
  const int i = pairs[2 * pp + rev], j = pairs[2 * pp + 1 - rev];
  const int W = in.W, H = in.H, HW = W * H;
  // this tile's pixels [lo, hi): tiles of whole wavefront steps
  const int tile_len = (((HW + tiles - 1) / tiles) + 63) & ~63;
  const int lo = (int)(pt - p * tiles) * tile_len;
  const int hi = min(HW, lo + tile_len);

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
  float* Q = reinterpret_cast<float*>(smem) + (size_t)wave * kPayload * kQueue;  // Q[k * kQueue + slot]
  int head = 0, tail = 0;  // wavefront-uniform queue positions

  // Wavefront w takes the pixels w*64 + lane + k*NT: first the FP32 association
  // decisions for every pixel, then the residual/Jacobian work only for the pixels
  // that passed, 64 at a time from the wavefront's queue (all lanes busy).  The
  // decisions are written without branches: every load is issued with clamped,
  // in-bounds indices (the target gather, the four gradient taps and G_i together,
  // right after the projection) and the tests only decide validity, so the loads of
  // a step overlap instead of waiting on each other; the source load of the next
  // step is issued before the current one is processed.
  // The source pixel's data and its ray factors (kx, ky) for the next step are
  // loaded one step ahead.  Past the last pixel (never valid) the row index runs
  // beyond the image: it is clamped for the load.
  int x = (lo + tid) % W, y = (lo + tid) / W;
  const int sx = NT % W, sy = NT / W;
  float4 s_next = ld_at(ndi, (unsigned)(lo + tid < hi ? lo + tid : HW - 1));
  float kx_next = ld_at(kx, (unsigned)x), ky_next = ld_at(ky, (unsigned)(y < H ? y : H - 1));
  for (int base = lo + wave * 64; base < hi; base += NT) {
    const int pix = base + lane;
    const int px = x, py = y;
    x += sx;
    y += sy;
    if (x >= W) {
      x -= W;
      y += 1;
    }
    const float4 s4 = s_next;
    const float kxp = kx_next, kyp = ky_next;
    {
      const int nxt = pix + NT;
      s_next = ld_at(ndi, (unsigned)(nxt < hi ? nxt : HW - 1));
      kx_next = ld_at(kx, (unsigned)x);
      ky_next = ld_at(ky, (unsigned)(y < H ? y : H - 1));
    }
    float wv[kPayload];
    bool valid;
    {
      const float D = s4.w;
      const float3 d = make_float3(mul_nc(kxp, D), mul_nc(kyp, D), D);
      const float3 c = xform32(R, t, d);
      const float iz = 1.0f / c.z;
      const float u = project32(in.fx, c.x, iz, in.cx);
      const float v = project32(in.fy, c.y, iz, in.cy);
      // the association: decided here from the projection, or given by the caller
      // (a fixed association, [job][pixel] word pairs as written to assoc_out)
      int xh, yh, xt, yt;
      float x0f, y0f;
      bool in_img, given_geo = true, given_photo = true;
      if (fixed == nullptr) {
        const float xf = floorf(u + 0.5f), yf = floorf(v + 0.5f);
        x0f = floorf(u);
        y0f = floorf(v);
        // clamped copies for addressing: the median of (value, 0, bound), one
        // instruction; a NaN value gives 0 (the hardware's median of three with a
        // NaN operand is the minimum of the other two)
        xh = (int)__builtin_amdgcn_fmed3f(xf, 0.0f, fWm1);
        yh = (int)__builtin_amdgcn_fmed3f(yf, 0.0f, fHm1);
        xt = (int)__builtin_amdgcn_fmed3f(x0f, 0.0f, fWm2);
        yt = (int)__builtin_amdgcn_fmed3f(y0f, 0.0f, fHm2);
        in_img = c.z > 0.0f && xf >= 0.0f && xf <= fWm1 && yf >= 0.0f && yf <= fHm1;
      } else {
        const size_t o = 2 * ((size_t)p * HW + (size_t)(pix < hi ? pix : HW - 1));
        const unsigned w0 = fixed[o], w1 = fixed[o + 1];
        const unsigned tg = min(w0 >> 2, (unsigned)(HW - 1));
        xh = (int)(tg % (unsigned)W);
        yh = (int)(tg / (unsigned)W);
        xt = min((int)(w1 % (unsigned)W), W - 2);
        yt = min((int)(w1 / (unsigned)W), H - 2);
        x0f = (float)xt;
        y0f = (float)yt;
        given_geo = (w0 & 1u) != 0;
        given_photo = (w0 & 2u) != 0;
        in_img = true;
      }
      // pixel indices below 2^24: 24-bit multiplies (full rate, unlike 32-bit ones)
      const unsigned th = __umul24((unsigned)yh, (unsigned)W) + (unsigned)xh;
      const unsigned t0 = __umul24((unsigned)yt, (unsigned)W) + (unsigned)xt;
      const float4 tq = ld_at(ndj, th);
      const float g00 = ld_at(gj, t0), g10 = ld_at(gj, t0 + 1u), g01 = ld_at(gj, t0 + (unsigned)W),
                  g11 = ld_at(gj, t0 + (unsigned)W + 1u);
      float Gi = ld_at(gi, (unsigned)(pix < hi ? pix : HW - 1));
      const float kxh = ld_at(kx, (unsigned)xh), kyh = ld_at(ky, (unsigned)yh);
      valid = pix < hi && !is_nan(s4.x) && in_img && !is_nan(tq.x);
      const float3 q = make_float3(mul_nc(kxh, tq.w), mul_nc(kyh, tq.w), tq.w);
      const float3 e = make_float3(c.x - q.x, c.y - q.y, c.z - q.z);
      const float3 n = make_float3(s4.x, s4.y, s4.z);
      const float3 m = rotate32(R, n);
      bool ph;
      if (fixed == nullptr) {
        valid = valid && dot32(e, e) < tau_d2 && dot32(m, make_float3(tq.x, tq.y, tq.z)) > tau_n;
        ph = x0f >= 0.0f && x0f <= fWm2 && y0f >= 0.0f && y0f <= fHm2;
      } else {
        valid = valid && given_geo;
        ph = given_photo;
      }
      ph = ph && !is_nan(Gi) && !(is_nan(g00) || is_nan(g10) || is_nan(g01) || is_nan(g11));
      if (!ph) Gi = __builtin_nanf("");
      // the association out (inspection): word 0 = target pixel << 2 | photometric << 1
      // | geometric, word 1 = first pixel of the bilinear footprint (0 where unused)
      if (assoc_out != nullptr && pix < hi) {
        const size_t o = 2 * ((size_t)p * HW + (size_t)pix);
        assoc_out[o] = valid ? ((th << 2) | 1u | (ph ? 2u : 0u)) : 0u;
        assoc_out[o + 1] = (valid && ph) ? t0 : 0u;
      }
      if constexpr (MODE == 2) {
        wv[0] = D; wv[1] = tq.w; wv[2] = n.x; wv[3] = n.y; wv[4] = n.z;
        wv[5] = (float)px; wv[6] = (float)py; wv[7] = (float)xh; wv[8] = (float)yh;
        wv[9] = x0f; wv[10] = y0f;
      } else {
        // bilinear weights within the footprint cell
        wv[0] = c.x; wv[1] = c.y; wv[2] = c.z; wv[3] = m.x; wv[4] = m.y; wv[5] = m.z;
        wv[6] = q.x; wv[7] = q.y; wv[8] = q.z; wv[9] = u - x0f; wv[10] = v - y0f;
      }
      wv[11] = Gi; wv[12] = g00; wv[13] = g10; wv[14] = g01; wv[15] = g11;
    }
    if constexpr (!JAC) {
      // energy only: too little work per pixel to be worth the queue
      if (valid) pixel_terms<MODE, JAC>(A, wv, R, t, Rd, td, kx64, ky64, in, fx64, fy64, cx64, cy64, swg, swp);
      continue;
    }
    // append the passing pixels to the queue in lane order
    const unsigned long long mask = __ballot(valid);
    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
    if (valid) {
      const int slot = (tail + rank) & (kQueue - 1);
#pragma unroll
      for (int k = 0; k < kPayload; ++k) Q[k * kQueue + slot] = wv[k];
    }
    tail += __popcll(mask);
    if (tail - head >= 64) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int slot = (head + lane) & (kQueue - 1);
      float w[kPayload];
#pragma unroll
      for (int k = 0; k < kPayload; ++k) w[k] = Q[k * kQueue + slot];
      pixel_terms<MODE, JAC>(A, w, R, t, Rd, td, kx64, ky64, in, fx64, fy64, cx64, cy64, swg, swp);
      head += 64;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  // the rest of the queue (fewer than 64)
  if (tail > head) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < tail - head) {
      const int slot = (head + lane) & (kQueue - 1);
      float w[kPayload];
#pragma unroll
      for (int k = 0; k < kPayload; ++k) w[k] = Q[k * kQueue + slot];
      pixel_terms<MODE, JAC>(A, w, R, t, Rd, td, kx64, ky64, in, fx64, fy64, cx64, cy64, swg, swp);
    }
  }
  __syncthreads();  // queues are dead: their LDS becomes the reduction buffer

  // Workgroup reduction in FP64, fixed order, 16 values at a time through LDS: with
  // 512 threads the upper half first adds onto the lower half; then each value's
  // RL lane sums are added in chunks of 16 lanes, and the chunk sums in order.
  double (*red)[RL] = reinterpret_cast<double (*)[RL]>(smem);
  double (*part)[NCH] = reinterpret_cast<double (*)[NCH]>(smem + 16 * RL);
  double* out = smem + 16 * RL + 16 * NCH;
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
    records[(size_t)pt * kRecWords + tid] = val;
  }
}

template <int MODE, bool JAC, int NT>
void launch_nt(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd, int tiles,
               unsigned* assoc_out) {
  const long long P = c.shape.P;
  const long long jobs = c.bidir ? 2 * P : P;
  Intr32 i32{(float)in.fx, (float)in.fy, (float)in.cx, (float)in.cy, in.width, in.height};
  float tau_d2 = (float)(prm.tau_dist * prm.tau_dist);
  float tau_n = (float)prm.tau_normal;
  double swg = sqrt(wd * prm.w_geo);
  double swp = sqrt(wd * prm.w_photo);
  unsigned grid = (unsigned)(8 * ((jobs * tiles + 7) / 8));
  hipLaunchKernelGGL((k_dense<MODE, JAC, NT>), dim3(grid), dim3(NT), 0, c.stream, c.pairs.as<int>(), P, c.bidir,
                     tiles, c.nd.as<float4>(), c.grad.as<float>(), c.kx.as<float>(), c.ky.as<float>(),
                     c.kx64.as<double>(), c.ky64.as<double>(), poses, i32, in.fx, in.fy, in.cx, in.cy, tau_d2, tau_n,
                     swg, swp, c.records.as<double>(), reinterpret_cast<const unsigned*>(prm.fixed_association),
                     assoc_out);
}

template <int MODE, bool JAC>
void launch_mode(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd, int nt,
                 int tiles, unsigned* masks) {
  switch (nt) {
    case 64: launch_nt<MODE, JAC, 64>(c, in, poses, prm, wd, tiles, masks); break;
    case 128: launch_nt<MODE, JAC, 128>(c, in, poses, prm, wd, tiles, masks); break;
    case 512: launch_nt<MODE, JAC, 512>(c, in, poses, prm, wd, tiles, masks); break;
    default: launch_nt<MODE, JAC, 256>(c, in, poses, prm, wd, tiles, masks); break;
  }
}

// Records of `tiles` partial records per job (the workspace grows only here, and is
// settled before any graph capture by dense_threads_for).
void ensure_records(Context& c, int tiles) {
  const long long jobs = (c.bidir ? 2 : 1) * c.shape.P;
  ensure(c.records, sizeof(double) * kRecWords * (size_t)(jobs * tiles + 1));
}

void launch_any(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                bool jac, int nt, int tiles, unsigned* masks = nullptr) {
  ensure_records(c, tiles);
  c.dense_tiles = tiles;
  c.dense_shape_last[jac ? 0 : 2] = nt;  // the launch shape for bf_dense_shape
  c.dense_shape_last[jac ? 1 : 3] = tiles;
  const int mode = prm.accumulate;
  if (jac) {
    if (mode == 2) launch_mode<2, true>(c, in, poses, prm, wd, nt, tiles, masks);
    else if (mode == 1) launch_mode<1, true>(c, in, poses, prm, wd, nt, tiles, masks);
    else launch_mode<0, true>(c, in, poses, prm, wd, nt, tiles, masks);
  } else {
    if (mode == 2) launch_mode<2, false>(c, in, poses, prm, wd, nt, tiles, masks);
    else launch_mode<0, false>(c, in, poses, prm, wd, nt, tiles, masks);
  }
}

// Launch shape of the dense pair jobs: threads per workgroup and tiles per job.
struct DenseShape {
  int nt, tiles;
};

// The caller's shape (dense_threads, and dense_tiles or 1), or the fastest of the
// candidates, timed once per (pixels per frame, precision mode, Jacobians, range of
// job counts) in this context.  Timing runs the real launch (it only rewrites the
// records) and synchronises the stream once.  Candidates: 64..512 threads with the
// job whole, and 128 or 256 threads with the job split into 2 or 4 tiles (more
// workgroups for the last round of a grid, shorter dependent loops per workgroup).
DenseShape choose_shape(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                        bool jac) {
  if (prm.dense_threads != 0) return {prm.dense_threads, prm.dense_tiles > 0 ? prm.dense_tiles : 1};
  int bucket = 0;
  const long long jobs = c.bidir ? 2 * c.shape.P : c.shape.P;
  while (bucket < 40 && (1LL << bucket) < jobs) ++bucket;
  const long long key = (((long long)in.width * in.height * 4 + prm.accumulate) * 2 + (jac ? 1 : 0)) * 64 + bucket;
  auto it = c.dense_threads.find(key);
  if (it != c.dense_threads.end()) return {it->second / 16, it->second % 16};
  static const DenseShape cand[] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {128, 2}, {256, 2}, {128, 4}, {256, 4}};
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  DenseShape best{256, 1};
  float best_ms = 1e30f;
  for (const DenseShape& d : cand) {
    launch_any(c, in, poses, prm, wd, jac, d.nt, d.tiles);  // warm-up
    check_hip(hipEventRecord(e0, c.stream), "hipEventRecord");
    for (int r = 0; r < 3; ++r) launch_any(c, in, poses, prm, wd, jac, d.nt, d.tiles);
    check_hip(hipEventRecord(e1, c.stream), "hipEventRecord");
    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (ms < best_ms) {
      best_ms = ms;
      best = d;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.dense_threads[key] = best.nt * 16 + best.tiles;
  return best;
}

// Whole-job records [jobs][kRecWords] from the tile records (the tiles of a job
// summed in tile order, as the edge kernel sums them).
__global__ void k_combine_records(const double* __restrict__ tiled, long long jobs, int tiles,
                                  double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= jobs * kRecWords) return;
  const long long job = k / kRecWords;
  const int w = (int)(k % kRecWords);
  double s = 0.0;
  for (int t = 0; t < tiles; ++t) s += tiled[((size_t)job * tiles + t) * kRecWords + w];
  out[k] = s;
}

}  // namespace

void launch_dense(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                  bool with_jacobians, unsigned* assoc_out) {
  if (c.shape.P == 0) return;
  const DenseShape d = choose_shape(c, in, poses, prm, wd, with_jacobians);
  launch_any(c, in, poses, prm, wd, with_jacobians, d.nt, d.tiles, assoc_out);
}

int dense_threads_for(Context& c, const bf_intrinsics& in, const double* poses, const bf_params& prm, double wd,
                      bool with_jacobians) {
  if (c.shape.P == 0) return 0;
  const DenseShape d = choose_shape(c, in, poses, prm, wd, with_jacobians);
  ensure_records(c, d.tiles);
  return d.nt * 16 + d.tiles;
}

void export_records(Context& c, double* out) {
  const long long jobs = (c.bidir ? 2 : 1) * c.shape.P;
  if (jobs == 0) return;
  const long long n = jobs * kRecWords;
  hipLaunchKernelGGL(k_combine_records, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream,
                     c.records.as<double>(), jobs, c.dense_tiles, out);
}

}  // namespace bf
