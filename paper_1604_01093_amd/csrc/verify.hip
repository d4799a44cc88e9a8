// Dense two-sided verification of frame pairs (paper Sec. 4.1.1, "Dense
// Verification"): for a pair (i, j) and the relative transform T_ji = T_j^-1 T_i
// of the given poses, every pixel of frame i with a valid normal is moved into
// camera j and associated with the nearest pixel of frame j; the association is
// valid when it passes the distance and normal tests of the dense term (same FP32
// decisions, same thresholds) and the intensities agree, |C_i(x,y) - C_j(x', y')|
// < tau_c at the associated pixel.  The re-projection error of the valid
// associations, |T_ji p - q|, is summed; the same is done from j to i.  The pair is
// valid when, in both directions, at least min_frac * W * H associations are valid
// and their mean error is at most max_err.
//
// One workgroup per (pair, direction); FP32 per pixel, FP64 fixed-order sums.
#include "internal.h"

namespace bf {

namespace {

__global__ void __launch_bounds__(256) k_verify(const int* __restrict__ pairs, long long P,
                                                const float4* __restrict__ nd, const float* __restrict__ inten,
                                                const float* __restrict__ kx, const float* __restrict__ ky,
                                                const double* __restrict__ poses, Intr32 in, float tau_d2,
                                                float tau_n, float tau_c, double* __restrict__ stats) {
  __shared__ double red[2][256];
  const long long job = blockIdx.x;
  if (job >= 2 * P) return;
  const long long p = job >> 1;
  const int dir = (int)(job & 1);
  const int a = pairs[2 * p + dir], b = pairs[2 * p + 1 - dir];  // source a, target b
  const int tid = threadIdx.x;
  const int W = in.W, H = in.H, HW = W * H;
  double Rd[9], td[3];
  relative_pose_nc(poses + (size_t)a * 16, poses + (size_t)b * 16, Rd, td);
  float R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
  for (int k = 0; k < 3; ++k) t[k] = (float)td[k];
  const float4* nda = nd + (size_t)a * HW;
  const float4* ndb = nd + (size_t)b * HW;
  const float* Ca = inten + (size_t)a * HW;
  const float* Cb = inten + (size_t)b * HW;
  const float fWm1 = (float)(W - 1), fHm1 = (float)(H - 1);
  float err = 0.0f;
  float cnt = 0.0f;
  for (int pix = tid; pix < HW; pix += 256) {
    const int px = pix % W, py = pix / W;
    const float4 s = nda[pix];
    if (is_nan(s.x)) continue;
    const float D = s.w;
    const float3 d = make_float3(mul_nc(kx[px], D), mul_nc(ky[py], D), D);
    const float3 c = xform32(R, t, d);
    if (!(c.z > 0.0f)) continue;
    const float iz = 1.0f / c.z;
    const float u = project32(in.fx, c.x, iz, in.cx);
    const float v = project32(in.fy, c.y, iz, in.cy);
    const float xf = floorf(u + 0.5f), yf = floorf(v + 0.5f);
    if (!(xf >= 0.0f && xf <= fWm1 && yf >= 0.0f && yf <= fHm1)) continue;
    const int xh = (int)xf, yh = (int)yf;
    const float4 tq = ndb[yh * W + xh];
    if (is_nan(tq.x)) continue;
    const float3 q = make_float3(mul_nc(kx[xh], tq.w), mul_nc(ky[yh], tq.w), tq.w);
    const float3 e = make_float3(c.x - q.x, c.y - q.y, c.z - q.z);
    const float e2 = dot32(e, e);
    if (!(e2 < tau_d2)) continue;
    const float3 m = rotate32(R, make_float3(s.x, s.y, s.z));
    if (!(dot32(m, make_float3(tq.x, tq.y, tq.z)) > tau_n)) continue;
    const float dc = Ca[pix] - Cb[yh * W + xh];
    if (!(fabsf(dc) < tau_c)) continue;
    err += sqrtf(e2);
    cnt += 1.0f;
  }
  red[0][tid] = (double)err;
  red[1][tid] = (double)cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    stats[4 * p + 2 * dir] = red[0][0];
    stats[4 * p + 2 * dir + 1] = red[1][0];
  }
}

__global__ void k_verify_decide(const double* __restrict__ stats, long long P, double max_err, double min_count,
                                uint8_t* __restrict__ valid) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  bool ok = true;
  for (int dir = 0; dir < 2; ++dir) {
    const double e = stats[4 * p + 2 * dir], n = stats[4 * p + 2 * dir + 1];
    ok = ok && n >= min_count && n > 0.0 && e / n <= max_err;
  }
  valid[p] = ok ? 1 : 0;
}

}  // namespace

void launch_verify(Context& c, const bf_frames& fr, const bf_intrinsics& in, const int* pairs, long long P,
                   const double* poses, const bf_params& prm, double tau_c, double max_err, double min_frac,
                   double* stats, uint8_t* valid) {
  if (P == 0) return;
  Intr32 i32{(float)in.fx, (float)in.fy, (float)in.cx, (float)in.cy, in.width, in.height};
  hipLaunchKernelGGL(k_verify, dim3((unsigned)(2 * P)), dim3(256), 0, c.stream, pairs, P, c.nd.as<float4>(),
                     fr.intensity, c.kx.as<float>(), c.ky.as<float>(), poses, i32,
                     (float)(prm.tau_dist * prm.tau_dist), (float)prm.tau_normal, (float)tau_c, stats);
  hipLaunchKernelGGL(k_verify_decide, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c.stream, stats, P, max_err,
                     min_frac * (double)in.width * (double)in.height, valid);
}

}  // namespace bf
