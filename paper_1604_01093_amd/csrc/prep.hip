// Per-frame preparation (paper Sec. 4.1.1: positions and normals of the
// low-resolution depth are computed once and cached per frame; Sec. 4.3: the
// photometric term reads the gradient of the luminance).
//
// Output per pixel: float4 (nx, ny, nz, depth) with a NaN normal where it is not
// valid, and the central-difference gradient magnitude G (NaN where invalid).
// Positions are not stored: P = (kx[x] D, ky[y] D, D) is recomputed from the depth
// with kx[x] = fl32((x - cx) / fx), 4 bytes per pixel instead of 12.
#include "internal.h"

namespace bf {

// depth_min <= d <= depth_max compared exactly (the FP32 depth widened to FP64)
__device__ __forceinline__ bool depth_ok(float d, double dmin, double dmax) {
  const double w = (double)d;
  return (d == d) && w >= dmin && w <= dmax && d != __builtin_inff();
}

// Ray coefficients (x - cx) / fx and (y - cy) / fy: FP64, and rounded to FP32.
__global__ void __launch_bounds__(256) k_ray_tables(double fx, double fy, double cx, double cy, int W, int H,
                                                    float* __restrict__ kx, float* __restrict__ ky,
                                                    double* __restrict__ kx64, double* __restrict__ ky64) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < W) {
    double k = ((double)t - cx) / fx;
    kx64[t] = k;
    kx[t] = (float)k;
  }
  if (t < H) {
    double k = ((double)t - cy) / fy;
    ky64[t] = k;
    ky[t] = (float)k;
  }
}

// The normal and gradient of one pixel from its depth and intensity and those of
// its four neighbours (zero where the pixel is on the image border).
__device__ __forceinline__ void prepare_pixel(int x, int y, bool inner, float d, float dl, float dr, float du,
                                              float dd, float lc, float ll, float lr, float lu, float ld,
                                              const float* __restrict__ kx, const float* __restrict__ ky,
                                              double dmin, double dmax, float4& out, float& g) {
  const float nan = __builtin_nanf("");
  out = make_float4(nan, nan, nan, d);
  g = nan;
  if (!inner) return;
  if (depth_ok(d, dmin, dmax) && depth_ok(dl, dmin, dmax) && depth_ok(dr, dmin, dmax) && depth_ok(du, dmin, dmax) &&
      depth_ok(dd, dmin, dmax)) {
#pragma clang fp contract(off)
    float kxl = kx[x - 1], kxr = kx[x + 1], kxc = kx[x];
    float kyu = ky[y - 1], kyd = ky[y + 1], kyc = ky[y];
    // d1 = P(x+1,y) - P(x-1,y), d2 = P(x,y+1) - P(x,y-1)
    float d1x = kxr * dr - kxl * dl, d1y = kyc * dr - kyc * dl, d1z = dr - dl;
    float d2x = kxc * dd - kxc * du, d2y = kyd * dd - kyu * du, d2z = dd - du;
    float cx_ = d1y * d2z - d1z * d2y;
    float cy_ = d1z * d2x - d1x * d2z;
    float cz_ = d1x * d2y - d1y * d2x;
    float l2 = (cx_ * cx_ + cy_ * cy_) + cz_ * cz_;
    if (l2 > 0.0f) {
      float nrm = sqrtf(l2);
      float nx = cx_ / nrm, ny = cy_ / nrm, nz = cz_ / nrm;
      float px = kxc * d, py = kyc * d;
      float s = (nx * px + ny * py) + nz * d;
      if (s > 0.0f) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
      }
      out.x = nx;
      out.y = ny;
      out.z = nz;
    }
  }
  if (isfinite(lc) && isfinite(ll) && isfinite(lr) && isfinite(lu) && isfinite(ld)) {
    float gx = (lr - ll) * 0.5f, gy = (ld - lu) * 0.5f;
    g = sqrtf(gx * gx + gy * gy);
  }
}

// kPrepPixels pixels per thread (strided by the workgroup size, so each step is
// coalesced), all their loads issued before any is used; grid
// (ceil(W*H / (256 kPrepPixels)), F).
constexpr int kPrepPixels = 4;

__global__ void __launch_bounds__(256) k_prepare(const float* __restrict__ depth, const float* __restrict__ inten,
                                                 const float* __restrict__ kx, const float* __restrict__ ky, int W,
                                                 int H, double dmin, double dmax, float4* __restrict__ nd,
                                                 float* __restrict__ grad) {
  const int HW = W * H;
  const size_t base = (size_t)blockIdx.y * HW;
  const float* D = depth + base;
  const float* L = inten + base;
  float v[kPrepPixels][10];
  bool inner[kPrepPixels];
#pragma unroll
  for (int u = 0; u < kPrepPixels; ++u) {
    const int pix = blockIdx.x * (256 * kPrepPixels) + u * 256 + threadIdx.x;
    const int x = pix % W, y = pix / W;
    const bool in = pix < HW;
    inner[u] = in && x > 0 && x < W - 1 && y > 0 && y < H - 1;
    v[u][0] = in ? D[pix] : 0.0f;
    v[u][5] = inner[u] ? L[pix] : 0.0f;
    if (inner[u]) {
      v[u][1] = D[pix - 1];
      v[u][2] = D[pix + 1];
      v[u][3] = D[pix - W];
      v[u][4] = D[pix + W];
      v[u][6] = L[pix - 1];
      v[u][7] = L[pix + 1];
      v[u][8] = L[pix - W];
      v[u][9] = L[pix + W];
    } else {
      for (int k = 1; k < 10; ++k)
        if (k != 5) v[u][k] = 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < kPrepPixels; ++u) {
    const int pix = blockIdx.x * (256 * kPrepPixels) + u * 256 + threadIdx.x;
    if (pix >= HW) break;
    const int x = pix % W, y = pix / W;
    float4 out;
    float g;
    prepare_pixel(x, y, inner[u], v[u][0], v[u][1], v[u][2], v[u][3], v[u][4], v[u][5], v[u][6], v[u][7], v[u][8],
                  v[u][9], kx, ky, dmin, dmax, out, g);
    nd[base + pix] = out;
    grad[base + pix] = g;
  }
}

void launch_prepare(Context& c, const bf_frames& fr, const bf_intrinsics& in, const bf_params& prm) {
  const int W = in.width, H = in.height;
  int n = W > H ? W : H;
  hipLaunchKernelGGL(k_ray_tables, dim3((n + 255) / 256), dim3(256), 0, c.stream, in.fx, in.fy, in.cx, in.cy, W, H,
                     c.kx.as<float>(), c.ky.as<float>(), c.kx64.as<double>(), c.ky64.as<double>());
  dim3 grid((W * H + 256 * kPrepPixels - 1) / (256 * kPrepPixels), fr.num_frames);
  hipLaunchKernelGGL(k_prepare, grid, dim3(256), 0, c.stream, fr.depth, fr.intensity, c.kx.as<float>(),
                     c.ky.as<float>(), W, H, prm.depth_min, prm.depth_max, c.nd.as<float4>(),
                     c.grad.as<float>());
}

}  // namespace bf
