// Quality metrics of the experiments (Sec. IV): PSNR over all voxels, and
// SSIM with an 11-tap Gaussian window of standard deviation 1.5 per axis (2D:
// per slice; 3D: 11 x 11 x 11), c1 = (0.01 L)^2, c2 = (0.03 L)^2, averaged over
// the positions where the window lies inside the data; and the relative change
// ||a - b|| / ||b|| used by the stopping test.
//
// SSIM runs as separable FP64 passes: the five window-weighted moments
// (x, y, x^2, y^2, xy) along W, then along H (and D), the last pass forming the
// SSIM value at each position.  Every reduction writes one FP64 partial per
// block and is summed in a fixed order (deterministic).
#include <cmath>

#include "common.hpp"

namespace cspnp {

namespace {

constexpr int kWin = 11;
constexpr int kRedGrid = 1024;

struct Window {
  double w[kWin];
};

Window gaussian_window() {
  Window g;
  double s = 0.0;
  for (int k = 0; k < kWin; ++k) {
    const double t = k - (kWin - 1) / 2.0;
    g.w[k] = std::exp(-(t * t) / (2.0 * 1.5 * 1.5));
    s += g.w[k];
  }
  for (int k = 0; k < kWin; ++k) g.w[k] /= s;
  return g;
}

__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = red[0] + red[1] + red[2] + red[3];
  return s;
}

__global__ __launch_bounds__(256) void sq_diff_partials(const float* __restrict__ a, const float* __restrict__ b,
                                                        size_t n, double* __restrict__ part_diff,
                                                        double* __restrict__ part_ref) {
  double sd = 0.0, sr = 0.0;
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const double t = (double)a[i] - (double)b[i];
    sd += t * t;
    if (part_ref) sr += (double)b[i] * (double)b[i];
  }
  double s = block_sum256(sd);
  if (threadIdx.x == 0) part_diff[blockIdx.x] = s;
  if (part_ref) {
    __syncthreads();
    s = block_sum256(sr);
    if (threadIdx.x == 0) part_ref[blockIdx.x] = s;
  }
}

__device__ double fixed_sum(const double* p, int n) {
  // single thread, fixed order
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += p[i];
  return s;
}

__global__ void finish_psnr(const double* __restrict__ part, size_t n, double peak, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = 10.0 * log10((double)n * peak * peak / fixed_sum(part, kRedGrid));
}

__global__ void finish_rel(const double* __restrict__ pd, const double* __restrict__ pr, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = sqrt(fixed_sum(pd, kRedGrid) / fixed_sum(pr, kRedGrid));
}

// pass along W: moments of (a, b) at valid columns; out[q][z][y][x0], q = 0..4
__global__ __launch_bounds__(256) void ssim_pass_w(const Window g, const float* __restrict__ a,
                                                   const float* __restrict__ b, int D, int H, int W,
                                                   double* __restrict__ out) {
  const int Wv = W - kWin + 1;
  const size_t n = (size_t)D * H * Wv, plane = n;
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const int x0 = (int)(i % Wv);
    const size_t row = i / Wv;  // z*H + y
    const size_t src = row * W + x0;
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const double va = a[src + k], vb = b[src + k], w = g.w[k];
      m[0] += w * va;
      m[1] += w * vb;
      m[2] += w * va * va;
      m[3] += w * vb * vb;
      m[4] += w * va * vb;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q * plane + i] = m[q];
  }
}

// generic pass along an axis of a [5][outer][len][inner] moment array: valid positions along len
__global__ __launch_bounds__(256) void ssim_pass_axis(const Window g, const double* __restrict__ in, size_t outer,
                                                      int len, size_t inner, double* __restrict__ out) {
  const int lv = len - kWin + 1;
  const size_t n = outer * lv * inner;
  const size_t in_plane = outer * len * inner;
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const size_t ii = i % inner;
    const size_t t = i / inner;
    const int l0 = (int)(t % lv);
    const size_t o = t / lv;
    const size_t src = (o * len + l0) * inner + ii;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kWin; ++k) s += g.w[k] * in[q * in_plane + src + (size_t)k * inner];
      out[q * n + i] = s;
    }
  }
}

// SSIM value at every position of a final [5][n] moment array; block partial sums
__global__ __launch_bounds__(256) void ssim_values(const double* __restrict__ m, size_t n, double c1, double c2,
                                                   double* __restrict__ part) {
  double acc = 0.0;
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const double mx = m[i], my = m[n + i];
    const double sxx = m[2 * n + i] - mx * mx, syy = m[3 * n + i] - my * my, sxy = m[4 * n + i] - mx * my;
    acc += ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2));
  }
  const double s = block_sum256(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void finish_mean(const double* __restrict__ part, size_t n, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = fixed_sum(part, kRedGrid) / (double)n;
}

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

size_t ssim_bytes(int D, int H, int W, int dims) {
  const size_t Wv = W - kWin + 1, Hv = H - kWin + 1;
  size_t n = align_up(5 * (size_t)D * H * Wv * 8) + align_up(5 * (size_t)D * Hv * Wv * 8);
  if (dims == 3) n += align_up(5 * (size_t)(D - kWin + 1) * Hv * Wv * 8);
  return n + align_up(kRedGrid * 8);
}

}  // namespace

hipError_t launch_rel_change(const float* a, const float* b, size_t n, double* out, void* ws, hipStream_t s) {
  double* pd = static_cast<double*>(ws);
  double* pr = pd + kRedGrid;
  hipLaunchKernelGGL(sq_diff_partials, dim3(kRedGrid), dim3(256), 0, s, a, b, n, pd, pr);
  hipLaunchKernelGGL(finish_rel, dim3(1), dim3(64), 0, s, pd, pr, out);
  return hipGetLastError();
}

size_t rel_change_ws_bytes() { return align_up(2 * kRedGrid * sizeof(double)); }

}  // namespace cspnp

using namespace cspnp;

CSPNP_API int cspnp_metrics_workspace_size(int32_t D, int32_t H, int32_t W, int32_t dims, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(CSPNP_EINVAL, "bytes is NULL");
  if (D < 1 || H < 1 || W < 1) return fail(CSPNP_EINVAL, "D, H, W must be >= 1");
  if (dims != 0 && dims != 2 && dims != 3) return fail(CSPNP_EINVAL, "dims must be 0 (PSNR), 2 or 3");
  if (dims >= 2 && (H < kWin || W < kWin)) return fail(CSPNP_EINVAL, "SSIM needs H, W >= 11");
  if (dims == 3 && D < kWin) return fail(CSPNP_EINVAL, "3D SSIM needs D >= 11");
  *bytes = dims == 0 ? align_up(2 * kRedGrid * sizeof(double)) : ssim_bytes(D, H, W, dims);
  return CSPNP_OK;
}

CSPNP_API int cspnp_psnr(const float* est, const float* ref, size_t n, double peak, double* out, void* ws,
                         void* stream) {
  clear_error();
  if (check_ptr(est, "est") || check_ptr(ref, "ref")) return CSPNP_EINVAL;
  if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(CSPNP_EINVAL, "out must be an aligned device double");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  if (n == 0 || !(peak > 0)) return fail(CSPNP_EINVAL, "n must be > 0 and peak > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* part = static_cast<double*>(ws);
  hipLaunchKernelGGL(sq_diff_partials, dim3(kRedGrid), dim3(256), 0, s, est, ref, n, part, nullptr);
  hipLaunchKernelGGL(finish_psnr, dim3(1), dim3(64), 0, s, part, n, peak, out);
  CSPNP_HIP(hipGetLastError());
  return CSPNP_OK;
}

CSPNP_API int cspnp_rel_change(const float* a, const float* b, size_t n, double* out, void* ws, void* stream) {
  clear_error();
  if (check_ptr(a, "a") || check_ptr(b, "b")) return CSPNP_EINVAL;
  if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(CSPNP_EINVAL, "out must be an aligned device double");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  CSPNP_HIP(launch_rel_change(a, b, n, out, ws, reinterpret_cast<hipStream_t>(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_ssim(const float* est, const float* ref, int32_t D, int32_t H, int32_t W, int32_t dims,
                         double L, double* out, void* ws, void* stream) {
  clear_error();
  size_t need = 0;
  if (int s = cspnp_metrics_workspace_size(D, H, W, dims, &need)) return s;
  if (dims == 0) return fail(CSPNP_EINVAL, "dims must be 2 or 3 for SSIM");
  if (check_ptr(est, "est") || check_ptr(ref, "ref")) return CSPNP_EINVAL;
  if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(CSPNP_EINVAL, "out must be an aligned device double");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  if (!(L > 0)) return fail(CSPNP_EINVAL, "L must be > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Window g = gaussian_window();
  const size_t Wv = W - kWin + 1, Hv = H - kWin + 1;
  char* w = static_cast<char*>(ws);
  double* t1 = reinterpret_cast<double*>(w);
  double* t2 = reinterpret_cast<double*>(w + align_up(5 * (size_t)D * H * Wv * 8));
  double* t3 = reinterpret_cast<double*>(reinterpret_cast<char*>(t2) + align_up(5 * (size_t)D * Hv * Wv * 8));
  double* part = reinterpret_cast<double*>(w + need - align_up(kRedGrid * 8));
  const dim3 G(kRedGrid), B(256);
  hipLaunchKernelGGL(ssim_pass_w, G, B, 0, s, g, est, ref, D, H, W, t1);
  hipLaunchKernelGGL(ssim_pass_axis, G, B, 0, s, g, t1, (size_t)D, H, Wv, t2);  // along H
  const double c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
  size_t npos = (size_t)D * Hv * Wv;
  const double* fin = t2;
  if (dims == 3) {
    hipLaunchKernelGGL(ssim_pass_axis, G, B, 0, s, g, t2, (size_t)1, D, Hv * Wv, t3);  // along D
    npos = (size_t)(D - kWin + 1) * Hv * Wv;
    fin = t3;
  }
  hipLaunchKernelGGL(ssim_values, G, B, 0, s, fin, npos, c1, c2, part);
  hipLaunchKernelGGL(finish_mean, dim3(1), dim3(64), 0, s, part, npos, out);
  CSPNP_HIP(hipGetLastError());
  return CSPNP_OK;
}
