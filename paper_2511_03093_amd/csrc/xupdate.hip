// x-step of the ADMM (eq. (v-update)) with the temporal term of Sec. III-C
// folded in: for every pixel p solve
//     (m m^T + gamma L + rho I) x = m y + rho (u - d)
// where m in {0,1}^R are the pixel's mask bits and L the z-Laplacian.
// Write A = T + U U^T with T = rho I + gamma L_N (the free-ends chain, a
// tridiagonal matrix shared by all pixels and LDL^T-factored on the host) and
// U = [m] (Neumann) or U = [m, sqrt(gamma) w], w = e_0 - e_{R-1} (periodic:
// the wrap pair).  The Woodbury identity (the paper's eq. (Woodbury), here
// with a 2 x 2 capacitance matrix) gives
//     x = a - alpha b - beta c,  a = T^{-1} rhs, b = T^{-1} m, c = T^{-1} w,
// with (alpha, beta) from the 2 x 2 system.  At gamma = 0, T = rho I and this is
// exactly the paper's element-wise update (end of Sec. III-B).
// One thread per pixel, the z-vector in FP64 registers, FP32 in/out; the
// kernel streams u, d (8 B/voxel) and writes f = x + d (4 B/voxel): HBM-bound.
#include <type_traits>

#include "xupdate_impl.hpp"

namespace cspnp {

namespace {

using xuimpl::load_bits;
using xuimpl::ld_at;
using xuimpl::pixel_solve;
using xuimpl::st_at;

// block shapes (threads along W, rows) selectable per plan
constexpr int kXuShapes[][2] = {{64, 4}, {64, 8}, {128, 2}, {256, 1}, {64, 2}, {64, 1}};
constexpr int kNumXuShapes = sizeof(kXuShapes) / sizeof(kXuShapes[0]);
constexpr int kXuMaxThreads = 512;

// `d` is the dual variable, or (d_from_f) the previous f, with d = f - u formed
// here exactly as the TV epilogue forms it; f_out may then alias `d`.
// The pixel's mask bits are one pixel-major word (uint16 for R <= 16).
template <int R>
using MaskWord = typename std::conditional<(R <= 16), uint16_t, uint32_t>::type;

template <int R>
__global__ __launch_bounds__(kXuMaxThreads) void xupdate_kernel(
    const ZSolve z, const MaskWord<R>* __restrict__ pmask, int H, int W,
    const float* __restrict__ y, const float* __restrict__ u, const float* d, int d_from_f,
    float* __restrict__ x_out, float* f_out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const uint32_t pix = (uint32_t)(h * W + w);
  const uint32_t off = 4u * pix;
  const uint32_t m = ld_at(pmask, (uint32_t)sizeof(MaskWord<R>) * pix);
  const double yv = (double)ld_at(y, off);
  double a[R];
  float dv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float ur = ld_at(u + r * HW, off);
    const float dr = ld_at(d + r * HW, off);
    dv[r] = d_from_f ? dr - ur : dr;
    a[r] = z.rho * ((double)ur - (double)dv[r]);
    if ((m >> r) & 1u) a[r] += yv;
  }
  pixel_solve<R>(z, m, a);
  if (x_out) {
#pragma unroll
    for (int r = 0; r < R; ++r) st_at(x_out + r * HW, off, (float)a[r]);
  }
  if (f_out) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // converted here, not kept as FP64 across the solve
      float dr = dv[r];
      asm volatile("" : "+v"(dr));
      st_at(f_out + r * HW, off, (float)(a[r] + (double)dr));
    }
  }
}

// x-step fused with the Tikhonov u-step and the d-step (in place on u, d):
//   f = x + d,  u = rho f / (2 lambda + rho),  d = f - u.
template <int R>
__global__ __launch_bounds__(kXuMaxThreads) void xupdate_tikhonov_kernel(
    const ZSolve z, double shrink, const uint32_t* __restrict__ bits, int H, int W, int Wq,
    const float* __restrict__ y, float* __restrict__ u, float* __restrict__ d,
    float* __restrict__ x_out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)h * W + w;
  const uint32_t m = load_bits<R>(bits, H, Wq, h, w);
  const double yv = (double)y[p];
  double a[R];
  float dv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float ur = u[r * HW + p];
    dv[r] = d[r * HW + p];
    a[r] = z.rho * ((double)ur - (double)dv[r]);
    if ((m >> r) & 1u) a[r] += yv;
  }
  pixel_solve<R>(z, m, a);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (x_out) x_out[r * HW + p] = (float)a[r];
    const double f = a[r] + (double)dv[r];
    const double un = shrink * f;
    u[r * HW + p] = (float)un;
    d[r * HW + p] = (float)(f - un);
  }
}

// Tikhonov prox of a given f (unfused u-step + d-step).
__global__ __launch_bounds__(256) void tikhonov_kernel(float shrink, size_t n, const float* __restrict__ f,
                                                       float* __restrict__ u, float* __restrict__ d_out) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const float fv = f[i];
    const float uv = shrink * fv;
    u[i] = uv;
    if (d_out) d_out[i] = fv - uv;
  }
}

template <int R>
hipError_t launch_r(const cspnp_plan& pl, const ZSolve& zs, const float* y, const float* u,
                    const float* d, int d_from_f, float* x_out, float* f_out, hipStream_t s) {
  const auto& de = pl.desc;
  const int bx = kXuShapes[pl.xu_block][0], by = kXuShapes[pl.xu_block][1];
  dim3 block(bx, by);
  dim3 grid((de.W + bx - 1) / bx, (de.H + by - 1) / by);
  hipLaunchKernelGGL(xupdate_kernel<R>, grid, block, 0, s, zs, static_cast<const MaskWord<R>*>(pl.pmask), de.H,
                     de.W, y, u, d, d_from_f, x_out, f_out);
  return hipGetLastError();
}

template <int R>
hipError_t launch_tik_r(const cspnp_plan& pl, const ZSolve& zs, double shrink, const float* y,
                        float* u, float* d, float* x_out, hipStream_t s) {
  const auto& de = pl.desc;
  const int bx = kXuShapes[pl.xu_block][0], by = kXuShapes[pl.xu_block][1];
  dim3 block(bx, by);
  dim3 grid((de.W + bx - 1) / bx, (de.H + by - 1) / by);
  hipLaunchKernelGGL(xupdate_tikhonov_kernel<R>, grid, block, 0, s, zs, shrink, pl.bits, de.H, de.W,
                     pl.Wq, y, u, d, x_out);
  return hipGetLastError();
}

template <int... Rs>
struct RTable {
  template <typename F>
  static hipError_t dispatch(int R, F&& f) {
    hipError_t e = hipErrorInvalidValue;
    ((R == Rs ? (e = f(std::integral_constant<int, Rs>{}), true) : false) || ...);
    return e;
  }
};
using AllR = RTable<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23,
                    24, 25, 26, 27, 28, 29, 30, 31, 32>;

}  // namespace

int xu_num_blocks() { return kNumXuShapes; }

void xu_block_info(int i, int* bx, int* by) {
  *bx = kXuShapes[i][0];
  *by = kXuShapes[i][1];
}

hipError_t launch_xupdate(const cspnp_plan& pl, const ZSolve& zs, const float* y, const float* u,
                          const float* d, float* x_out, float* f_out, hipStream_t s, bool d_from_f) {
  if (pl.desc.N > 1) return launch_xupdate_multishot(pl, zs.rho, zs.gamma, y, u, d, d_from_f, x_out, f_out, s);
  return AllR::dispatch(pl.desc.R, [&](auto rc) {
    return launch_r<decltype(rc)::value>(pl, zs, y, u, d, d_from_f ? 1 : 0, x_out, f_out, s);
  });
}

hipError_t launch_xupdate_tikhonov(const cspnp_plan& pl, const ZSolve& zs, double lambda,
                                   const float* y, float* u, float* d, float* x_out,
                                   hipStream_t s) {
  const double shrink = zs.rho / (2.0 * lambda + zs.rho);
  return AllR::dispatch(pl.desc.R, [&](auto rc) {
    return launch_tik_r<decltype(rc)::value>(pl, zs, shrink, y, u, d, x_out, s);
  });
}

hipError_t launch_tikhonov(const cspnp_plan& pl, double lambda, double rho, const float* f,
                           float* u, float* d_out, hipStream_t s) {
  const size_t n = (size_t)pl.desc.N * pl.desc.R * pl.desc.H * pl.desc.W;
  const float shrink = (float)(rho / (2.0 * lambda + rho));
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(tikhonov_kernel, dim3((unsigned)blocks), dim3(256), 0, s, shrink, n, f, u, d_out);
  return hipGetLastError();
}

}  // namespace cspnp
