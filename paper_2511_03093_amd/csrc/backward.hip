// Reverse mode through the unrolled ADMM iterations (the library's
// differentiable solve): gradients of <xbar, x^K> with respect to the frames y
// and the scalars rho, lambda, gamma.
//
// Forward (cspnp_solve_ckpt): the usual iteration, storing (u, d) at the start
// of every segment of `ckpt_every` iterations.  Backward (cspnp_solve_bwd):
// segments in reverse; each is recomputed from its checkpoint keeping
// (u^k, d^k, f^{k+1}), then its iterations are reversed:
//   d' = f - u', u' = D_theta(f):   fbar = dbar' + D^T(ubar' - dbar')
//   TV (Chambolle from p = 0): the inner iterates p^t, w^t are rebuilt by the
//   same arithmetic as the fused forward kernel, then reversed one inner step
//   at a time:  gbar = (tau/s)(pbar' - (pbar'.p') g/|g|),  wbar = -div gbar,
//   pbar = pbar'/s - grad wbar,  fbar -= wbar/theta,  thetabar += <wbar, f/theta^2>;
//   the output step u = f - theta div p^K gives fbar += ubar, pbar^K = theta grad ubar,
//   thetabar -= <ubar, div p^K>.
//   x-step x = A^{-1}(m y + rho (u - d)), A symmetric:  lam = A^{-1}(fbar + xbar),
//   ybar += m.lam, ubar = rho lam, dbar = fbar - rho lam,
//   rhobar += <lam, u - d - x>, gammabar -= <lam, L x>.
// Scalar sums are FP64 block partials reduced in a fixed order (deterministic).
#include <algorithm>
#include <vector>

#include "multishot_impl.hpp"
#include "xupdate_impl.hpp"

namespace cspnp {
ZSolve make_zsolve(int R, int zbc, double rho, double gamma);
}

using namespace cspnp;

namespace {

constexpr int kThreads = 256;
constexpr int kGrid = 1024;  // fixed grid of the grid-stride kernels (one FP64 partial per block)

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(kThreads) void fill_zero(float* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) p[i] = 0.f;
}

__global__ void zero_doubles(double* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0.0;
}

struct Geo {
  int H, W;
  size_t HW, vol;
};

__device__ __forceinline__ void coords(const Geo& g, size_t i, int& h, int& w) {
  const size_t r = i % g.HW;
  h = (int)(r / g.W);
  w = (int)(r % g.W);
}

// w = div p - f/theta (same operation order as the fused forward kernel)
__global__ __launch_bounds__(kThreads) void tvb_w(Geo g, const float* __restrict__ px, const float* __restrict__ py,
                                                  const float* __restrict__ f, float inv_theta, float* __restrict__ wo) {
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    const float pxl = w > 0 ? px[i - 1] : 0.f;
    const float pyu = h > 0 ? py[i - g.W] : 0.f;
    const float pxc = w < g.W - 1 ? px[i] : 0.f;
    const float pyc = h < g.H - 1 ? py[i] : 0.f;
    wo[i] = (((pxc - pxl) + pyc) - pyu) - __fmul_rn(f[i], inv_theta);
  }
}

__device__ __forceinline__ void grad_at(const Geo& g, const float* __restrict__ w, size_t i, int h, int x, float& gx,
                                        float& gy) {
  const float c = w[i];
  gx = x < g.W - 1 ? (w[i + 1] - c) : 0.f;
  gy = h < g.H - 1 ? (w[i + g.W] - c) : 0.f;
}

// p' = (p + tau grad w) / (1 + tau |grad w|)
__global__ __launch_bounds__(kThreads) void tvb_p(Geo g, const float* __restrict__ wv, const float* __restrict__ px,
                                                  const float* __restrict__ py, float tau, float* __restrict__ pxo,
                                                  float* __restrict__ pyo) {
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    float gx, gy;
    grad_at(g, wv, i, h, w, gx, gy);
    const float q = fmaf(gx, gx, gy * gy);
    const float rs = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(q), 1.f));
    pxo[i] = fmaf(tau, gx, px[i]) * rs;
    pyo[i] = fmaf(tau, gy, py[i]) * rs;
  }
}

// output step: ut = ubar - dbar;  fbar = ubar;  pbar = theta grad ut;  thetabar -= <ut, div p^K>
__global__ __launch_bounds__(kThreads) void tvb_init(Geo g, const float* __restrict__ ubar, const float* __restrict__ dbar,
                                                     const float* __restrict__ pKx, const float* __restrict__ pKy,
                                                     float theta, float* __restrict__ fbar, float* __restrict__ pbx,
                                                     float* __restrict__ pby, double* __restrict__ partial) {
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    const float ut = ubar[i] - dbar[i];
    fbar[i] = ubar[i];
    const float utr = w < g.W - 1 ? ubar[i + 1] - dbar[i + 1] : ut;
    const float utd = h < g.H - 1 ? ubar[i + g.W] - dbar[i + g.W] : ut;
    pbx[i] = theta * (utr - ut);
    pby[i] = theta * (utd - ut);
    const float pxl = w > 0 ? pKx[i - 1] : 0.f;
    const float pyu = h > 0 ? pKy[i - g.W] : 0.f;
    const float pxc = w < g.W - 1 ? pKx[i] : 0.f;
    const float pyc = h < g.H - 1 ? pKy[i] : 0.f;
    acc -= (double)ut * (double)((pxc - pxl) + (pyc - pyu));
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// reverse of p' = (p + tau g)/s: gbar, and pbar <- pbar/s (in place)
__global__ __launch_bounds__(kThreads) void tvb_g(Geo g, const float* __restrict__ wv, const float* __restrict__ qx,
                                                  const float* __restrict__ qy, float tau, float* __restrict__ pbx,
                                                  float* __restrict__ pby, float* __restrict__ gbx,
                                                  float* __restrict__ gby) {
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    float gx, gy;
    grad_at(g, wv, i, h, w, gx, gy);
    const float q = fmaf(gx, gx, gy * gy);
    const float mag = __builtin_amdgcn_sqrtf(q);
    const float rs = __builtin_amdgcn_rcpf(fmaf(tau, mag, 1.f));
    const float bx = pbx[i], by = pby[i];
    const float a = bx * qx[i] + by * qy[i];
    float nx = 0.f, ny = 0.f;
    if (mag > 0.f) {
      const float im = 1.f / mag;
      nx = gx * im;
      ny = gy * im;
    }
    gbx[i] = tau * rs * (bx - a * nx);
    gby[i] = tau * rs * (by - a * ny);
    pbx[i] = bx * rs;
    pby[i] = by * rs;
  }
}

// wbar = -div gbar;  fbar -= wbar/theta;  thetabar += <wbar, f/theta^2>
__global__ __launch_bounds__(kThreads) void tvb_wbar(Geo g, const float* __restrict__ gbx, const float* __restrict__ gby,
                                                     const float* __restrict__ f, float theta, float* __restrict__ wbar,
                                                     float* __restrict__ fbar, double* __restrict__ partial) {
  double acc = 0.0;
  const double it2 = 1.0 / ((double)theta * (double)theta);
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    const float xl = w > 0 ? gbx[i - 1] : 0.f;
    const float yu = h > 0 ? gby[i - g.W] : 0.f;
    const float xc = w < g.W - 1 ? gbx[i] : 0.f;
    const float yc = h < g.H - 1 ? gby[i] : 0.f;
    const float wb = -((xc - xl) + (yc - yu));
    wbar[i] = wb;
    fbar[i] -= wb / theta;
    acc += (double)wb * (double)f[i] * it2;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// pbar -= grad wbar
__global__ __launch_bounds__(kThreads) void tvb_pbar(Geo g, const float* __restrict__ wbar, float* __restrict__ pbx,
                                                     float* __restrict__ pby) {
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < g.vol; i += (size_t)gridDim.x * kThreads) {
    int h, w;
    coords(g, i, h, w);
    float gx, gy;
    grad_at(g, wbar, i, h, w, gx, gy);
    pbx[i] -= gx;
    pby[i] -= gy;
  }
}

// Tikhonov u' = c f:  fbar = dbar + c (ubar - dbar);  partials of lambda, rho
__global__ __launch_bounds__(kThreads) void tikb(size_t n, const float* __restrict__ ubar, const float* __restrict__ dbar,
                                                 const float* __restrict__ f, double c, double dc_dlam, double dc_drho,
                                                 float* __restrict__ fbar, double* __restrict__ part_lam,
                                                 double* __restrict__ part_rho) {
  double al = 0.0, ar = 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const double ut = (double)ubar[i] - (double)dbar[i];
    fbar[i] = (float)((double)dbar[i] + c * ut);
    al += ut * (double)f[i] * dc_dlam;
    ar += ut * (double)f[i] * dc_drho;
  }
  double s = block_sum(al);
  if (threadIdx.x == 0) part_lam[blockIdx.x] = s;
  __syncthreads();
  s = block_sum(ar);
  if (threadIdx.x == 0) part_rho[blockIdx.x] = s;
}

template <int R>
__global__ __launch_bounds__(kThreads) void xupdate_bwd(const ZSolve z, int periodic_lap, const uint32_t* __restrict__ bits,
                                                        int H, int W, int Wq, const float* __restrict__ fbar,
                                                        const float* __restrict__ xbar, const float* __restrict__ uk,
                                                        const float* __restrict__ dk, const float* __restrict__ fk,
                                                        float* __restrict__ ybar, float* __restrict__ ubar,
                                                        float* __restrict__ dbar, double* __restrict__ part_rho,
                                                        double* __restrict__ part_gam) {
  const size_t HW = (size_t)H * W;
  double ar = 0.0, ag = 0.0;
  for (size_t p = blockIdx.x * (size_t)kThreads + threadIdx.x; p < HW; p += (size_t)gridDim.x * kThreads) {
    const int h = (int)(p / W), w = (int)(p % W);
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
    double lam[R], xv[R];
    float fb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      fb[r] = fbar[r * HW + p];
      lam[r] = (double)fb[r] + (xbar ? (double)xbar[r * HW + p] : 0.0);
      xv[r] = (double)fk[r * HW + p] - (double)dk[r * HW + p];
    }
    xuimpl::pixel_solve<R>(z, m, lam);
    double yb = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((m >> r) & 1u) yb += lam[r];
      const double g = (double)uk[r * HW + p] - (double)dk[r * HW + p] - xv[r];
      ar += lam[r] * g;
      // (L x)_r: chain neighbours, plus the wrap pair when periodic
      double lx;
      if (R == 1) {
        lx = 0.0;
      } else if (periodic_lap) {
        const int rm = (r + R - 1) % R, rp = (r + 1) % R;
        lx = 2.0 * xv[r] - xv[rm] - xv[rp];
      } else {
        lx = (r > 0 ? xv[r] - xv[r - 1] : 0.0) + (r < R - 1 ? xv[r] - xv[r + 1] : 0.0);
      }
      ag -= lam[r] * lx;
      ubar[r * HW + p] = (float)(z.rho * lam[r]);
      dbar[r * HW + p] = (float)((double)fb[r] - z.rho * lam[r]);
    }
    ybar[p] += (float)yb;
  }
  double s = block_sum(ar);
  if (threadIdx.x == 0) part_rho[blockIdx.x] = s;
  __syncthreads();
  s = block_sum(ag);
  if (threadIdx.x == 0) part_gam[blockIdx.x] = s;
}

// The same for N > 1 shots: lam = A^{-1}(fbar + xbar) by the block elimination
// (A symmetric), ybar_j += m . lam_j per shot, (L x) over the chain of all N R slices.
template <int R>
__global__ __launch_bounds__(kThreads) void xupdate_bwd_ms(int N, double rho, double gamma, int periodic_solve,
                                                           int periodic_lap, const uint32_t* __restrict__ bits, int H,
                                                           int W, int Wq, const float* __restrict__ fbar,
                                                           const float* __restrict__ xbar, const float* __restrict__ uk,
                                                           const float* __restrict__ dk, const float* __restrict__ fk,
                                                           float* __restrict__ ybar, float* __restrict__ ubar,
                                                           float* __restrict__ dbar, double* __restrict__ part_rho,
                                                           double* __restrict__ part_gam, double* __restrict__ scratch) {
  const size_t HW = (size_t)H * W;
  const int NR = N * R;
  double ar = 0.0, ag = 0.0;
  for (size_t p = blockIdx.x * (size_t)kThreads + threadIdx.x; p < HW; p += (size_t)gridDim.x * kThreads) {
    const int h = (int)(p / W), w = (int)(p % W);
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
    auto xval = [&](int g) { return (double)fk[(size_t)g * HW + p] - (double)dk[(size_t)g * HW + p]; };
    double yb = 0.0;
    msimpl::solve<R>(
        m, N, rho, gamma, periodic_solve, HW, p, scratch,
        [&](int j, int r) {
          const size_t o = (size_t)(j * R + r) * HW + p;
          return (double)fbar[o] + (xbar ? (double)xbar[o] : 0.0);
        },
        [&](int g, double lam) {
          const size_t o = (size_t)g * HW + p;
          const int r = g % R;
          if ((m >> r) & 1u) yb += lam;
          if (r == R - 1) {
            ybar[(size_t)(g / R) * HW + p] += (float)yb;
            yb = 0.0;
          }
          const double xv = xval(g);
          ar += lam * ((double)uk[o] - (double)dk[o] - xv);
          double lx;
          if (NR == 1) {
            lx = 0.0;
          } else if (periodic_lap) {
            lx = 2.0 * xv - xval((g + NR - 1) % NR) - xval((g + 1) % NR);
          } else {
            lx = (g > 0 ? xv - xval(g - 1) : 0.0) + (g < NR - 1 ? xv - xval(g + 1) : 0.0);
          }
          ag -= lam * lx;
          ubar[o] = (float)(rho * lam);
          dbar[o] = (float)((double)fbar[o] - rho * lam);
        });
  }
  double s = block_sum(ar);
  if (threadIdx.x == 0) part_rho[blockIdx.x] = s;
  __syncthreads();
  s = block_sum(ag);
  if (threadIdx.x == 0) part_gam[blockIdx.x] = s;
}

// acc[slot] += sum(partial[0..n)) in a fixed order
__global__ void reduce_into(const double* __restrict__ partial, int n, double* __restrict__ acc, int slot) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[slot] += red[0];
}

// param_bar = [rho, lambda, gamma] from the accumulators [rho, lambda, gamma, theta]
__global__ void finish_params(const double* __restrict__ acc, double lam, double rho, int tv, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double r = acc[0], l = acc[1];
    if (tv) {
      l += acc[3] / rho;
      r -= acc[3] * lam / (rho * rho);
    }
    out[0] = r;
    out[1] = l;
    out[2] = acc[2];
  }
}

template <int... Rs>
struct RTab {
  template <typename F>
  static hipError_t dispatch(int R, F&& f) {
    hipError_t e = hipErrorInvalidValue;
    ((R == Rs ? (e = f(std::integral_constant<int, Rs>{}), true) : false) || ...);
    return e;
  }
};
using AllR = RTab<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27,
                  28, 29, 30, 31, 32>;

// ---- workspace layout -------------------------------------------------------

struct BwdLayout {
  size_t vol_bytes;
  int c;      // checkpoint interval
  int inner;  // TV inner iterations (0 for Tikhonov)
  size_t off_seg_u, off_seg_d, off_seg_f;  // c volumes each
  size_t off_tape_p;                        // (inner+1) x 2 volumes
  size_t off_tape_w;                        // inner volumes
  size_t off_adj;                           // ubar, dbar, fbar, pbx, pby, gbx, gby, wbar
  size_t off_part;                          // 3 x kGrid doubles
  size_t off_acc;                           // 4 doubles
  size_t total;
};

BwdLayout bwd_layout(const cspnp_plan& pl, const cspnp_params& p, int c) {
  BwdLayout L;
  const size_t vol = (size_t)pl.desc.N * pl.desc.R * pl.desc.H * pl.desc.W;
  L.vol_bytes = align_up(vol * sizeof(float));
  L.c = c;
  L.inner = pl.desc.denoiser == CSPNP_DENOISER_TV ? p.tv_inner : 0;
  size_t o = 0;
  L.off_seg_u = o; o += (size_t)c * L.vol_bytes;
  L.off_seg_d = o; o += (size_t)c * L.vol_bytes;
  L.off_seg_f = o; o += (size_t)c * L.vol_bytes;
  L.off_tape_p = o; o += (size_t)(L.inner + 1) * 2 * L.vol_bytes;
  L.off_tape_w = o; o += (size_t)L.inner * L.vol_bytes;
  L.off_adj = o; o += 8 * L.vol_bytes;
  L.off_part = o; o += align_up(3 * kGrid * sizeof(double));
  L.off_acc = o; o += align_up(4 * sizeof(double));
  // the forward recompute's denoiser workspace (multi-pass TV only)
  o += align_up(tv_workspace_bytes(pl, p.tv_inner));
  L.total = o;
  return L;
}

size_t ckpt_slots(int iters, int c) { return (size_t)((iters + c - 1) / c); }

hipError_t launch_fill(float* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero, dim3(kGrid), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t enqueue_denoise_fwd(const cspnp_plan& pl, const cspnp_params& p, const float* f, float* u, float* d,
                               void* dws, hipStream_t s) {
  if (pl.desc.denoiser == CSPNP_DENOISER_TV)
    return launch_tv(pl, p.lambda, p.rho, p.tv_inner, p.tv_tau, f, u, d, dws, s);
  return launch_tikhonov(pl, p.lambda, p.rho, f, u, d, s);
}

#define TRY(x)                            \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

hipError_t enqueue_backward(const cspnp_plan& pl, const cspnp_params& p, const float* y, int c, const float* ckpt,
                            const float* xbar, float* ybar, double* param_bar, char* ws, hipStream_t s) {
  const auto& de = pl.desc;
  const BwdLayout L = bwd_layout(pl, p, c);
  const size_t vol = (size_t)de.N * de.R * de.H * de.W;
  const size_t frame = (size_t)de.N * de.H * de.W;
  auto V = [&](size_t off, size_t k) { return reinterpret_cast<float*>(ws + off + k * L.vol_bytes); };
  float* ubar = V(L.off_adj, 0);
  float* dbar = V(L.off_adj, 1);
  float* fbar = V(L.off_adj, 2);
  float* pbx = V(L.off_adj, 3);
  float* pby = V(L.off_adj, 4);
  float* gbx = V(L.off_adj, 5);
  float* gby = V(L.off_adj, 6);
  float* wbar = V(L.off_adj, 7);
  double* part = reinterpret_cast<double*>(ws + L.off_part);
  double* acc = reinterpret_cast<double*>(ws + L.off_acc);
  void* dws = ws + L.off_acc + align_up(4 * sizeof(double));
  Geo g{de.H, de.W, (size_t)de.H * de.W, vol};
  const ZSolve zs = make_zsolve(de.R, de.zbc, p.rho, p.gamma);
  const int periodic_lap = (de.zbc == CSPNP_ZBC_PERIODIC) ? 1 : 0;
  const double theta = p.lambda / p.rho;
  const bool tv = de.denoiser == CSPNP_DENOISER_TV;
  const float thetaf = (float)theta;
  const float inv_theta = theta > 0 ? (float)(1.0 / theta) : 0.f;
  const float tau = (float)p.tv_tau;
  const int K = p.iters;
  const dim3 G(kGrid), B(kThreads);

  TRY(launch_fill(ybar, frame, s));
  TRY(launch_fill(ubar, vol, s));
  TRY(launch_fill(dbar, vol, s));
  hipLaunchKernelGGL(zero_doubles, dim3(1), dim3(64), 0, s, acc, 4);
  TRY(hipGetLastError());
  const int nseg = (int)ckpt_slots(K, c);
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int k0 = sg * c, k1 = std::min(K, k0 + c), len = k1 - k0;
    // recompute the segment from its checkpoint
    TRY(hipMemcpyAsync(V(L.off_seg_u, 0), ckpt + (size_t)(2 * sg) * vol, vol * 4, hipMemcpyDeviceToDevice, s));
    TRY(hipMemcpyAsync(V(L.off_seg_d, 0), ckpt + (size_t)(2 * sg + 1) * vol, vol * 4, hipMemcpyDeviceToDevice, s));
    for (int i = 0; i < len; ++i) {
      TRY(launch_xupdate(pl, zs, y, V(L.off_seg_u, i), V(L.off_seg_d, i), nullptr, V(L.off_seg_f, i), s));
      if (i + 1 < len) TRY(enqueue_denoise_fwd(pl, p, V(L.off_seg_f, i), V(L.off_seg_u, i + 1), V(L.off_seg_d, i + 1), dws, s));
    }
    for (int i = len - 1; i >= 0; --i) {
      const int k = k0 + i;
      const float* fk = V(L.off_seg_f, i);
      if (k == K - 1) {
        TRY(launch_fill(fbar, vol, s));  // x^K does not depend on u^K, d^K
      } else if (tv && theta > 0 && L.inner > 0) {
        // rebuild the TV tape p^0..p^n, w^0..w^{n-1}
        float* P0x = V(L.off_tape_p, 0);
        float* P0y = V(L.off_tape_p, 1);
        TRY(launch_fill(P0x, vol, s));
        TRY(launch_fill(P0y, vol, s));
        for (int t = 0; t < L.inner; ++t) {
          hipLaunchKernelGGL(tvb_w, G, B, 0, s, g, V(L.off_tape_p, 2 * t), V(L.off_tape_p, 2 * t + 1), fk, inv_theta,
                             V(L.off_tape_w, t));
          hipLaunchKernelGGL(tvb_p, G, B, 0, s, g, V(L.off_tape_w, t), V(L.off_tape_p, 2 * t), V(L.off_tape_p, 2 * t + 1),
                             tau, V(L.off_tape_p, 2 * t + 2), V(L.off_tape_p, 2 * t + 3));
        }
        hipLaunchKernelGGL(tvb_init, G, B, 0, s, g, ubar, dbar, V(L.off_tape_p, 2 * L.inner),
                           V(L.off_tape_p, 2 * L.inner + 1), thetaf, fbar, pbx, pby, part);
        hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part, kGrid, acc, 3);
        for (int t = L.inner - 1; t >= 0; --t) {
          hipLaunchKernelGGL(tvb_g, G, B, 0, s, g, V(L.off_tape_w, t), V(L.off_tape_p, 2 * t + 2),
                             V(L.off_tape_p, 2 * t + 3), tau, pbx, pby, gbx, gby);
          hipLaunchKernelGGL(tvb_wbar, G, B, 0, s, g, gbx, gby, fk, thetaf, wbar, fbar, part);
          hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part, kGrid, acc, 3);
          hipLaunchKernelGGL(tvb_pbar, G, B, 0, s, g, wbar, pbx, pby);
        }
        TRY(hipGetLastError());
      } else if (tv) {
        // zero prox weight or no inner iteration: u' = f exactly, fbar = dbar + (ubar - dbar) = ubar
        TRY(hipMemcpyAsync(fbar, ubar, vol * 4, hipMemcpyDeviceToDevice, s));
      } else {
        const double den = 2.0 * p.lambda + p.rho;
        hipLaunchKernelGGL(tikb, G, B, 0, s, vol, ubar, dbar, fk, p.rho / den, -2.0 * p.rho / (den * den),
                           2.0 * p.lambda / (den * den), fbar, part, part + kGrid);
        hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part, kGrid, acc, 1);
        hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part + kGrid, kGrid, acc, 0);
        TRY(hipGetLastError());
      }
      TRY(AllR::dispatch(de.R, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        if (de.N == 1) {
          hipLaunchKernelGGL(xupdate_bwd<R>, G, B, 0, s, zs, periodic_lap, pl.bits, de.H, de.W, pl.Wq, fbar,
                             k == K - 1 ? xbar : nullptr, V(L.off_seg_u, i), V(L.off_seg_d, i), fk, ybar, ubar, dbar,
                             part, part + kGrid);
        } else {
          const int periodic_solve = (periodic_lap && de.N * de.R >= 2 && p.gamma > 0) ? 1 : 0;
          hipLaunchKernelGGL(xupdate_bwd_ms<R>, G, B, 0, s, de.N, p.rho, p.gamma, periodic_solve, periodic_lap,
                             pl.bits, de.H, de.W, pl.Wq, fbar, k == K - 1 ? xbar : nullptr, V(L.off_seg_u, i),
                             V(L.off_seg_d, i), fk, ybar, ubar, dbar, part, part + kGrid, pl.ms_scratch);
        }
        return hipGetLastError();
      }));
      hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part, kGrid, acc, 0);
      hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part + kGrid, kGrid, acc, 2);
      TRY(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(finish_params, dim3(1), dim3(64), 0, s, acc, p.lambda, p.rho, tv ? 1 : 0, param_bar);
  return hipGetLastError();
}

int validate_diff(const cspnp_plan* plan, const cspnp_params* p, int c) {
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, p)) return s;
  if (c < 1) return fail(CSPNP_EINVAL, "ckpt_every must be >= 1");
  if (plan->desc.denoiser == CSPNP_DENOISER_BM3D)
    return fail(CSPNP_EUNSUPPORTED, "the backward is implemented for the TV and Tikhonov denoisers");
  if (plan->desc.denoiser == CSPNP_DENOISER_TV && p->tv_inner > 16)
    return fail(CSPNP_EUNSUPPORTED, "the backward supports tv_inner <= 16");
  return CSPNP_OK;
}

size_t solve_ws(const cspnp_plan& pl, const cspnp_params& p) {
  size_t n = 0;
  (void)cspnp_workspace_size(&pl, &p, CSPNP_WS_SOLVE, &n);
  return n;
}

}  // namespace

CSPNP_API int cspnp_ckpt_size(const cspnp_plan* plan, const cspnp_params* params, int ckpt_every, size_t* bytes) {
  clear_error();
  if (int s = validate_diff(plan, params, ckpt_every)) return s;
  if (!bytes) return fail(CSPNP_EINVAL, "bytes is NULL");
  const size_t vol = (size_t)plan->desc.N * plan->desc.R * plan->desc.H * plan->desc.W;
  *bytes = ckpt_slots(params->iters, ckpt_every) * 2 * vol * sizeof(float);
  return CSPNP_OK;
}

CSPNP_API int cspnp_bwd_workspace_size(const cspnp_plan* plan, const cspnp_params* params, int ckpt_every,
                                       size_t* bytes) {
  clear_error();
  if (int s = validate_diff(plan, params, ckpt_every)) return s;
  if (!bytes) return fail(CSPNP_EINVAL, "bytes is NULL");
  *bytes = bwd_layout(*plan, *params, ckpt_every).total;
  return CSPNP_OK;
}

CSPNP_API int cspnp_solve_ckpt(const cspnp_plan* plan, const cspnp_params* params, const float* y, float* u, float* d,
                               float* x, int ckpt_every, float* ckpt, void* ws, void* stream) {
  clear_error();
  if (int s = validate_diff(plan, params, ckpt_every)) return s;
  if (params->iters < 1) return fail(CSPNP_EINVAL, "iters must be >= 1 for the differentiable solve");
  if (check_ptr(ckpt, "ckpt")) return CSPNP_EINVAL;
  const size_t vol = (size_t)plan->desc.N * plan->desc.R * plan->desc.H * plan->desc.W;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int K = params->iters, c = ckpt_every;
  cspnp_params seg = *params;
  seg.flags |= CSPNP_FLAG_NO_GRAPH;
  for (int k0 = 0; k0 < K; k0 += c) {
    const size_t slot = (size_t)(k0 / c);
    CSPNP_HIP(hipMemcpyAsync(ckpt + 2 * slot * vol, u, vol * 4, hipMemcpyDeviceToDevice, st));
    CSPNP_HIP(hipMemcpyAsync(ckpt + (2 * slot + 1) * vol, d, vol * 4, hipMemcpyDeviceToDevice, st));
    seg.iters = std::min(c, K - k0);
    // x is written by the segment's last iteration; the final segment leaves x^K
    if (int s = cspnp_solve(plan, &seg, y, u, d, x, ws, stream)) return s;
  }
  return CSPNP_OK;
}

CSPNP_API int cspnp_solve_bwd(const cspnp_plan* cplan, const cspnp_params* params, const float* y, int ckpt_every,
                              const float* ckpt, const float* x_bar, float* y_bar, double* param_bar, void* ws,
                              void* stream) {
  clear_error();
  if (int s = validate_diff(cplan, params, ckpt_every)) return s;
  if (params->iters < 1) return fail(CSPNP_EINVAL, "iters must be >= 1 for the backward");
  if (check_ptr(y, "y") || check_ptr(ckpt, "ckpt") || check_ptr(x_bar, "x_bar") || check_ptr(y_bar, "y_bar"))
    return CSPNP_EINVAL;
  if (param_bar == nullptr || reinterpret_cast<uintptr_t>(param_bar) % 8)
    return fail(CSPNP_EINVAL, "param_bar must be an 8-byte aligned device pointer");
  if (ws == nullptr || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  CSPNP_HIP(enqueue_backward(*cplan, *params, y, ckpt_every, ckpt, x_bar, y_bar, param_bar, static_cast<char*>(ws), st));
  return CSPNP_OK;
}
