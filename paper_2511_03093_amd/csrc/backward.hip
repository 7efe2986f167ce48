// Reverse mode through the unrolled ADMM iterations (the library's
// differentiable solve): gradients of <xbar, x^K> with respect to the frames y
// and the scalars rho, lambda, gamma.
//
// Forward (cspnp_solve_ckpt): the usual iteration, storing (u, d) at the start
// of every segment of `ckpt_every` iterations.  Backward (cspnp_solve_bwd):
// segments in reverse; each is recomputed from its checkpoint keeping
// (u^k, d^k, f^{k+1}), then its iterations are reversed:
//   d' = f - u', u' = D_theta(f):   fbar = dbar' + D^T(ubar' - dbar')
//   TV (Chambolle from p = 0): the fused forward tile writes the inner iterates
//   p^1..p^K to a tape, and one tile kernel reverses all K inner steps with the
//   adjoint in registers:  gbar = (tau/s)(pbar' - (pbar'.p') g/|g|),
//   wbar = -div gbar, pbar = pbar'/s - grad wbar,  fbar -= wbar/theta,
//   thetabar += <wbar, f/theta^2>; the output step u = f - theta div p^K gives
//   fbar += ubar, pbar^K = theta grad ubar, thetabar -= <ubar, div p^K>.
//   x-step x = A^{-1}(m y + rho (u - d)), A symmetric:  lam = A^{-1}(fbar + xbar),
//   ybar += m.lam, ubar = rho lam, dbar = fbar - rho lam,
//   rhobar += <lam, u - d - x>, gammabar -= <lam, L x>.
// Scalar sums are FP64 block partials reduced in a fixed order (deterministic).
#include <algorithm>
#include <vector>

#include "multishot_impl.hpp"
#include "tv_impl.hpp"
#include "xupdate_impl.hpp"

namespace cspnp {
ZSolve make_zsolve(int R, int zbc, double rho, double gamma);
}

using namespace cspnp;

namespace {

constexpr int kThreads = 256;
constexpr int kGrid = 1024;  // fixed grid of the grid-stride kernels (one FP64 partial per block)
constexpr int kMsLanes = 64;              // N > 1 x-step VJP: one wave per workgroup on the LDS path
constexpr size_t kMsMaxLds = 80 * 1024;  // its LDS block: N R <= 64

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

// ---- reverse of the TV u-step, all inner steps in one tile --------------------
// One workgroup per (tile, slice); lane L of wave k holds the S x CX pixels of rows
// k*S.. and columns L*CX.. of the tile.  The adjoint pbar stays in registers
// through all K reverse steps; f/theta and the fbar accumulator sit in LDS (each
// lane reads back only what it wrote), which keeps the step free of register
// spills at four waves per SIMD.  Step t reads p^t of
// the strip's rows -1..S from the tape (p^0 = 0) and recomputes w^t, g, 1/s and
// p^{t+1} in the forward tile's operation order; two LDS exchanges per step carry
// the last-row gbar_y of each strip down and the first-row wbar up.  Each step
// spreads the error of the unknown values beyond the tile one pixel inward and the
// output step one more, so tiles overlap by K + 1 pixels and write only their
// interior.  Per step, with p' = (p + tau g)/s:
//   gbar = (tau/s)(pbar - (pbar.p') g/|g|),  wbar = -div gbar,  pbar <- pbar/s - grad wbar,
//   fbar -= wbar/theta,  thetabar += <wbar, f/theta^2>;
// output step u = f - theta div p^K:  fbar = ubar, pbar = theta grad(ubar - dbar),
//   thetabar -= <ubar - dbar, div p^K>   (fbar starts at dbar + (ubar - dbar)).
struct TvbArgs {
  const float* f;     // f^{k+1}, NR*H*W
  const float* ubar;  // cotangent of u' (of the slice volume)
  const float* dbar;  // cotangent of d' = f - u'
  const float* tape;  // px^t at tape + 2 t stride, py^t at tape + (2 t + 1) stride, t = 1..K
  size_t stride;
  float* fbar;
  double* part;  // one FP64 partial of thetabar per workgroup
  int H, W, tilesX, IX, IY, halo, K;
  float theta, inv_theta, tau;
};

constexpr int kTvbCX = 2, kTvbS = 7, kTvbNW = 16;

template <int CX, int S, int NW>
__global__ __launch_bounds__(64 * NW) void tvb_tile(const TvbArgs a) {
#pragma clang fp contract(off)
  using namespace tvimpl;
  // Each exchange buffer is written and read between two barriers that separate it
  // from its next write, so one copy of each suffices.
  __shared__ float xg[NW][64 * CX];  // gbar_y of each strip's last row
  __shared__ float xw[NW][64 * CX];  // wbar of each strip's first row
  __shared__ double red[NW];
  // per-lane state kept in LDS (each lane reads only what it wrote): f/theta of the
  // strip rows 0..S and the fbar accumulator
  __shared__ float fsl[NW][S + 1][64][CX];
  __shared__ float fbl[NW][S][64][CX];
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  const int tx = blockIdx.x % a.tilesX, ty = blockIdx.x / a.tilesX;
  const size_t base = (size_t)blockIdx.y * a.H * a.W;
  const int ox = tx * a.IX - a.halo, oy = ty * a.IY - a.halo;
  const int c0 = ox + L * CX, r0 = oy + k * S;  // r0 wave-uniform

  uint32_t coff[CX];
  bool cin[CX], cgx[CX], cxl[CX], cout[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) {
    const int gc = c0 + c;
    coff[c] = 4u * (uint32_t)min(max(gc, 0), a.W - 1);
    cin[c] = gc >= 0 && gc < a.W;
    cgx[c] = gc >= 0 && gc < a.W - 1;  // the pixel has an x-gradient
    cxl[c] = gc >= 1 && gc < a.W;      // its left neighbour is in the image
    const int tcc = L * CX + c;
    cout[c] = tcc >= a.halo && tcc < a.halo + a.IX && gc < a.W;
  }
  auto row_off = [&](int s) -> uint32_t { return 4u * (uint32_t)min(max(r0 + s, 0), a.H - 1) * (uint32_t)a.W; };
  auto rin = [&](int s) { return r0 + s >= 0 && r0 + s < a.H; };
  auto rgy = [&](int s) { return r0 + s >= 0 && r0 + s < a.H - 1; };
  auto ryu = [&](int s) { return r0 + s >= 1 && r0 + s < a.H; };
  auto rout = [&](int s) {
    const int tr = k * S + s;
    return tr >= a.halo && tr < a.halo + a.IY && r0 + s < a.H;
  };

  const Rsrc fr = slice_rsrc(a.f + base, a.H, a.W);
  const Rsrc ur = slice_rsrc(a.ubar + base, a.H, a.W);
  const Rsrc dr = slice_rsrc(a.dbar + base, a.H, a.W);
  float bx[S][CX], by[S][CX];
  auto fs = [&](int s) -> float(&)[CX] { return fsl[k][s][L]; };
  double acc = 0.0;
  {
    float ut[S + 1][CX];
#pragma unroll
    for (int s = 0; s <= S; ++s) {
      const uint32_t ro = row_off(s);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float fv = ld(fr, coff[c], ro), uv = ld(ur, coff[c], ro), dv = ld(dr, coff[c], ro);
        const bool in = rin(s) && cin[c];
        fs(s)[c] = in ? __fmul_rn(fv, a.inv_theta) : 0.f;
        ut[s][c] = uv - dv;
        if (s < S) fbl[k][s][L][c] = uv;
      }
    }
    // p^K for the output step's thetabar term
    const Rsrc kx = slice_rsrc(a.tape + (size_t)(2 * a.K) * a.stride + base, a.H, a.W);
    const Rsrc ky = slice_rsrc(a.tape + (size_t)(2 * a.K + 1) * a.stride + base, a.H, a.W);
    float pyu[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) pyu[c] = ryu(0) ? ld(ky, coff[c], row_off(-1)) : 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t ro = row_off(s);
      float pxs[CX], pys[CX];
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        pxs[c] = ld(kx, coff[c], ro);
        pys[c] = ld(ky, coff[c], ro);
      }
      const float left = from_left(pxs[CX - 1]);
      const float right = from_right(ut[s][0]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        // pbar^K = theta grad(ut), Neumann ends
        const float utr = (c < CX - 1) ? ut[s][c + 1] : right;
        bx[s][c] = a.theta * ((cgx[c] ? utr : ut[s][c]) - ut[s][c]);
        by[s][c] = a.theta * ((rgy(s) ? ut[s + 1][c] : ut[s][c]) - ut[s][c]);
        const float pxl = cxl[c] ? ((c > 0) ? pxs[c - 1] : left) : 0.f;
        const float pxc = cgx[c] ? pxs[c] : 0.f;
        const float pyc = rgy(s) ? pys[c] : 0.f;
        const float pu = ryu(s) ? pyu[c] : 0.f;
        if (rout(s) && cout[c]) acc -= (double)ut[s][c] * (double)((pxc - pxl) + (pyc - pu));
      }
#pragma unroll
      for (int c = 0; c < CX; ++c) pyu[c] = pys[c];
    }
  }

  const float tau = a.tau;
  const double itheta = 1.0 / (double)a.theta;
  for (int t = a.K - 1; t >= 0; --t) {
    // p^t row by row (p^0 = 0; zero outside the image), w^t in the forward tile's
    // operation order, then gbar and pbar <- pbar / s for each row of the strip
    const bool tp = t > 0;
    const Rsrc tx_ = slice_rsrc(a.tape + (size_t)(2 * t) * a.stride + base, a.H, a.W);
    const Rsrc ty_ = slice_rsrc(a.tape + (size_t)(2 * t + 1) * a.stride + base, a.H, a.W);
    // all of the step's tape loads are issued first, so their latencies overlap
    float tpx[S + 1][CX], tpy[S + 2][CX];  // px rows 0..S, py rows -1..S
#pragma unroll
    for (int s = -1; s <= S; ++s) {
      const uint32_t ro = row_off(s);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        if (s >= 0) tpx[s][c] = ld(tx_, coff[c], ro);  // in-bounds (clamped); masked below
        tpy[s + 1][c] = ld(ty_, coff[c], ro);
      }
    }
    // keep the loads together (one wait for all of them, not one per row)
#pragma unroll
    for (int s = 0; s <= S + 1; ++s)
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        if (s <= S) asm volatile("" : "+v"(tpx[s][c]));
        asm volatile("" : "+v"(tpy[s][c]));
      }
    auto mrow = [&](int s, float& v, int c) { v = (tp && rin(s) && cin[c]) ? v : 0.f; };
    auto wrow = [&](const float (&pxr)[CX], const float (&pyr)[CX], const float (&pyup)[CX], int s, float (&wr)[CX]) {
      const float left = from_left(pxr[CX - 1]);
      float fr_[CX];
#pragma unroll
      for (int c = 0; c < CX; ++c) fr_[c] = fs(s)[c];
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float pxl = (c > 0) ? pxr[c - 1] : left;
        wr[c] = (((pxr[c] - pxl) + pyr[c]) - pyup[c]) - fr_[c];
      }
    };
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      mrow(-1, tpy[0][c], c);
      mrow(0, tpx[0][c], c);
      mrow(0, tpy[1][c], c);
    }
    float wc[CX];
    wrow(tpx[0], tpy[1], tpy[0], 0, wc);
    float gbx[S][CX], gby[S][CX];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float wn[CX];
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        mrow(s + 1, tpx[s + 1][c], c);
        mrow(s + 1, tpy[s + 2][c], c);
      }
      wrow(tpx[s + 1], tpy[s + 2], tpy[s + 1], s + 1, wn);
      const float right = from_right(wc[0]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float wr = (c < CX - 1) ? wc[c + 1] : right;
        const float gx = cgx[c] ? (wr - wc[c]) : 0.f;
        const float gy = rgy(s) ? (wn[c] - wc[c]) : 0.f;
        const float q = fmaf(gx, gx, gy * gy);
        const float mag = __builtin_amdgcn_sqrtf(q);
        const float rs = __builtin_amdgcn_rcpf(fmaf(tau, mag, 1.f));
        const float qx = fmaf(tau, gx, tpx[s][c]) * rs;  // p^{t+1}
        const float qy = fmaf(tau, gy, tpy[s + 1][c]) * rs;
        const float av = bx[s][c] * qx + by[s][c] * qy;
        float nx = 0.f, ny = 0.f;
        if (mag > 0.f) {
          const float im = __builtin_amdgcn_rcpf(mag);
          nx = gx * im;
          ny = gy * im;
        }
        const float trs = tau * rs;
        gbx[s][c] = trs * (bx[s][c] - av * nx);
        gby[s][c] = trs * (by[s][c] - av * ny);
        bx[s][c] = bx[s][c] * rs;
        by[s][c] = by[s][c] * rs;
      }
#pragma unroll
      for (int c = 0; c < CX; ++c) wc[c] = wn[c];
    }
#pragma unroll
    for (int c = 0; c < CX; ++c) xg[k][L * CX + c] = gby[S - 1][c];
    __syncthreads();
    // wbar = -div gbar;  fbar -= wbar/theta;  thetabar += <wbar, f/theta^2>
    float wb[S][CX];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float left = from_left(gbx[s][CX - 1]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float xl = cxl[c] ? ((c > 0) ? gbx[s][c - 1] : left) : 0.f;
        const float xc = cgx[c] ? gbx[s][c] : 0.f;
        const float yc = rgy(s) ? gby[s][c] : 0.f;
        const float yu = ryu(s) ? ((s > 0) ? gby[s - 1][c] : ((k > 0) ? xg[k - 1][L * CX + c] : 0.f)) : 0.f;
        const float v = -((xc - xl) + (yc - yu));
        wb[s][c] = v;
        fbl[k][s][L][c] = fbl[k][s][L][c] - v * a.inv_theta;
        if (rout(s) && cout[c]) acc += (double)v * (double)fs(s)[c] * itheta;
      }
    }
#pragma unroll
    for (int c = 0; c < CX; ++c) xw[k][L * CX + c] = wb[0][c];
    __syncthreads();
    // pbar -= grad wbar
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float right = from_right(wb[s][0]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float wr = (c < CX - 1) ? wb[s][c + 1] : right;
        const float wd = (s < S - 1) ? wb[s + 1][c] : ((k < NW - 1) ? xw[k + 1][L * CX + c] : 0.f);
        const float gx = cgx[c] ? (wr - wb[s][c]) : 0.f;
        const float gy = rgy(s) ? (wd - wb[s][c]) : 0.f;
        bx[s][c] = bx[s][c] - gx;
        by[s][c] = by[s][c] - gy;
      }
    }
  }
  // interior fbar, and the workgroup's thetabar partial (fixed-order reduction)
  const Rsrc fo = slice_rsrc(a.fbar + base, a.H, a.W);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (!rout(s)) continue;
    const uint32_t ro = row_off(s);
#pragma unroll
    for (int c = 0; c < CX; ++c)
      if (cout[c]) st(fbl[k][s][L][c], fo, coff[c], ro);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (L == 0) red[k] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < NW; ++i) sum += red[i];
    a.part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sum;
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
  using xuimpl::ld_at;
  using xuimpl::st_at;
  // slice accesses as scalar base + 32-bit lane offset (H W <= 2^30)
  const uint32_t HW = (uint32_t)H * (uint32_t)W;
  const size_t HWs = HW;
  double ar = 0.0, ag = 0.0;
  for (uint32_t p = blockIdx.x * kThreads + threadIdx.x; p < HW; p += gridDim.x * kThreads) {
    // slice bases are formed afresh in every pass (the empty asm hides the
    // pointers' identity): hoisted out of the loop, 7 R of them would not fit
    // the scalar registers
    const uint32_t* bits_ = bits;
    const float *fbar_ = fbar, *xbar_ = xbar, *uk_ = uk, *dk_ = dk, *fk_ = fk;
    float *ubar_ = ubar, *dbar_ = dbar;
    asm volatile("" : "+s"(bits_), "+s"(fbar_), "+s"(xbar_), "+s"(uk_), "+s"(dk_), "+s"(fk_), "+s"(ubar_), "+s"(dbar_));
    const uint32_t h = p / (uint32_t)W, w = p - h * (uint32_t)W;
    const uint32_t off = 4u * p, boff = 4u * (h * (uint32_t)Wq + (w >> 5)), bit = w & 31u;
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) m |= ((ld_at(bits_ + (size_t)r * H * Wq, boff) >> bit) & 1u) << r;
    double lam[R];
    float fb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      fb[r] = ld_at(fbar_ + r * HWs, off);
      lam[r] = (double)fb[r] + (xbar_ ? (double)ld_at(xbar_ + r * HWs, off) : 0.0);
    }
    xuimpl::pixel_solve<R>(z, m, lam);
    // The state loads go after the solve (not hoisted above it): with both groups
    // live at once the kernel needed ~450 registers, one wave per SIMD.
    asm volatile("" ::: "memory");
    float uv[R], dv[R], fv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uv[r] = ld_at(uk_ + r * HWs, off);
      dv[r] = ld_at(dk_ + r * HWs, off);
      fv[r] = ld_at(fk_ + r * HWs, off);
    }
    auto xv = [&](int r) { return (double)fv[r] - (double)dv[r]; };  // x^{k+1} = f - d
    double yb = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((m >> r) & 1u) yb += lam[r];
      const double g = (double)uv[r] - (double)dv[r] - xv(r);
      ar += lam[r] * g;
      // (L x)_r: chain neighbours, plus the wrap pair when periodic
      double lx;
      if (R == 1) {
        lx = 0.0;
      } else if (periodic_lap) {
        const int rm = (r + R - 1) % R, rp = (r + 1) % R;
        lx = 2.0 * xv(r) - xv(rm) - xv(rp);
      } else {
        lx = (r > 0 ? xv(r) - xv(r - 1) : 0.0) + (r < R - 1 ? xv(r) - xv(r + 1) : 0.0);
      }
      ag -= lam[r] * lx;
      st_at(ubar_ + r * HWs, off, (float)(z.rho * lam[r]));
      st_at(dbar_ + r * HWs, off, (float)((double)fb[r] - z.rho * lam[r]));
    }
    float* yo = ybar;
    st_at(yo, off, ld_at((const float*)yo, off) + (float)yb);
  }
  double s = block_sum(ar);
  if (threadIdx.x == 0) part_rho[blockIdx.x] = s;
  __syncthreads();
  s = block_sum(ag);
  if (threadIdx.x == 0) part_gam[blockIdx.x] = s;
}

// Sum over one wave (blocks of 64 threads); lane 0 returns it.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// The same for N > 1 shots: lam = A^{-1}(fbar + xbar) by the block elimination
// (A symmetric), ybar_j += m . lam_j per shot, (L x) over the chain of all N R slices.
// LDS: one wave per workgroup keeps its pixels' forward vectors ([2][NR][64] doubles)
// and the fbar values of the right-hand side ([NR][64] floats) in LDS; otherwise the
// vectors live in the plan's HBM scratch volume (the periodic wrap's always does).
// x^k = f - d is loaded once per slice: each block keeps its R values and the
// neighbours across block boundaries are carried from the block before (and the
// first block of the next one loaded ahead).
template <int R, bool LDS>
__global__ __launch_bounds__(kThreads) void xupdate_bwd_ms(int N, double rho, double gamma, int periodic_solve,
                                                           int periodic_lap, const uint32_t* __restrict__ bits, int H,
                                                           int W, int Wq, const float* __restrict__ fbar,
                                                           const float* __restrict__ xbar, const float* __restrict__ uk,
                                                           const float* __restrict__ dk, const float* __restrict__ fk,
                                                           float* __restrict__ ybar, float* __restrict__ ubar,
                                                           float* __restrict__ dbar, double* __restrict__ part_rho,
                                                           double* __restrict__ part_gam, double* __restrict__ scratch) {
  extern __shared__ double lds_scratch[];
  const size_t HW = (size_t)H * W;
  const int NR = N * R;
  float* const fl = reinterpret_cast<float*>(lds_scratch + 2 * (size_t)NR * blockDim.x);
  double ar = 0.0, ag = 0.0;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < HW; p += (size_t)gridDim.x * blockDim.x) {
    const int h = (int)(p / W), w = (int)(p % W);
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
    auto xval = [&](int g) { return (double)fk[(size_t)g * HW + p] - (double)dk[(size_t)g * HW + p]; };
    struct Raw {
      float fb[R], xb[R];
      int j;
    };
    // x of the slice before the current block (periodic: the chain's last slice before block 0)
    double x_before = (periodic_lap && NR > 1) ? xval(NR - 1) : 0.0, x_first = 0.0;
    auto fetch = [&](int j, Raw& raw) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const size_t o = (size_t)(j * R + r) * HW + p;
        raw.fb[r] = fbar[o];
        raw.xb[r] = xbar ? xbar[o] : 0.f;
      }
      raw.j = j;
    };
    auto rhs = [&](const Raw& raw, int r) {
      if constexpr (LDS) fl[(size_t)(raw.j * R + r) * blockDim.x + threadIdx.x] = raw.fb[r];
      return (double)raw.fb[r] + (xbar ? (double)raw.xb[r] : 0.0);
    };
    auto out = [&](int j, const double (&lamj)[R]) {
      double xs[R], uv[R];
      float fb[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const size_t o = (size_t)(j * R + r) * HW + p;
        xs[r] = xval(j * R + r);
        uv[r] = (double)uk[o] - (double)dk[o];
        fb[r] = LDS ? fl[(size_t)(j * R + r) * blockDim.x + threadIdx.x] : fbar[o];
      }
      if (j == 0) x_first = xs[0];
      // x of the slice after the block: the next block's first, or (periodic) the chain's first
      const double x_after = j + 1 < N ? xval((j + 1) * R) : (periodic_lap ? x_first : 0.0);
      double yb = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int g = j * R + r;
        const double lam = lamj[r];
        const size_t o = (size_t)g * HW + p;
        if ((m >> r) & 1u) yb += lam;
        const double xv = xs[r];
        ar += lam * (uv[r] - xv);
        const double xm = r > 0 ? xs[r - 1] : x_before, xp = r < R - 1 ? xs[r + 1] : x_after;
        double lx;
        if (NR == 1) {
          lx = 0.0;
        } else if (periodic_lap) {
          lx = 2.0 * xv - xm - xp;
        } else {
          lx = (g > 0 ? xv - xm : 0.0) + (g < NR - 1 ? xv - xp : 0.0);
        }
        ag -= lam * lx;
        ubar[o] = (float)(rho * lam);
        dbar[o] = (float)((double)fb[r] - rho * lam);
      }
      ybar[(size_t)j * HW + p] += (float)yb;
      x_before = xs[R - 1];
    };
    double* const yw = scratch + 2 * (size_t)NR * HW;
    if constexpr (LDS)
      msimpl::solve<R, Raw>(m, N, rho, gamma, periodic_solve, blockDim.x, threadIdx.x, lds_scratch, yw, HW, p, fetch,
                            rhs, out);
    else
      msimpl::solve<R, Raw>(m, N, rho, gamma, periodic_solve, HW, p, scratch, yw, HW, p, fetch, rhs, out);
  }
  if constexpr (LDS) {
    const double s = wave_sum(ar), t = wave_sum(ag);
    if (threadIdx.x == 0) {
      part_rho[blockIdx.x] = s;
      part_gam[blockIdx.x] = t;
    }
  } else {
    double s = block_sum(ar);
    if (threadIdx.x == 0) part_rho[blockIdx.x] = s;
    __syncthreads();
    s = block_sum(ag);
    if (threadIdx.x == 0) part_gam[blockIdx.x] = s;
  }
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

struct TvbGrid {
  int halo, IX, IY, tilesX, tiles;
};
TvbGrid tvb_grid(int H, int W, int inner) {
  TvbGrid g;
  g.halo = inner + 1;
  g.IX = 64 * kTvbCX - 2 * g.halo;
  g.IY = kTvbNW * kTvbS - 2 * g.halo;
  g.tilesX = (W + g.IX - 1) / g.IX;
  g.tiles = g.tilesX * ((H + g.IY - 1) / g.IY);
  return g;
}

// ---- workspace layout -------------------------------------------------------

struct BwdLayout {
  size_t vol_bytes;
  int c;      // checkpoint interval
  int inner;  // TV inner iterations (0 for Tikhonov)
  size_t off_seg_u, off_seg_d, off_seg_f;  // c volumes each
  size_t off_tape_p;                        // (inner+1) x 2 volumes: p^t at 2t, 2t+1 (t >= 1)
  size_t off_adj;                           // ubar, dbar, fbar
  size_t off_part;                          // max(3 kGrid, TV tiles) doubles
  size_t n_part;
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
  L.off_adj = o; o += 3 * L.vol_bytes;
  L.n_part = 3 * (size_t)kGrid;
  if (L.inner > 0)
    L.n_part = std::max(L.n_part, (size_t)tvb_grid(pl.desc.H, pl.desc.W, L.inner).tiles * pl.desc.N * pl.desc.R);
  L.off_part = o; o += align_up(L.n_part * sizeof(double));
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
  double* part = reinterpret_cast<double*>(ws + L.off_part);
  double* acc = reinterpret_cast<double*>(ws + L.off_acc);
  void* dws = ws + L.off_acc + align_up(4 * sizeof(double));
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
        // the tape p^1..p^K of this iteration's TV step, then its reverse in one pass
        float* tape = V(L.off_tape_p, 0);
        TRY(launch_tv_tape(pl, p.lambda, p.rho, L.inner, p.tv_tau, fk, tape, L.vol_bytes / sizeof(float), s));
        const TvbGrid tg = tvb_grid(de.H, de.W, L.inner);
        TvbArgs ta;
        ta.f = fk;
        ta.ubar = ubar;
        ta.dbar = dbar;
        ta.tape = tape;
        ta.stride = L.vol_bytes / sizeof(float);
        ta.fbar = fbar;
        ta.part = part;
        ta.H = de.H;
        ta.W = de.W;
        ta.tilesX = tg.tilesX;
        ta.IX = tg.IX;
        ta.IY = tg.IY;
        ta.halo = tg.halo;
        ta.K = L.inner;
        ta.theta = thetaf;
        ta.inv_theta = inv_theta;
        ta.tau = tau;
        const int nblk = tg.tiles * de.N * de.R;
        hipLaunchKernelGGL((tvb_tile<kTvbCX, kTvbS, kTvbNW>), dim3(tg.tiles, de.N * de.R), dim3(64 * kTvbNW), 0, s, ta);
        hipLaunchKernelGGL(reduce_into, dim3(1), dim3(256), 0, s, part, nblk, acc, 3);
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
          // kGrid workgroups either way: reduce_into sums kGrid partials
          const size_t lds = (size_t)de.N * de.R * kMsLanes * (2 * sizeof(double) + sizeof(float));
          if (lds <= kMsMaxLds)
            hipLaunchKernelGGL((xupdate_bwd_ms<R, true>), G, dim3(kMsLanes), lds, s, de.N, p.rho, p.gamma,
                               periodic_solve, periodic_lap, pl.bits, de.H, de.W, pl.Wq, fbar,
                               k == K - 1 ? xbar : nullptr, V(L.off_seg_u, i), V(L.off_seg_d, i), fk, ybar, ubar,
                               dbar, part, part + kGrid, pl.ms_scratch);
          else
            hipLaunchKernelGGL((xupdate_bwd_ms<R, false>), G, B, 0, s, de.N, p.rho, p.gamma, periodic_solve,
                               periodic_lap, pl.bits, de.H, de.W, pl.Wq, fbar, k == K - 1 ? xbar : nullptr,
                               V(L.off_seg_u, i), V(L.off_seg_d, i), fk, ybar, ubar, dbar, part, part + kGrid,
                               pl.ms_scratch);
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
  char* wsc = static_cast<char*>(ws);
  if (params->flags & CSPNP_FLAG_NO_GRAPH) {
    CSPNP_HIP(enqueue_backward(*cplan, *params, y, ckpt_every, ckpt, x_bar, y_bar, param_bar, wsc, st));
    return CSPNP_OK;
  }
  // captured once per (parameters, pointers) into the plan's graph cache, like cspnp_solve
  cspnp_plan* plan = const_cast<cspnp_plan*>(cplan);
  std::vector<uint8_t> key;
  const char tag[4] = {'b', 'w', 'd', 0};
  key_append(key, tag);
  key_append(key, params->lambda); key_append(key, params->rho); key_append(key, params->gamma);
  key_append(key, params->iters); key_append(key, params->tv_inner); key_append(key, params->tv_tau);
  key_append(key, ckpt_every);
  key_append(key, y); key_append(key, ckpt); key_append(key, x_bar); key_append(key, y_bar);
  key_append(key, param_bar); key_append(key, ws);
  GraphEntry* ge = plan->graph.find(key);
  if (!ge) {
    CSPNP_HIP(hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_backward(*plan, *params, y, ckpt_every, ckpt, x_bar, y_bar, param_bar, wsc,
                                    plan->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(plan->capture_stream, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e, "backward launch during capture"); }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e3, "hipGraphInstantiate"); }
    ge = &plan->graph.slot();
    ge->graph = g;
    ge->exec = ex;
    ge->key = key;
    ge->last_use = ++plan->graph.clock;
  }
  CSPNP_HIP(hipGraphLaunch(ge->exec, st));
  return CSPNP_OK;
}
