// TV u-step: Chambolle's dual projection (the TV solver the paper cites for
// the denoising step, Sec. III-B) for every slice of f, with the d-step
// fused into the epilogue:
//     theta = lambda / rho, p = 0,
//     repeat: w = div p - f/theta, g = grad w,
//             p = (p + tau g) / (1 + tau |g|),
//     u = f - theta div p,  d = f - u.
// grad: forward differences, zero on the last column/row; div = -grad^T.
//
// Tiling.  A workgroup of NW waves owns a (64*CX) x (NW*S) pixel tile of one
// slice: lane L of wave k holds rows k*S..k*S+S-1 and columns L*CX..L*CX+CX-1
// of p and f/theta in registers for all inner iterations.  Horizontal
// neighbours come from the adjacent lane by DPP wave shifts, vertical
// neighbours across waves through LDS (two barriers per inner iteration).
// Values beyond the tile edge are not available, and the error they cause
// spreads one pixel per iteration, so the tile carries a halo of `iters`
// pixels (one more when p is loaded) and writes only its interior.  Pixels
// outside the image keep p = 0, which realises the boundary cases of div.
// When tv_inner is too large for one tile, passes of at most kMaxFused
// iterations exchange p through an HBM workspace.
#include "common.hpp"

namespace cspnp {

namespace {

constexpr int kMaxFused = 16;

struct TvLaunch {
  const float* f;
  float* u;
  float* d_out;
  const float* p_in;  // px at p_in, py at p_in + NR*H*W (NULL: start from p = 0)
  float* p_out;       // intermediate pass output (NULL on the final pass)
  int H, W;
  int tilesX;
  int IX, IY;  // interior size
  int halo;
  int iters;
  float theta, inv_theta, tau;
  size_t vol;  // NR*H*W
};

// lane i <- lane i-1 (0 for lane 0)
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
// lane i <- lane i+1 (0 for lane 63)
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

template <int CX, int S, int NW>
__global__ __launch_bounds__(64 * NW) void tv_kernel(const TvLaunch a) {
  __shared__ float lds_py[NW][64 * CX];
  __shared__ float lds_w[NW][64 * CX];
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  const int tile = blockIdx.x;
  const int tx = tile % a.tilesX, ty = tile / a.tilesX;
  const size_t HW = (size_t)a.H * a.W;
  const size_t base = (size_t)blockIdx.y * HW;
  const int ox = tx * a.IX - a.halo, oy = ty * a.IY - a.halo;
  const int c0 = ox + L * CX;
  const int r0 = oy + k * S;
  const float* __restrict__ fn = a.f + base;

  float px[S][CX], py[S][CX], fs[S][CX];
  float colx[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) {
    const int gc = c0 + c;
    colx[c] = (gc >= 0 && gc < a.W - 1) ? 1.f : 0.f;
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int gr = r0 + s;
    const bool rin = gr >= 0 && gr < a.H;
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      const int gc = c0 + c;
      const bool in = rin && gc >= 0 && gc < a.W;
      const size_t off = (size_t)gr * a.W + gc;
      fs[s][c] = in ? __fmul_rn(fn[off], a.inv_theta) : 0.f;
      if (a.p_in) {
        px[s][c] = in ? a.p_in[base + off] : 0.f;
        py[s][c] = in ? a.p_in[a.vol + base + off] : 0.f;
      } else {
        px[s][c] = 0.f;
        py[s][c] = 0.f;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CX; ++c) lds_py[k][L * CX + c] = py[S - 1][c];
  __syncthreads();

  const float tau = a.tau;
  for (int it = 0; it < a.iters; ++it) {
    float pyab[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) pyab[c] = (k > 0) ? lds_py[k - 1][L * CX + c] : 0.f;
    float wcur[CX];
    {
      const float left = from_left(px[0][CX - 1]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float pxl = (c > 0) ? px[0][c - 1] : left;
        wcur[c] = (px[0][c] - pxl) + (py[0][c] - pyab[c]) - fs[0][c];
      }
    }
#pragma unroll
    for (int c = 0; c < CX; ++c) lds_w[k][L * CX + c] = wcur[c];
    __syncthreads();
    float wbl[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) wbl[c] = (k < NW - 1) ? lds_w[k + 1][L * CX + c] : 0.f;

#pragma unroll
    for (int s = 0; s < S; ++s) {
      float wnext[CX];
      if (s < S - 1) {
        const float left = from_left(px[s + 1][CX - 1]);
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          const float pxl = (c > 0) ? px[s + 1][c - 1] : left;
          wnext[c] = (px[s + 1][c] - pxl) + (py[s + 1][c] - py[s][c]) - fs[s + 1][c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < CX; ++c) wnext[c] = wbl[c];
      }
      const float right = from_right(wcur[0]);
      const int gr = r0 + s;
      const bool ry = gr >= 0 && gr < a.H - 1;  // wave-uniform
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float wr = (c < CX - 1) ? wcur[c + 1] : right;
        const float gx = (wr - wcur[c]) * colx[c];
        const float gy = ry ? (wnext[c] - wcur[c]) : 0.f;
        const float q = fmaf(gx, gx, gy * gy);
        const float rs = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(q), 1.f));
        px[s][c] = fmaf(tau, gx, px[s][c]) * rs;
        py[s][c] = fmaf(tau, gy, py[s][c]) * rs;
      }
#pragma unroll
      for (int c = 0; c < CX; ++c) wcur[c] = wnext[c];
    }
#pragma unroll
    for (int c = 0; c < CX; ++c) lds_py[k][L * CX + c] = py[S - 1][c];
    __syncthreads();
  }

  // epilogue: interior pixels only
  const int tc0 = L * CX;
  if (a.p_out) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int tr = k * S + s, gr = r0 + s;
      if (tr < a.halo || tr >= a.halo + a.IY || gr >= a.H) continue;
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const int tcc = tc0 + c, gc = c0 + c;
        if (tcc < a.halo || tcc >= a.halo + a.IX || gc >= a.W) continue;
        const size_t off = base + (size_t)gr * a.W + gc;
        a.p_out[off] = px[s][c];
        a.p_out[a.vol + off] = py[s][c];
      }
    }
    return;
  }
  float pyab[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) pyab[c] = (k > 0) ? lds_py[k - 1][L * CX + c] : 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float left = from_left(px[s][CX - 1]);
    const int tr = k * S + s, gr = r0 + s;
    const bool rowok = tr >= a.halo && tr < a.halo + a.IY && gr < a.H;
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      const float pxl = (c > 0) ? px[s][c - 1] : left;
      const float pyu = (s > 0) ? py[s - 1][c] : pyab[c];
      const float dv = (px[s][c] - pxl) + (py[s][c] - pyu);
      const int tcc = tc0 + c, gc = c0 + c;
      if (rowok && tcc >= a.halo && tcc < a.halo + a.IX && gc < a.W) {
        const size_t off = (size_t)gr * a.W + gc;
        const float fv = fn[off];
        const float uv = fv - a.theta * dv;
        a.u[base + off] = uv;
        if (a.d_out) a.d_out[base + off] = fv - uv;
      }
    }
  }
}

template <int CX, int S, int NW>
hipError_t launch_shape(const TvLaunch& base_args, int NR, hipStream_t st) {
  TvLaunch a = base_args;
  const int TW = 64 * CX, TH = NW * S;
  a.IX = TW - 2 * a.halo;
  a.IY = TH - 2 * a.halo;
  if (a.IX < 1 || a.IY < 1) return hipErrorInvalidValue;
  a.tilesX = (a.W + a.IX - 1) / a.IX;
  const int tilesY = (a.H + a.IY - 1) / a.IY;
  dim3 grid(a.tilesX * tilesY, NR);
  hipLaunchKernelGGL((tv_kernel<CX, S, NW>), grid, dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

// Tile shapes: lane columns CX, rows per lane S, waves NW -> (64 CX) x (NW S) pixels.
struct ShapeEntry {
  TvShapeInfo info;
  hipError_t (*launch)(const TvLaunch&, int, hipStream_t);
};
#define CSPNP_TV_SHAPE(CX, S, NW) {{CX, S, NW, 64 * CX, NW * S}, &launch_shape<CX, S, NW>}
const ShapeEntry kShapes[] = {
    CSPNP_TV_SHAPE(2, 16, 8),  CSPNP_TV_SHAPE(2, 16, 12), CSPNP_TV_SHAPE(2, 8, 16),
    CSPNP_TV_SHAPE(2, 12, 16), CSPNP_TV_SHAPE(3, 8, 16),  CSPNP_TV_SHAPE(3, 12, 8), 
    CSPNP_TV_SHAPE(3, 16, 8),  CSPNP_TV_SHAPE(1, 16, 8),  CSPNP_TV_SHAPE(2, 8, 8),
    CSPNP_TV_SHAPE(1, 8, 8),
};
#undef CSPNP_TV_SHAPE
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int passes_for(int tv_inner) { return tv_inner <= kMaxFused ? 1 : (tv_inner + kMaxFused - 1) / kMaxFused; }

}  // namespace

size_t tv_workspace_bytes(const cspnp_plan& pl, int tv_inner) {
  if (passes_for(tv_inner) <= 1) return 0;
  const size_t vol = (size_t)pl.desc.N * pl.desc.R * pl.desc.H * pl.desc.W;
  return 4 * vol * sizeof(float);  // two (px, py) buffers, ping-pong
}

int tv_num_shapes() { return kNumShapes; }

TvShapeInfo tv_shape_info(int i) { return kShapes[i].info; }

int tv_default_shape(int H, int W, int NR, int tv_inner) {
  // fewest tile-pixels per launch, then the larger block (better latency hiding)
  const int halo = tv_inner <= kMaxFused ? tv_inner : kMaxFused + 1;
  long best = -1;
  int bi = 0;
  for (int i = 0; i < kNumShapes; ++i) {
    const auto& s = kShapes[i].info;
    const int ix = s.cols - 2 * halo, iy = s.rows - 2 * halo;
    if (ix < 8 || iy < 8) continue;
    const long tiles = (long)((W + ix - 1) / ix) * ((H + iy - 1) / iy) * NR;
    const long work = tiles * s.cols * s.rows;
    if (best < 0 || work < best) { best = work; bi = i; }
  }
  return bi;
}

hipError_t launch_tv(const cspnp_plan& pl, double lambda, double rho, int tv_inner, double tau,
                     const float* f, float* u, float* d_out, void* ws, hipStream_t st) {
  return launch_tv_shape(pl, pl.tv_shape, lambda, rho, tv_inner, tau, f, u, d_out, ws, st);
}

hipError_t launch_tv_shape(const cspnp_plan& pl, int shape, double lambda, double rho, int tv_inner,
                           double tau, const float* f, float* u, float* d_out, void* ws, hipStream_t st) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  TvLaunch a{};
  a.f = f;
  a.u = u;
  a.d_out = d_out;
  a.H = de.H;
  a.W = de.W;
  a.vol = (size_t)NR * de.H * de.W;
  const double theta = lambda / rho;
  a.theta = (float)theta;
  a.inv_theta = theta > 0 ? (float)(1.0 / theta) : 0.f;
  a.tau = (float)tau;
  if (shape < 0 || shape >= kNumShapes) return hipErrorInvalidValue;
  const ShapeEntry& sh = kShapes[shape];
  if (theta == 0.0) tv_inner = 0;  // prox of a zero weight is the identity
  const int passes = passes_for(tv_inner);
  float* bufs[2] = {static_cast<float*>(ws), static_cast<float*>(ws) + 2 * a.vol};
  int done = 0;
  for (int ps = 0; ps < passes; ++ps) {
    const int k = (tv_inner - done) / (passes - ps);
    const bool last = ps == passes - 1;
    a.iters = k;
    a.p_in = ps == 0 ? nullptr : bufs[(ps - 1) & 1];
    a.p_out = last ? nullptr : bufs[ps & 1];
    a.halo = k + ((last && a.p_in) ? 1 : 0);
    hipError_t e = sh.launch(a, NR, st);
    if (e != hipSuccess) return e;
    done += k;
  }
  return hipSuccess;
}

}  // namespace cspnp
