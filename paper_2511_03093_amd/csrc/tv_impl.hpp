// Chambolle dual-projection tile (shared by the single-problem and the
// batched TV kernels).  See tv.hip for the algorithm and the tiling.
#pragma once

#include "common.hpp"

namespace cspnp {
namespace tvimpl {

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

// LDS exchange between vertically adjacent waves, double-buffered by inner-iteration parity:
// [parity][wave][0] = the wave's bottom-row p_y, [parity][wave][1] = its top-row partial
// divergence (px - px_left) + py.  Every w is evaluated as (((px - px_left) + py) - py_up) - f/theta,
// so the wave above rebuilds the w of the row below its strip bit for bit.
template <int CX, int NW>
using TvExchange = float[2][NW][2][64 * CX];

template <int CX, int S, int NW, bool BORDER>
__device__ __forceinline__ void tv_tile_impl(const TvLaunch& a, const int k, const int L, const int ox, const int oy,
                                             const size_t base, TvExchange<CX, NW>& xch) {
  // No implicit contraction: a p value must round identically whether its
  // neighbour reads it from a register or through the LDS exchange (the
  // intended fused multiply-adds are written as fmaf).
#pragma clang fp contract(off)
  const int c0 = ox + L * CX;
  const int r0 = oy + k * S;
  const float* __restrict__ fn = a.f + base;

  float px[S][CX], py[S][CX], fs[S][CX], fsb[CX];
  float colx[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) {
    const int gc = c0 + c;
    colx[c] = (gc >= 0 && gc < a.W - 1) ? 1.f : 0.f;
  }
#pragma unroll
  for (int s = 0; s <= S; ++s) {
    const int gr = r0 + s;
    const bool rin = gr >= 0 && gr < a.H;
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      const int gc = c0 + c;
      const bool in = rin && gc >= 0 && gc < a.W;
      const size_t off = (size_t)gr * a.W + gc;
      const float v = in ? __fmul_rn(fn[off], a.inv_theta) : 0.f;
      if (s == S) {
        fsb[c] = v;  // the first row of the wave below (its w is rebuilt here)
        continue;
      }
      fs[s][c] = v;
      if (a.p_in) {
        px[s][c] = in ? a.p_in[base + off] : 0.f;
        py[s][c] = in ? a.p_in[a.vol + base + off] : 0.f;
      } else {
        px[s][c] = 0.f;
        py[s][c] = 0.f;
      }
    }
  }
  // publish the initial exchange values
  {
    const float left = from_left(px[0][CX - 1]);
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      xch[0][k][0][L * CX + c] = py[S - 1][c];
      xch[0][k][1][L * CX + c] = (px[0][c] - ((c > 0) ? px[0][c - 1] : left)) + py[0][c];
    }
  }
  __syncthreads();

  const float tau = a.tau;
  for (int it = 0; it < a.iters; ++it) {
    const int b = it & 1;
    float pyab[CX], wbl[CX], wcur[CX];
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      pyab[c] = (k > 0) ? xch[b][k - 1][0][L * CX + c] : 0.f;
      wbl[c] = (k < NW - 1) ? ((xch[b][k + 1][1][L * CX + c] - py[S - 1][c]) - fsb[c]) : 0.f;
    }
    {
      const float left = from_left(px[0][CX - 1]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float pxl = (c > 0) ? px[0][c - 1] : left;
        wcur[c] = (((px[0][c] - pxl) + py[0][c]) - pyab[c]) - fs[0][c];
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float wnext[CX];
      if (s < S - 1) {
        const float left = from_left(px[s + 1][CX - 1]);
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          const float pxl = (c > 0) ? px[s + 1][c - 1] : left;
          wnext[c] = (((px[s + 1][c] - pxl) + py[s + 1][c]) - py[s][c]) - fs[s + 1][c];
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
        const float gx = BORDER ? (wr - wcur[c]) * colx[c] : (wr - wcur[c]);
        const float gy = BORDER ? (ry ? (wnext[c] - wcur[c]) : 0.f) : (wnext[c] - wcur[c]);
        const float q = fmaf(gx, gx, gy * gy);
        const float rs = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(q), 1.f));
        px[s][c] = fmaf(tau, gx, px[s][c]) * rs;
        py[s][c] = fmaf(tau, gy, py[s][c]) * rs;
      }
#pragma unroll
      for (int c = 0; c < CX; ++c) wcur[c] = wnext[c];
    }
    {
      const int nb = b ^ 1;
      const float left = from_left(px[0][CX - 1]);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        xch[nb][k][0][L * CX + c] = py[S - 1][c];
        xch[nb][k][1][L * CX + c] = (px[0][c] - ((c > 0) ? px[0][c - 1] : left)) + py[0][c];
      }
    }
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
  const int bf = a.iters & 1;
  float pyab[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) pyab[c] = (k > 0) ? xch[bf][k - 1][0][L * CX + c] : 0.f;
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

// One tile of one slice.  Tiles that lie strictly inside [0, W-1) x [0, H-1) need no
// boundary masks and take the unmasked code path.
template <int CX, int S, int NW>
__device__ __forceinline__ void tv_tile(const TvLaunch& a, const int tile, const int slice,
                                        TvExchange<CX, NW>& xch) {
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  const int tx = tile % a.tilesX, ty = tile / a.tilesX;
  const size_t base = (size_t)slice * a.H * a.W;
  const int ox = tx * a.IX - a.halo, oy = ty * a.IY - a.halo;
  const bool interior = ox >= 0 && oy >= 0 && ox + 64 * CX <= a.W - 1 && oy + NW * S <= a.H - 1;
  if (interior)
    tv_tile_impl<CX, S, NW, false>(a, k, L, ox, oy, base, xch);
  else
    tv_tile_impl<CX, S, NW, true>(a, k, L, ox, oy, base, xch);
}

}  // namespace tvimpl
}  // namespace cspnp
