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
  // Tape (the backward's record of the inner iterates): when the tape variant of
  // the tile is instantiated, p^t after inner iteration t = 1..iters is stored at
  // tape + 2 t tape_stride (px) and tape + (2 t + 1) tape_stride (py), interior
  // pixels of every tile (so the whole slice), and no u is written.
  float* tape;
  size_t tape_stride;
};

// lane i <- lane i-1 (0 for lane 0)
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
// lane i <- lane i+1 (0 for lane 63)
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
// lane i <- lane i+1; lane 63 keeps `own` (no source lane: the DPP write is disabled)
__device__ __forceinline__ float from_right_or(float own, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(own), __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// Buffer resources over one H x W slice.  Every offset the tile uses is clamped
// into the slice, so the hardware range check is never what keeps an access in
// bounds; the resource form lets a load take the wave-uniform row offset in an
// SGPR and the lane's column offset in a 32-bit VGPR (no 64-bit address math).
// Plans keep H*W <= 2^30, so every offset fits the 32-bit byte range.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc slice_rsrc(const float* p, int H, int W) {
  const uint64_t bytes = (uint64_t)H * (uint64_t)W * 4u;
  const uint32_t n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)n, 0x00020000);
}
__device__ __forceinline__ float ld(Rsrc r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void st(float v, Rsrc r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
}

// LDS exchange between vertically adjacent waves, double-buffered by inner-iteration parity:
// [parity][wave][0] = the wave's bottom-row p_y, [parity][wave][1] = its top-row partial
// divergence (px - px_left) + py.  Every w is evaluated as (((px - px_left) + py) - py_up) - f/theta,
// so the wave above rebuilds the w of the row below its strip bit for bit.
template <int CX, int NW>
using TvExchange = float[2][NW][2][64 * CX];
// The f values of every lane's S x CX pixels, kept for the epilogue (u = f - theta div p
// needs f itself, and only f/theta stays in registers).  Lane-private: element (s, c) of
// lane L in wave k sits at [k][s * CX + c][L], so a wave's accesses are conflict-free.
template <int CX, int S, int NW>
using TvStage = float[NW][S * CX][64];

// BX: the tile is wider than the image, so columns outside it need the x-gradient
// mask.  Otherwise every tile lies inside [0, W) (edge tiles are moved inward) and
// the only column without an x-gradient inside the tile is W-1, the last column
// of lane 63 in the right edge tile: there the right neighbour taken is the pixel
// itself, so g_x = w - w = 0 exactly, with no mask.  Rows without a y-gradient (the
// last image row, and rows outside the image) are wave-uniform and take a branch
// of their own.  Interior (written) columns are [ix0, ix1).
// COLD: the launch starts from p = 0 (no p_in).  Every value the first inner
// iteration exchanges is then +0, so it is published, and the barrier passed,
// while the tile's loads are still in flight: each wave starts computing as soon
// as its own rows have arrived.
template <int CX, int S, int NW, bool BX, bool TAPE = false, bool COLD = false>
__device__ __forceinline__ void tv_tile_impl(const TvLaunch& a, const int k, const int L, const int ox, const int oy,
                                             const int ix0, const int ix1,
                                             const size_t base, TvExchange<CX, NW>& xch, TvStage<CX, S, NW>& fst) {
  // No implicit contraction: a p value must round identically whether its
  // neighbour reads it from a register or through the LDS exchange (the
  // intended fused multiply-adds are written as fmaf).
#pragma clang fp contract(off)
  const int c0 = ox + L * CX;
  const int r0 = oy + k * S;  // wave-uniform

  // lane column byte offsets (clamped into the slice) and column masks
  uint32_t coff[CX];
  float colx[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) {
    const int gc = c0 + c;
    coff[c] = 4u * (uint32_t)min(max(gc, 0), a.W - 1);
    colx[c] = (gc >= 0 && gc < a.W - 1) ? 1.f : 0.f;
  }
  auto col_in = [&](int c) { return c0 + c >= 0 && c0 + c < a.W; };
  auto row_off = [&](int s) -> uint32_t { return 4u * (uint32_t)min(max(r0 + s, 0), a.H - 1) * (uint32_t)a.W; };
  // bit s set: row r0 + s lies in the image (s = 0..S) / has a y-gradient (r0 + s < H - 1)
  uint32_t rows_in = 0, rows_gy = 0;
#pragma unroll
  for (int s = 0; s <= S; ++s) {
    const int gr = r0 + s;
    rows_in |= (gr >= 0 && gr < a.H) ? (1u << s) : 0u;
    rows_gy |= (gr >= 0 && gr < a.H - 1) ? (1u << s) : 0u;
  }
  rows_in = __builtin_amdgcn_readfirstlane(rows_in);
  rows_gy = __builtin_amdgcn_readfirstlane(rows_gy);

  const Rsrc fr = slice_rsrc(a.f + base, a.H, a.W);
  float px[S][CX], py[S][CX], fs[S][CX], fsb[CX];
  {
    // every load in flight at once, masked afterwards
    float raw[S + 1][CX];
#pragma unroll
    for (int s = 0; s <= S; ++s) {
      const uint32_t ro = row_off(s);
#pragma unroll
      for (int c = 0; c < CX; ++c) raw[s][c] = ld(fr, coff[c], ro);
    }
    if constexpr (COLD) {
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        xch[0][k][0][L * CX + c] = 0.f;
        xch[0][k][1][L * CX + c] = 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int c = 0; c < CX; ++c) px[s][c] = py[s][c] = 0.f;
    } else if (a.p_in) {
      const Rsrc xr = slice_rsrc(a.p_in + base, a.H, a.W);
      const Rsrc yr = slice_rsrc(a.p_in + a.vol + base, a.H, a.W);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const uint32_t ro = row_off(s);
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          px[s][c] = ld(xr, coff[c], ro);
          py[s][c] = ld(yr, coff[c], ro);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int c = 0; c < CX; ++c) px[s][c] = py[s][c] = 0.f;
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int c = 0; c < CX; ++c) fst[k][s * CX + c][L] = raw[s][c];
#pragma unroll
    for (int s = 0; s <= S; ++s) {
      const bool rin = (rows_in >> s) & 1u;
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const bool in = rin && (!BX || col_in(c));
        const float v = in ? __fmul_rn(raw[s][c], a.inv_theta) : 0.f;
        if (s == S) {
          fsb[c] = v;  // the first row of the wave below (its w is rebuilt here)
          continue;
        }
        fs[s][c] = v;
        if constexpr (!COLD) {
          px[s][c] = in ? px[s][c] : 0.f;
          py[s][c] = in ? py[s][c] : 0.f;
        }
      }
    }
  }
  if constexpr (!COLD) {
    // publish the initial exchange values
    const float left = from_left(px[0][CX - 1]);
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      xch[0][k][0][L * CX + c] = py[S - 1][c];
      xch[0][k][1][L * CX + c] = (px[0][c] - ((c > 0) ? px[0][c - 1] : left)) + py[0][c];
    }
    __syncthreads();
  }

  // interior pixels (the ones this tile writes): bit s of interior_rows() is set when
  // row r0 + s is an interior row of the tile inside the image
  auto interior_rows = [&]() {
    uint32_t m = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int tr = k * S + s, gr = r0 + s;
      m |= (tr >= a.halo && tr < a.halo + a.IY && gr < a.H) ? (1u << s) : 0u;
    }
    return __builtin_amdgcn_readfirstlane(m);
  };
  auto col_out = [&](int c) {
    const int gc = c0 + c;
    return gc >= ix0 && gc < ix1;
  };

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
      // x-gradients first, for both branches: the last one takes its right
      // neighbour through a DPP operand of the subtraction itself
      float gxs[CX];
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const float d = ((c < CX - 1) ? wcur[c + 1] : (BX ? from_right(wcur[0]) : from_right_or(wcur[c], wcur[0]))) -
                        wcur[c];
        gxs[c] = BX ? d * colx[c] : d;
      }
      if ((rows_gy >> s) & 1u) {
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          const float gx = gxs[c];
          const float gy = wnext[c] - wcur[c];
          const float q = fmaf(gx, gx, gy * gy);
          const float rs = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(q), 1.f));
          px[s][c] = fmaf(tau, gx, px[s][c]) * rs;
          py[s][c] = fmaf(tau, gy, py[s][c]) * rs;
        }
      } else {
        // no y-gradient on this row (g_y = 0): the same values with the zero terms dropped
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          const float gx = gxs[c];
          const float rs = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(gx * gx), 1.f));
          px[s][c] = fmaf(tau, gx, px[s][c]) * rs;
          py[s][c] = py[s][c] * rs;
        }
      }
#pragma unroll
      for (int c = 0; c < CX; ++c) wcur[c] = wnext[c];
    }
    if constexpr (TAPE) {
      const uint32_t rows_out = interior_rows();
      const Rsrc tx = slice_rsrc(a.tape + (size_t)(2 * (it + 1)) * a.tape_stride + base, a.H, a.W);
      const Rsrc ty = slice_rsrc(a.tape + (size_t)(2 * (it + 1) + 1) * a.tape_stride + base, a.H, a.W);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (!((rows_out >> s) & 1u)) continue;
        const uint32_t ro = row_off(s);
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          if (!col_out(c)) continue;
          st(px[s][c], tx, coff[c], ro);
          st(py[s][c], ty, coff[c], ro);
        }
      }
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
  if constexpr (TAPE) return;

  // epilogue: interior pixels only
  const uint32_t rows_out = interior_rows();
  if (a.p_out) {
    const Rsrc xw = slice_rsrc(a.p_out + base, a.H, a.W);
    const Rsrc yw = slice_rsrc(a.p_out + a.vol + base, a.H, a.W);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (!((rows_out >> s) & 1u)) continue;
      const uint32_t ro = row_off(s);
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        if (!col_out(c)) continue;
        st(px[s][c], xw, coff[c], ro);
        st(py[s][c], yw, coff[c], ro);
      }
    }
    return;
  }
  const int bf = a.iters & 1;
  float pyab[CX];
#pragma unroll
  for (int c = 0; c < CX; ++c) pyab[c] = (k > 0) ? xch[bf][k - 1][0][L * CX + c] : 0.f;
  float fv[S][CX];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < CX; ++c) fv[s][c] = fst[k][s * CX + c][L];
  const Rsrc uw = slice_rsrc(a.u + base, a.H, a.W);
  const Rsrc dw = slice_rsrc(a.d_out ? a.d_out + base : a.u + base, a.H, a.W);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float left = from_left(px[s][CX - 1]);
    if (!((rows_out >> s) & 1u)) continue;
    const uint32_t ro = row_off(s);
#pragma unroll
    for (int c = 0; c < CX; ++c) {
      const float pxl = (c > 0) ? px[s][c - 1] : left;
      const float pyu = (s > 0) ? py[s - 1][c] : pyab[c];
      const float dv = (px[s][c] - pxl) + (py[s][c] - pyu);
      if (col_out(c)) {
        const float uv = fv[s][c] - a.theta * dv;
        st(uv, uw, coff[c], ro);
        if (a.d_out) st(fv[s][c] - uv, dw, coff[c], ro);
      }
    }
  }
}

// One tile of one slice.  When the image is at least a tile wide every tile lies
// inside it and takes the unmasked code path; otherwise the masked one.
template <int CX, int S, int NW, bool TAPE = false, bool COLD = false>
__device__ __forceinline__ void tv_tile(const TvLaunch& a, const int tile, const int slice,
                                        TvExchange<CX, NW>& xch, TvStage<CX, S, NW>& fst) {
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  const int tx = tile % a.tilesX, ty = tile / a.tilesX;
  const size_t base = (size_t)slice * a.H * a.W;
  const int ix0 = tx * a.IX, ix1 = min(ix0 + a.IX, a.W);
  const int oy = ty * a.IY - a.halo;
  if (a.W >= 64 * CX) {
    // edge tiles moved inward to the image edge: the interior keeps a halo of
    // `halo` columns on every side that is not the image boundary
    const int ox = min(max(ix0 - a.halo, 0), a.W - 64 * CX);
    tv_tile_impl<CX, S, NW, false, TAPE, COLD>(a, k, L, ox, oy, ix0, ix1, base, xch, fst);
  } else {
    tv_tile_impl<CX, S, NW, true, TAPE, COLD>(a, k, L, ix0 - a.halo, oy, ix0, ix1, base, xch, fst);
  }
}

}  // namespace tvimpl
}  // namespace cspnp
