// Per-pixel z-solve of the x-step (shared by the forward, batched and
// backward kernels): A = T + U U^T with T = rho I + gamma L_N LDL^T-factored
// on the host, U = [m] or [m, sqrt(gamma) w]; see xupdate.hip.
#pragma once

#include "common.hpp"

namespace cspnp {
namespace xuimpl {

template <int R>
__device__ __forceinline__ void tsolve(const ZSolve& z, double (&v)[R]) {
  // L z = v, then z *= D^{-1}, then L^T x = z
#pragma unroll
  for (int i = 1; i < R; ++i) v[i] = fma(-z.l[i], v[i - 1], v[i]);
  v[R - 1] *= z.invd[R - 1];
#pragma unroll
  for (int i = R - 2; i >= 0; --i) v[i] = fma(-z.l[i + 1], v[i + 1], v[i] * z.invd[i]);
}

// Solves the pixel system; on return a[] holds x.
template <int R>
__device__ __forceinline__ void pixel_solve(const ZSolve& z, uint32_t m, double (&a)[R]) {
  double b[R];
#pragma unroll
  for (int r = 0; r < R; ++r) b[r] = (double)((m >> r) & 1u);
  tsolve<R>(z, a);
  tsolve<R>(z, b);
  double mTa = 0.0, mTb = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if ((m >> r) & 1u) {
      mTa += a[r];
      mTb += b[r];
    }
  }
  if (z.periodic) {
    const double g = z.gamma;
    const double wTa = a[0] - a[R - 1];
    const double wTb = b[0] - b[R - 1];
    // [1 + mTb, wTb; g wTb, 1 + g wc] [alpha; beta'] = [mTa; g wTa], beta' = sqrt(g) beta
    const double c11 = 1.0 + mTb, c12 = wTb, c21 = g * wTb, c22 = 1.0 + g * z.wc;
    const double r1 = mTa, r2 = g * wTa;
    const double inv = 1.0 / (c11 * c22 - c12 * c21);
    const double alpha = (r1 * c22 - c12 * r2) * inv;
    const double beta = (c11 * r2 - c21 * r1) * inv;
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = a[r] - alpha * b[r] - beta * z.c[r];
  } else {
    const double alpha = mTa / (1.0 + mTb);
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = fma(-alpha, b[r], a[r]);
  }
}

// Every slice access is (wave-uniform slice base) + (32-bit lane byte offset):
// the slice base is formed by scalar arithmetic and the lane offset once, so a
// load or store costs no vector address arithmetic (plans keep H W <= 2^30, so
// every byte offset within a slice fits 32 bits).
// The base goes through readfirstlane so that it stays a scalar pair (left to
// itself the compiler re-associates base + r HW + offset into per-lane 64-bit
// multiply-adds).
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gchar* sbase(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gchar*)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t off) {
  typedef __attribute__((address_space(1))) const T gT;
  return *(gT*)(sbase(base) + off);
}
__device__ __forceinline__ void st_at(float* base, uint32_t off, float v) {
  typedef __attribute__((address_space(1))) float gT;
  *(gT*)(sbase(base) + off) = v;
}

template <int R, typename Word = const uint32_t>
__device__ __forceinline__ uint32_t load_bits(Word* __restrict__ bits, int H, int Wq, int h, int w) {
  uint32_t m = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
  return m;
}

}  // namespace xuimpl
}  // namespace cspnp
