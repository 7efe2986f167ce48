// Per-pixel solve of the x-step system for N > 1 shots per volume (shared by the
// forward x-step and its vector-Jacobian product; A is symmetric, so both solve
// with the same matrix).  Sec. III-A: N coded frames of R slices each; the
// temporal chain of Sec. III-C runs over all N*R slices and crosses shot
// boundaries.  Per pixel p:
//     A = T + sum_j m_j m_j^T  (+ gamma w w^T with the periodic wrap, w = e_1 - e_NR),
//     T = rho I + gamma L over the free-ends chain of N*R slices,
// m_j the pixel's R mask bits placed in block j (the same masks every shot).
// Block elimination: A without the wrap is block tridiagonal; block j is
// tridiagonal + rank one, and consecutive blocks couple only through the pair
// (last of j, first of j+1), so the Schur complement of blocks 1..j-1 changes
// only the first diagonal entry of block j.  Each block is applied with the
// Sherman-Morrison formula on its tridiagonal part (Thomas, FP64), the forward
// sweep stores y_j = S_j^{-1} b~_j and z_j = S_j^{-1} e_R, and the backward sweep
// is x_j = y_j + gamma x_{j+1,1} z_j.  The wrap is a final Sherman-Morrison step
// with a second right-hand side w.  Work O(N R) per pixel; the forward vectors
// live in an FP64 scratch of 3 N R doubles per pixel (the first two in LDS or an HBM
// volume, the wrap's in an HBM volume).
#pragma once

#include "common.hpp"

namespace cspnp {
namespace msimpl {

template <int R>
__device__ __forceinline__ void thomas(const double (&l)[R], const double (&invd)[R], double (&v)[R]) {
#pragma unroll
  for (int i = 1; i < R; ++i) v[i] = fma(-l[i], v[i - 1], v[i]);
  v[R - 1] *= invd[R - 1];
#pragma unroll
  for (int i = R - 2; i >= 0; --i) v[i] = fma(-l[i + 1], v[i + 1], v[i] * invd[i]);
}

// Right-hand side in two steps: fetch(j, raw) issues the loads of block j into the
// caller's Raw record, rhs(raw, r) -> double forms entry (j R + r) from it.  Block
// j + 1 is fetched before block j is eliminated, so its loads overlap that work.
// out(j, x_j) is called once per block j = 0..N-1 in order with the block's R entries.
// scratch: two [NR][stride] double arrays (y and z of the forward sweep); this
// pixel's column is q (an HBM volume with stride H W and q the pixel, or an LDS
// block with stride = threads and q the lane).  yw: the periodic wrap's third
// array, [NR][yw_stride] at column yw_q (an HBM volume in every caller).
template <int R, typename Raw, typename Fetch, typename Rhs, typename Out>
__device__ __forceinline__ void solve(uint32_t m, int N, double rho, double gamma, int periodic, size_t stride, size_t q,
                                      double* __restrict__ scratch, double* __restrict__ yw, size_t yw_stride,
                                      size_t yw_q, Fetch&& fetch, Rhs&& rhs, Out&& out) {
  const int NR = N * R;
  const size_t HW = stride, p = q;
  double* Yb = scratch;                    // [NR][stride]
  double* Zs = scratch + (size_t)NR * HW;  // [NR][stride]
  auto Yw = [&](int gi) -> double& { return yw[(size_t)gi * yw_stride + yw_q]; };
  double sigma = 0.0, carry_b = 0.0, carry_w = 0.0;
  Raw raw_next;
  fetch(0, raw_next);
  for (int j = 0; j < N; ++j) {
    const Raw raw = raw_next;
    if (j + 1 < N) fetch(j + 1, raw_next);
    double bb[R], bw[R], l[R], invd[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bb[r] = rhs(raw, r);
      bw[r] = 0.0;
    }
    bb[0] += carry_b;
    if (periodic) {
      if (j == 0) bw[0] += 1.0;
      if (j == N - 1) bw[R - 1] -= 1.0;
      bw[0] += carry_w;
    }
    // LDL^T of this block's tridiagonal part (first diagonal entry reduced by the Schur term)
    double dprev = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gi = j * R + r;
      const int deg = NR == 1 ? 0 : ((gi == 0 || gi == NR - 1) ? 1 : 2);
      double t = rho + gamma * deg;
      if (r == 0) t -= sigma;
      if (r == 0) {
        l[0] = 0.0;
        dprev = t;
      } else {
        l[r] = -gamma / dprev;
        dprev = t - l[r] * (-gamma);
      }
      invd[r] = 1.0 / dprev;
    }
    double pm[R], er[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      pm[r] = (double)((m >> r) & 1u);
      er[r] = r == R - 1 ? 1.0 : 0.0;
    }
    thomas<R>(l, invd, pm);
    thomas<R>(l, invd, bb);
    thomas<R>(l, invd, er);
    if (periodic) thomas<R>(l, invd, bw);
    double mp = 0.0, mb = 0.0, me = 0.0, mw = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((m >> r) & 1u) {
        mp += pm[r];
        mb += bb[r];
        me += er[r];
        mw += bw[r];
      }
    const double inv = 1.0 / (1.0 + mp);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bb[r] -= pm[r] * (mb * inv);
      er[r] -= pm[r] * (me * inv);
      if (periodic) bw[r] -= pm[r] * (mw * inv);
      const size_t g = (size_t)(j * R + r) * HW + p;
      Yb[g] = bb[r];
      Zs[g] = er[r];
      if (periodic) Yw(j * R + r) = bw[r];
    }
    sigma = gamma * gamma * er[R - 1];
    carry_b = gamma * bb[R - 1];
    carry_w = gamma * bw[R - 1];
  }
  // backward sweep, x_j = y_j + gamma x_{j+1,1} z_j (overwriting y in the scratch).  The
  // wrap's vector lives in global memory: block j - 1's entries are loaded while block
  // j is worked on, and the output pass below prefetches the same way.
  double nb = 0.0, nw = 0.0;
  double xb_first = 0.0, xb_last = 0.0, xw_first = 0.0, xw_last = 0.0;
  double ywn[R];
  if (periodic) {
#pragma unroll
    for (int r = 0; r < R; ++r) ywn[r] = Yw((N - 1) * R + r);
  }
  for (int j = N - 1; j >= 0; --j) {
    double ywc[R];
    if (periodic) {
#pragma unroll
      for (int r = 0; r < R; ++r) ywc[r] = ywn[r];
      if (j > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) ywn[r] = Yw((j - 1) * R + r);
      }
    }
    double nb_next = 0.0, nw_next = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t g = (size_t)(j * R + r) * HW + p;
      const double z = Zs[g];
      const double xb = Yb[g] + gamma * nb * z;
      Yb[g] = xb;
      if (r == 0) nb_next = xb;
      if (j == N - 1 && r == R - 1) xb_last = xb;
      if (j == 0 && r == 0) xb_first = xb;
      if (periodic) {
        const double xw = ywc[r] + gamma * nw * z;
        Yw(j * R + r) = xw;
        if (r == 0) nw_next = xw;
        if (j == N - 1 && r == R - 1) xw_last = xw;
        if (j == 0 && r == 0) xw_first = xw;
      }
    }
    nb = nb_next;
    nw = nw_next;
  }
  double coef = 0.0;
  if (periodic) coef = gamma * (xb_first - xb_last) / (1.0 + gamma * (xw_first - xw_last));
  // the solution block by block: out(j, x_j) sees all R entries of block j at once, so
  // its own loads for the block can be issued together
  if (periodic) {
#pragma unroll
    for (int r = 0; r < R; ++r) ywn[r] = Yw(r);
  }
  for (int j = 0; j < N; ++j) {
    double ywc[R];
    if (periodic) {
#pragma unroll
      for (int r = 0; r < R; ++r) ywc[r] = ywn[r];
      if (j + 1 < N) {
#pragma unroll
        for (int r = 0; r < R; ++r) ywn[r] = Yw((j + 1) * R + r);
      }
    }
    double xv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t o = (size_t)(j * R + r) * HW + p;
      xv[r] = Yb[o];
      if (periodic) xv[r] -= coef * ywc[r];
    }
    out(j, xv);
  }
}

}  // namespace msimpl
}  // namespace cspnp
