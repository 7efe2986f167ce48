// x-step for N > 1 shots per volume (Sec. III-A: N coded frames of R slices
// each; the temporal chain of Sec. III-C runs over all N*R slices and crosses
// shot boundaries).  Per pixel p:
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
// with a second right-hand side w.  Work O(N R) per pixel; the forward
// vectors live in an FP64 scratch volume owned by the plan.
#include "common.hpp"

namespace cspnp {

namespace {

template <int R>
__device__ __forceinline__ void thomas(const double (&l)[R], const double (&invd)[R], double (&v)[R]) {
#pragma unroll
  for (int i = 1; i < R; ++i) v[i] = fma(-l[i], v[i - 1], v[i]);
  v[R - 1] *= invd[R - 1];
#pragma unroll
  for (int i = R - 2; i >= 0; --i) v[i] = fma(-l[i + 1], v[i + 1], v[i] * invd[i]);
}

template <int R>
__global__ __launch_bounds__(256) void xupdate_multishot(const uint32_t* __restrict__ bits, int H, int W, int Wq,
                                                         int N, double rho, double gamma, int periodic,
                                                         const float* __restrict__ y, const float* __restrict__ u,
                                                         const float* d, int d_from_f, float* __restrict__ x_out,
                                                         float* f_out, double* __restrict__ scratch) {
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int h = (int)(p / W), w = (int)(p % W);
  const int NR = N * R;
  uint32_t m = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
  double* Yb = scratch;                    // [NR][HW]
  double* Zs = scratch + (size_t)NR * HW;  // [NR][HW]
  double* Yw = scratch + 2 * (size_t)NR * HW;
  double sigma = 0.0, carry_b = 0.0, carry_w = 0.0;
  for (int j = 0; j < N; ++j) {
    double bb[R], bw[R], l[R], invd[R];
    const double yj = (double)y[(size_t)j * HW + p];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t g = (size_t)(j * R + r) * HW + p;
      const float ur = u[g];
      const float dr = d_from_f ? d[g] - ur : d[g];
      bb[r] = rho * ((double)ur - (double)dr);
      if ((m >> r) & 1u) bb[r] += yj;
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
      if (periodic) Yw[g] = bw[r];
    }
    sigma = gamma * gamma * er[R - 1];
    carry_b = gamma * bb[R - 1];
    carry_w = gamma * bw[R - 1];
  }
  // backward sweep, x_j = y_j + gamma x_{j+1,1} z_j (overwriting y in the scratch)
  double nb = 0.0, nw = 0.0;
  double xb_first = 0.0, xb_last = 0.0, xw_first = 0.0, xw_last = 0.0;
  for (int j = N - 1; j >= 0; --j) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t g = (size_t)(j * R + r) * HW + p;
      const double z = Zs[g];
      const double xb = Yb[g] + gamma * nb * z;
      Yb[g] = xb;
      if (j == N - 1 && r == R - 1) xb_last = xb;
      if (j == 0 && r == 0) xb_first = xb;
      if (periodic) {
        const double xw = Yw[g] + gamma * nw * z;
        Yw[g] = xw;
        if (j == N - 1 && r == R - 1) xw_last = xw;
        if (j == 0 && r == 0) xw_first = xw;
      }
    }
    nb = Yb[(size_t)(j * R) * HW + p];
    if (periodic) nw = Yw[(size_t)(j * R) * HW + p];
  }
  double coef = 0.0;
  if (periodic) coef = gamma * (xb_first - xb_last) / (1.0 + gamma * (xw_first - xw_last));
  for (int g = 0; g < NR; ++g) {
    const size_t o = (size_t)g * HW + p;
    double xv = Yb[o];
    if (periodic) xv -= coef * Yw[o];
    const float ur = u[o];
    const float dr = d_from_f ? d[o] - ur : d[o];
    if (x_out) x_out[o] = (float)xv;
    if (f_out) f_out[o] = (float)(xv + (double)dr);
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

}  // namespace

size_t multishot_scratch_bytes(const cspnp_desc& de) {
  return de.N > 1 ? 3 * (size_t)de.N * de.R * de.H * de.W * sizeof(double) : 0;
}

hipError_t launch_xupdate_multishot(const cspnp_plan& pl, double rho, double gamma, const float* y, const float* u,
                                    const float* d, bool d_from_f, float* x_out, float* f_out, hipStream_t s) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  const int periodic = (de.zbc == CSPNP_ZBC_PERIODIC && NR >= 2 && gamma > 0) ? 1 : 0;
  const size_t HW = (size_t)de.H * de.W;
  const unsigned blocks = (unsigned)((HW + 255) / 256);
  return AllR::dispatch(de.R, [&](auto rc) {
    hipLaunchKernelGGL(xupdate_multishot<decltype(rc)::value>, dim3(blocks), dim3(256), 0, s, pl.bits, de.H, de.W,
                       pl.Wq, de.N, rho, gamma, periodic, y, u, d, d_from_f ? 1 : 0, x_out, f_out, pl.ms_scratch);
    return hipGetLastError();
  });
}

}  // namespace cspnp
