// x-step for N > 1 shots per volume: the per-pixel block elimination of
// multishot_impl.hpp with the right-hand side m y + rho (u - d), writing x and
// f = x + d.
#include "multishot_impl.hpp"

namespace cspnp {

namespace {

// LDS: the forward vectors y and z of a wave's 64 pixels live in LDS ([2][NR][64]
// doubles, then the d values as [NR][64] floats) when they fit, else in the plan's
// HBM scratch volume; the periodic wrap's vectors are always in that volume (LDS for
// two arrays lets three workgroups share a CU: at 200x200 pixels every wave is then
// resident at once).
template <int R, bool LDS>
__global__ __launch_bounds__(256) void xupdate_multishot(const uint32_t* __restrict__ bits, int H, int W, int Wq,
                                                         int N, double rho, double gamma, int periodic,
                                                         const float* __restrict__ y, const float* __restrict__ u,
                                                         const float* d, int d_from_f, float* __restrict__ x_out,
                                                         float* f_out, double* __restrict__ scratch) {
  extern __shared__ double lds_scratch[];
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  const int h = (int)(p / W), w = (int)(p % W);
  uint32_t m = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) m |= ((bits[((size_t)r * H + h) * Wq + (w >> 5)] >> (w & 31)) & 1u) << r;
  auto dual = [&](size_t g) {
    const float ur = u[g];
    return d_from_f ? d[g] - ur : d[g];
  };
  // LDS path: the d values of the lane's NR slices are kept in LDS after the
  // [2][NR][64] doubles of the forward sweep, for the output (no second read of u, d)
  const int NR = N * R;
  float* const dl = reinterpret_cast<float*>(lds_scratch + 2 * (size_t)NR * blockDim.x);
  struct Raw {
    float u[R], d[R], y;
    int j;
  };
  auto fetch = [&](int j, Raw& raw) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t g = (size_t)(j * R + r) * HW + p;
      raw.u[r] = u[g];
      raw.d[r] = d[g];
    }
    raw.y = y[(size_t)j * HW + p];
    raw.j = j;
  };
  auto rhs = [&](const Raw& raw, int r) {
    const float ur = raw.u[r];
    const float dr = d_from_f ? raw.d[r] - ur : raw.d[r];
    if constexpr (LDS) dl[(size_t)(raw.j * R + r) * blockDim.x + threadIdx.x] = dr;
    double v = rho * ((double)ur - (double)dr);
    if ((m >> r) & 1u) v += (double)raw.y;
    return v;
  };
  auto out = [&](int j, const double (&xv)[R]) {
    // the block's d values first (f_out may alias the d source), then the stores
    float dr[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      dr[r] = LDS ? dl[(size_t)(j * R + r) * blockDim.x + threadIdx.x] : dual((size_t)(j * R + r) * HW + p);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t o = (size_t)(j * R + r) * HW + p;
      if (x_out) x_out[o] = (float)xv[r];
      if (f_out) f_out[o] = (float)(xv[r] + (double)dr[r]);
    }
  };
  double* const yw = scratch + 2 * (size_t)N * R * HW;  // the wrap's array: HBM on both paths
  if constexpr (LDS)
    msimpl::solve<R, Raw>(m, N, rho, gamma, periodic, blockDim.x, threadIdx.x, lds_scratch, yw, HW, p, fetch, rhs,
                          out);
  else
    msimpl::solve<R, Raw>(m, N, rho, gamma, periodic, HW, p, scratch, yw, HW, p, fetch, rhs, out);
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

constexpr int kLdsLanes = 64;                     // one wave per workgroup on the LDS path
constexpr size_t kMaxLdsScratch = 80 * 1024;      // N R <= 64: at least two workgroups per CU

}  // namespace

// The HBM scratch volume: the forward x-step uses it when the LDS block does not fit,
// the backward's x-step product always.
size_t multishot_scratch_bytes(const cspnp_desc& de) {
  return de.N > 1 ? 3 * (size_t)de.N * de.R * de.H * de.W * sizeof(double) : 0;
}

size_t multishot_lds_bytes(const cspnp_desc& de) {
  return (size_t)de.N * de.R * kLdsLanes * (2 * sizeof(double) + sizeof(float));
}

hipError_t launch_xupdate_multishot(const cspnp_plan& pl, double rho, double gamma, const float* y, const float* u,
                                    const float* d, bool d_from_f, float* x_out, float* f_out, hipStream_t s) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  const int periodic = (de.zbc == CSPNP_ZBC_PERIODIC && NR >= 2 && gamma > 0) ? 1 : 0;
  const size_t HW = (size_t)de.H * de.W;
  const size_t lds = multishot_lds_bytes(de);
  return AllR::dispatch(de.R, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    if (lds <= kMaxLdsScratch) {
      // one wave per workgroup, its pixels' forward vectors in LDS
      hipLaunchKernelGGL((xupdate_multishot<R, true>), dim3((unsigned)((HW + kLdsLanes - 1) / kLdsLanes)),
                         dim3(kLdsLanes), lds, s, pl.bits, de.H, de.W, pl.Wq, de.N, rho, gamma, periodic, y, u, d,
                         d_from_f ? 1 : 0, x_out, f_out, pl.ms_scratch);
    } else {
      hipLaunchKernelGGL((xupdate_multishot<R, false>), dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, pl.bits,
                         de.H, de.W, pl.Wq, de.N, rho, gamma, periodic, y, u, d, d_from_f ? 1 : 0, x_out, f_out,
                         pl.ms_scratch);
    }
    return hipGetLastError();
  });
}

}  // namespace cspnp
