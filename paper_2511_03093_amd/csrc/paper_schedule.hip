// Algorithm 1 exactly as the paper prints it: the temporal term stays on the
// u-block.  Each iteration
//   v-step: eq. (v-update) (no temporal term), per pixel;
//   u-step: one Gauss-Seidel sweep n = 1..NR of eq. (u-update): slice n denoises
//           g_n = (rho (v_n + d_n) + gamma (u_{n-1} + u_{n+1})) / (rho + c_n gamma)
//           at strength lambda / (rho + c_n gamma), c_n the number of z-neighbours
//           (2 with the periodic wrap; the newest available neighbour values);
//   d-step: d = d + v - u.
// The sweep is sequential in n, so each slice is its own launch, with a tile
// shape chosen for one slice (small tiles over many CUs); the sequential sweep is
// the schedule's cost, measured as such.
#include <algorithm>

#include "common.hpp"

namespace cspnp {

namespace {

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

// g = (rho (v + d) + gamma (ua + ub)) / (rho + c gamma), FP64 arithmetic
__global__ __launch_bounds__(256) void gs_datum(size_t n, const float* __restrict__ v, const float* __restrict__ d,
                                                const float* __restrict__ ua, const float* __restrict__ ub,
                                                double rho, double gamma, double denom, float* __restrict__ g) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    double s = rho * ((double)v[i] + (double)d[i]);
    double nb = 0.0;
    if (ua) nb += (double)ua[i];
    if (ub) nb += (double)ub[i];
    g[i] = (float)((s + gamma * nb) / denom);
  }
}

// Tikhonov with the temporal term: u = (rho (v + d) + gamma (ua + ub)) / (2 lambda + rho + c gamma)
__global__ __launch_bounds__(256) void gs_tikhonov(size_t n, const float* __restrict__ v, const float* __restrict__ d,
                                                   const float* ua, const float* ub, double rho, double gamma,
                                                   double denom, float* u) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    double s = rho * ((double)v[i] + (double)d[i]);
    double nb = 0.0;
    if (ua) nb += (double)ua[i];
    if (ub) nb += (double)ub[i];
    u[i] = (float)((s + gamma * nb) / denom);
  }
}

// d = d + v - u
__global__ __launch_bounds__(256) void dstep(size_t n, float* __restrict__ d, const float* __restrict__ v,
                                             const float* __restrict__ u) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull)
    d[i] = (float)(((double)d[i] + (double)v[i]) - (double)u[i]);
}

unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 8192); }

// TV tile shape for a launch over NR slices on `cus` compute units: the fewest
// tile-pixels one CU works through (tile size x ceil(tiles / CUs)), then the
// larger block.  For one slice this picks small tiles spread over the device.
int tv_shape_for_cus(int H, int W, int NR, int tv_inner, int cus) {
  const int halo = tv_inner;  // single pass (tv_inner <= 16 in this schedule's launches)
  long best = -1;
  int bi = 0, bthreads = 0;
  for (int i = 0; i < tv_num_shapes(); ++i) {
    const TvShapeInfo s = tv_shape_info(i);
    const int ix = s.cols - 2 * halo, iy = s.rows - 2 * halo;
    if (ix < 8 || iy < 8) continue;
    const long tiles = (long)((W + ix - 1) / ix) * ((H + iy - 1) / iy) * NR;
    const long cost = (tiles + cus - 1) / cus * (long)s.cols * s.rows;
    const int threads = 64 * s.nw;
    if (best < 0 || cost < best || (cost == best && threads > bthreads)) {
      best = cost;
      bi = i;
      bthreads = threads;
    }
  }
  return best < 0 ? tv_default_shape(H, W, NR, tv_inner) : bi;
}

}  // namespace

size_t paper_workspace_bytes(const cspnp_plan& pl, int tv_inner) {
  const size_t slice = (size_t)pl.desc.H * pl.desc.W;
  return align_up(slice * sizeof(float)) + align_up(tv_workspace_bytes(pl, tv_inner));
}

hipError_t enqueue_paper_iterations(const cspnp_plan& pl, const cspnp_params& p, const float* y, float* u, float* d,
                                    float* x, void* ws, hipStream_t s) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  const size_t HW = (size_t)de.H * de.W;
  const size_t vol = HW * NR;
  float* g = static_cast<float*>(ws);
  void* tws = static_cast<char*>(ws) + align_up(HW * sizeof(float));
  const ZSolve zs = make_zsolve(de.R, de.zbc, p.rho, 0.0);  // the paper's v-step carries no temporal term
  const bool periodic = de.zbc == CSPNP_ZBC_PERIODIC;
  // each u-step launch denoises one slice: small tiles spread it over the device
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl.device) != hipSuccess || cus < 1) cus = 256;
  const int shape = tv_shape_for_cus(de.H, de.W, 1, p.tv_inner, cus);
  for (int k = 0; k < p.iters; ++k) {
    hipError_t e = launch_xupdate(pl, zs, y, u, d, x, nullptr, s);  // v^{k+1} into x
    if (e != hipSuccess) return e;
    for (int n = 0; n < NR; ++n) {
      const float* ua = nullptr;
      const float* ub = nullptr;
      int c = 0;
      if (NR >= 2) {
        int na = n - 1, nb = n + 1;
        if (periodic) {
          na = (n + NR - 1) % NR;
          nb = (n + 1) % NR;
        }
        if (na >= 0 && na < NR) { ua = u + na * HW; ++c; }
        if (nb >= 0 && nb < NR) { ub = u + nb * HW; ++c; }
      }
      const double wsum = p.rho + c * p.gamma;
      if (de.denoiser == CSPNP_DENOISER_TIKHONOV) {
        hipLaunchKernelGGL(gs_tikhonov, dim3(grid_for(HW)), dim3(256), 0, s, HW, x + n * HW, d + n * HW, ua, ub, p.rho,
                           p.gamma, 2.0 * p.lambda + wsum, u + n * HW);
        e = hipGetLastError();
      } else {
        hipLaunchKernelGGL(gs_datum, dim3(grid_for(HW)), dim3(256), 0, s, HW, x + n * HW, d + n * HW, ua, ub, p.rho,
                           p.gamma, wsum, g);
        e = hipGetLastError();
        if (e == hipSuccess)
          e = launch_tv_shape(pl, shape, p.lambda, wsum, p.tv_inner, p.tv_tau, g, u + n * HW, nullptr, tws, s, 1);
      }
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(dstep, dim3(grid_for(vol)), dim3(256), 0, s, vol, d, x, u);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cspnp
