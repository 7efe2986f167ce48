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
// neighbours across waves through double-buffered LDS (one barrier per inner
// iteration).
// Values beyond the tile edge are not available, and the error they cause
// spreads one pixel per iteration, so the tile carries a halo of `iters`
// pixels (one more when p is loaded) and writes only its interior.  Pixels
// outside the image keep p = 0, which realises the boundary cases of div.
// When tv_inner is too large for one tile, passes of at most kMaxFused
// iterations exchange p through an HBM workspace.
#include "tv_impl.hpp"

namespace cspnp {

namespace {

using tvimpl::TvLaunch;
using tvimpl::tv_tile;

constexpr int kMaxFused = 16;

// COLD: the launch starts from p = 0 (a single pass, or the first of several).
template <int CX, int S, int NW, bool COLD>
__global__ __launch_bounds__(64 * NW) void tv_kernel(const TvLaunch a) {
  __shared__ tvimpl::TvExchange<CX, NW> xch;
  __shared__ tvimpl::TvStage<CX, S, NW> fst;
  tv_tile<CX, S, NW, false, COLD>(a, blockIdx.x, blockIdx.y, xch, fst);
}

// The backward's tape: the same tile with p^1..p^K written out (128 x 192 tiles).
constexpr int kTapeCX = 2, kTapeS = 12, kTapeNW = 16;

__global__ __launch_bounds__(64 * kTapeNW) void tv_tape_kernel(const TvLaunch a) {
  __shared__ tvimpl::TvExchange<kTapeCX, kTapeNW> xch;
  __shared__ tvimpl::TvStage<kTapeCX, kTapeS, kTapeNW> fst;
  tv_tile<kTapeCX, kTapeS, kTapeNW, true, true>(a, blockIdx.x, blockIdx.y, xch, fst);
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
  if (a.p_in)
    hipLaunchKernelGGL((tv_kernel<CX, S, NW, false>), grid, dim3(64 * NW), 0, st, a);
  else
    hipLaunchKernelGGL((tv_kernel<CX, S, NW, true>), grid, dim3(64 * NW), 0, st, a);
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

hipError_t launch_tv_tape(const cspnp_plan& pl, double lambda, double rho, int tv_inner, double tau, const float* f,
                          float* tape, size_t tape_stride, hipStream_t st) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  if (tv_inner < 1 || tv_inner > kMaxFused) return hipErrorInvalidValue;
  TvLaunch a{};
  a.f = f;
  a.H = de.H;
  a.W = de.W;
  a.vol = (size_t)NR * de.H * de.W;
  const double theta = lambda / rho;
  a.theta = (float)theta;
  a.inv_theta = theta > 0 ? (float)(1.0 / theta) : 0.f;
  a.tau = (float)tau;
  a.iters = tv_inner;
  a.halo = tv_inner;
  a.tape = tape;
  a.tape_stride = tape_stride;
  a.IX = 64 * kTapeCX - 2 * a.halo;
  a.IY = kTapeNW * kTapeS - 2 * a.halo;
  a.tilesX = (a.W + a.IX - 1) / a.IX;
  const int tilesY = (a.H + a.IY - 1) / a.IY;
  hipLaunchKernelGGL(tv_tape_kernel, dim3(a.tilesX * tilesY, NR), dim3(64 * kTapeNW), 0, st, a);
  return hipGetLastError();
}

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
                           double tau, const float* f, float* u, float* d_out, void* ws, hipStream_t st,
                           int nslices) {
  const auto& de = pl.desc;
  const int NR = nslices > 0 ? nslices : de.N * de.R;
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
