// BM3D u-step (the paper's third plug-in prior, Sec. III-B; Dabov et al. 2007),
// every slice of f at noise level sigma, two stages:
//   1. match on f (tau = 3000/255^2) -> 3D transform -> hard threshold 2.7 sigma
//      -> inverse -> aggregate: basic estimate (kept in FP64);
//   2. match on the basic estimate (tau = 400/255^2) -> transform both groups
//      -> Wiener shrinkage W = B^2/(B^2 + sigma^2) of the noisy group -> inverse
//      -> aggregate: u; d = f - u.
// 8x8 blocks, reference grid step 3 (plus the last position), +-19 search
// window clipped to the slice, groups of at most 16 blocks (reference first,
// then by (distance, raster index)) truncated to a power of two, orthonormal
// DCT-II per block and orthonormal Haar along the group.
//
// The two discrete decisions (which blocks form a group, which coefficients
// survive the threshold) are taken in FP64.  Block distances are evaluated in
// a fixed order -- for each block column the sum over rows of (a - b)^2, then
// the sum of the column sums, without fused multiply-adds -- so they are
// reproducible exactly.
//
// Kernels: bm3d_match (one wave per row of 62 references, lane = reference,
// column sums shared through LDS, the search region of 8 reference rows staged
// in LDS, the 15 best candidates kept sorted in registers), bm3d_filter (one wave per group: the
// group's 64 pixels per block across 64 lanes, the 2D DCT through LDS, the
// Haar transform along the group in registers, aggregation of an 8 x 8 tile of
// groups into LDS with FP64 atomics, then once per pixel into the numerator and
// denominator volumes), bm3d_divide_* (division).
#include <cmath>

#include "common.hpp"

namespace cspnp {

namespace {

constexpr int kP = 8;
constexpr int kStep = 3;
constexpr int kRadius = 19;
constexpr int kNmax = 16;
constexpr int kMRefs = 62;                                        // references per matching wave
constexpr int kMWaves = 8;                                        // reference rows per matching workgroup
constexpr int kMRows = (kMWaves - 1) * kStep + kP + 2 * kRadius;  // 67 region rows
constexpr int kMCols = 64 * 3 + 2 * kRadius;                      // 230 region columns
constexpr int kRowStride = kP + 1;                                // DCT scratch: padded block rows
constexpr int kBlkStride = kP * kRowStride;
constexpr int kFTile = 8;                                         // filter workgroup: 8 x 8 references
constexpr int kFWaves = 8;
constexpr int kFReg = (kFTile - 1) * kStep + kP + 2 * kRadius;    // 67: the tile's blocks lie in this square
constexpr double kTauHt = 3000.0 / (255.0 * 255.0);
constexpr double kTauWie = 400.0 / (255.0 * 255.0);
constexpr double kLambda3d = 2.7;


__host__ __device__ inline int ref_count(int n) { return (n - kP) / kStep + 1 + (((n - kP) % kStep) ? 1 : 0); }
__device__ inline int ref_pos(int i, int n) { return min(i * kStep, n - kP); }

// Block matching, one wave per row of references: lane i is the reference of
// column index ix0 + i (lanes 62 and 63 hold none and only help with column
// sums).  For every displacement (dy, dx) in [-19, 19]^2 the wave forms the
// column sums s(x) = sum_r (a - b)^2 over the block's 8 rows for every column x
// its references cover -- each lane three consecutive columns, exchanged
// through LDS -- and a reference's distance is the sum of its 8 column sums in
// column order.  That is exactly the fixed order a distance is defined with
// (column sums over rows, then their sum, no fused multiply-add), so sharing
// column sums between the references of a row changes no rounding.  The
// workgroup's 8 reference rows and their search region are staged in LDS.
template <typename T>
__global__ __launch_bounds__(64 * kMWaves) void bm3d_match(const T* __restrict__ img, int H, int W, double tau,
                                                           int* __restrict__ matches, int* __restrict__ counts) {
#pragma clang fp contract(off)
  __shared__ T reg[kMRows * kMCols];
  __shared__ double colbuf[kMWaves][64 * 3];
  const int nry = ref_count(H), nrx = ref_count(W);
  const int slice = blockIdx.z;
  const int iy0 = blockIdx.y * kMWaves, ix0 = blockIdx.x * kMRefs;
  // first column of lane 0 (the reference position of ix0: 3 ix0, or W - 8 when ix0 is the
  // last, irregular reference) and the region origin; the region may reach outside the image
  // and is filled with clamped reads there (never a valid candidate)
  const int xbase = ref_pos(ix0, W);
  const int oy = ref_pos(iy0, H) - kRadius, ox = xbase - kRadius;
  const T* __restrict__ im = img + (size_t)slice * H * W;
  for (int i = threadIdx.x; i < kMRows * kMCols; i += 64 * kMWaves) {
    const int y = i / kMCols, x = i - y * kMCols;
    const int gy = min(max(oy + y, 0), H - 1), gx = min(max(ox + x, 0), W - 1);
    reg[i] = im[(size_t)gy * W + gx];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int iy = iy0 + wave;
  if (iy >= nry) return;  // the whole wave leaves; only wave-level synchronisation follows
  const int ry = ref_pos(iy, H);
  const int ix = ix0 + lane;
  const bool is_ref = lane < kMRefs && ix < nrx;
  const int rx = is_ref ? ref_pos(ix, W) : xbase;
  const int k0 = rx - xbase;  // this reference's first column among the wave's columns
  const int ryl = ry - oy;    // region row of the reference block's first row (19..40)
  double a[kP][3];
#pragma unroll
  for (int rr = 0; rr < kP; ++rr)
#pragma unroll
    for (int j = 0; j < 3; ++j) a[rr][j] = (double)reg[(ryl + rr) * kMCols + 3 * lane + j + kRadius];
  double bd[kNmax - 1];
  int bi[kNmax - 1];
#pragma unroll
  for (int k = 0; k < kNmax - 1; ++k) {
    bd[k] = INFINITY;
    bi[k] = 0x7fffffff;
  }
  double* cb = colbuf[wave];
  for (int dy = -kRadius; dy <= kRadius; ++dy) {
    const int cy = ry + dy;
    if (cy < 0 || cy > H - kP) continue;  // wave-uniform: no reference of the row has this candidate row
    const T* crow = reg + (ryl + dy) * kMCols + 3 * lane + kRadius;
    for (int dx = -kRadius; dx <= kRadius; ++dx) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double col = 0.0;
#pragma unroll
        for (int rr = 0; rr < kP; ++rr) {
          const double t = a[rr][j] - (double)crow[rr * kMCols + j + dx];
          col = col + t * t;
        }
        cb[3 * lane + j] = col;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const int cx = rx + dx;
      if (is_ref && cx >= 0 && cx <= W - kP && (dy != 0 || dx != 0)) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kP; ++c) acc = acc + cb[k0 + c];
        const double d = acc * (1.0 / (kP * kP));
        if (d <= tau && d < bd[kNmax - 2]) {
          // insertion: walk the (distance, raster index) ordered list, carrying the displaced entry
          double cd = d;
          int ci = cy * W + cx;
#pragma unroll
          for (int k = 0; k < kNmax - 1; ++k) {
            const bool better = cd < bd[k] || (cd == bd[k] && ci < bi[k]);
            const double td = bd[k];
            const int ti = bi[k];
            bd[k] = better ? cd : td;
            bi[k] = better ? ci : ti;
            cd = better ? td : cd;
            ci = better ? ti : ci;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
  if (!is_ref) return;
  const size_t g = ((size_t)slice * nry + iy) * nrx + ix;
  int* out = matches + g * kNmax;
  out[0] = ry * W + rx;
  int nvalid = 1;
#pragma unroll
  for (int k = 0; k < kNmax - 1; ++k) {
    out[k + 1] = bi[k];
    if (bd[k] != INFINITY) ++nvalid;
  }
  int n = 1;
  while (n * 2 <= nvalid) n *= 2;
  counts[g] = n;
}

// In-register orthonormal Haar along the group (full decomposition), N a power of two:
// each level maps pairs to (sum, difference)/sqrt(2), averages first, then recurses on them.
template <int N>
__device__ __forceinline__ void haar_fwd(double (&v)[kNmax]) {
  const double s = 0.70710678118654752440;
  double t[kNmax];
#pragma unroll
  for (int len = N; len > 1; len >>= 1) {
#pragma unroll
    for (int i = 0; i < len / 2; ++i) {
      t[i] = (v[2 * i] + v[2 * i + 1]) * s;
      t[len / 2 + i] = (v[2 * i] - v[2 * i + 1]) * s;
    }
#pragma unroll
    for (int i = 0; i < len; ++i) v[i] = t[i];
  }
}

template <int N>
__device__ __forceinline__ void haar_inv(double (&v)[kNmax]) {
  const double s = 0.70710678118654752440;
  double t[kNmax];
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
    for (int i = 0; i < len / 2; ++i) {
      const double a = v[i], b = v[len / 2 + i];
      t[2 * i] = (a + b) * s;
      t[2 * i + 1] = (a - b) * s;
    }
#pragma unroll
    for (int i = 0; i < len; ++i) v[i] = t[i];
  }
}

template <bool INVERSE>
__device__ __forceinline__ void haar(double (&v)[kNmax], int n) {
  switch (n) {
    case 2: INVERSE ? haar_inv<2>(v) : haar_fwd<2>(v); break;
    case 4: INVERSE ? haar_inv<4>(v) : haar_fwd<4>(v); break;
    case 8: INVERSE ? haar_inv<8>(v) : haar_fwd<8>(v); break;
    case 16: INVERSE ? haar_inv<16>(v) : haar_fwd<16>(v); break;
    default: break;  // n = 1: identity
  }
}

// 2D DCT (forward: C X C^T, inverse: C^T X C) of the wave's n blocks; lane = 8*r + c
// holds pixel (r, c) of every block in v[b].  buf: the wave's LDS scratch
// [kNmax][kBlkStride]; rows are padded to 9 doubles so that the eight rows a row
// pass reads at once fall in distinct LDS banks.
// The DCT matrix lives in device (global) memory; a pointer read from an
// argument struct is generic, and generic loads could alias the LDS scratch,
// which would keep the compiler from hoisting them out of the block loops.
typedef __attribute__((address_space(1))) const double gdouble;

template <bool INVERSE>
__device__ __forceinline__ void dct2(const double* Cp, double (&v)[kNmax], int n, double* buf, int lane) {
  const gdouble* __restrict__ C = (const gdouble*)Cp;
  const int r = lane >> 3, c = lane & 7;
  const int me = r * kRowStride + c;
  // pass 1 along rows: forward Y[r][k=c] = sum_j C[c][j] X[r][j]; inverse Y[r][j=c] = sum_m X[r][m] C[m][c]
#pragma unroll
  for (int b = 0; b < kNmax; ++b)
    if (b < n) buf[b * kBlkStride + me] = v[b];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int b = 0; b < kNmax; ++b)
    if (b < n) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kP; ++j)
        s += (INVERSE ? C[j * kP + c] : C[c * kP + j]) * buf[b * kBlkStride + r * kRowStride + j];
      v[b] = s;
    }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int b = 0; b < kNmax; ++b)
    if (b < n) buf[b * kBlkStride + me] = v[b];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // pass 2 along columns: forward Z[k=r][m=c] = sum_i C[r][i] Y[i][c]; inverse X[i=r][c] = sum_k C[k][r] Y[k][c]
#pragma unroll
  for (int b = 0; b < kNmax; ++b)
    if (b < n) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < kP; ++i)
        s += (INVERSE ? C[i * kP + r] : C[r * kP + i]) * buf[b * kBlkStride + i * kRowStride + c];
      v[b] = s;
    }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct FilterArgs {
  const double* C;  // device DCT matrix, C[k*8 + j] = a_k cos(pi (2j+1) k / 16)
  double sigma;
  double thr;  // hard threshold (stage 1)
  int H, W, nry, nrx;
  int wiener;
};

// One workgroup per 8 x 8 tile of references, one wave per group (each wave
// filters eight groups in turn).  Stage 1 (wiener = 0): noisy = img.  Stage 2:
// basic drives the Wiener weights.  Every block of the tile's groups lies in the
// 67 x 67 region around the tile (the search window reaches 19 pixels out), so
// the weighted block estimates are first summed into that region in LDS and the
// region is then added to the slice's numerator and denominator once per pixel.
__global__ __launch_bounds__(64 * kFWaves) void bm3d_filter(const FilterArgs a, const float* __restrict__ img,
                                                            const double* __restrict__ basic,
                                                            const int* __restrict__ matches,
                                                            const int* __restrict__ counts, double* __restrict__ num,
                                                            double* __restrict__ den) {
  __shared__ double lds[kFWaves][kNmax * kBlkStride];
  __shared__ double accn[kFReg * kFReg];
  __shared__ double accd[kFReg * kFReg];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slice = blockIdx.z;
  const int iy0 = blockIdx.y * kFTile, ix0 = blockIdx.x * kFTile;
  const int oy = ref_pos(iy0, a.H) - kRadius, ox = ref_pos(ix0, a.W) - kRadius;
  const size_t HW = (size_t)a.H * a.W;
  for (int i = threadIdx.x; i < kFReg * kFReg; i += 64 * kFWaves) {
    accn[i] = 0.0;
    accd[i] = 0.0;
  }
  __syncthreads();
  const int r = lane >> 3, c = lane & 7;
  double* buf = lds[wave];
  for (int k = wave; k < kFTile * kFTile; k += kFWaves) {
    const int iy = iy0 + k / kFTile, ix = ix0 + k % kFTile;
    if (iy >= a.nry || ix >= a.nrx) continue;  // wave-uniform
    const size_t g = ((size_t)slice * a.nry + iy) * a.nrx + ix;
    const int n = counts[g];
    const int* m = matches + g * kNmax;
    int off[kNmax];
    double v[kNmax], bv[kNmax];
#pragma unroll
    for (int b = 0; b < kNmax; ++b) {
      off[b] = 0;
      v[b] = 0.0;
      bv[b] = 0.0;
      if (b < n) {
        const int idx = m[b];
        const int y = idx / a.W, x = idx - y * a.W;
        const int o = (y + r) * a.W + (x + c);
        off[b] = (y + r - oy) * kFReg + (x + c - ox);
        v[b] = (double)img[slice * HW + o];
        if (a.wiener) bv[b] = basic[slice * HW + o];
      }
    }
    dct2<false>(a.C, v, n, buf, lane);
    haar<false>(v, n);
    double w;
    if (!a.wiener) {
      double kept = 0.0;
#pragma unroll
      for (int b = 0; b < kNmax; ++b)
        if (b < n) {
          if (fabs(v[b]) >= a.thr) kept += 1.0;
          else v[b] = 0.0;
        }
      kept = wave_sum(kept);
      w = 1.0 / (a.sigma * a.sigma * fmax(1.0, kept));
    } else {
      dct2<false>(a.C, bv, n, buf, lane);
      haar<false>(bv, n);
      double wn = 0.0;
      const double s2 = a.sigma * a.sigma;
#pragma unroll
      for (int b = 0; b < kNmax; ++b)
        if (b < n) {
          const double bb = bv[b] * bv[b];
          const double wc = bb / (bb + s2);
          v[b] *= wc;
          wn += wc * wc;
        }
      wn = wave_sum(wn);
      w = 1.0 / (s2 * (wn > 0.0 ? wn : 1.0));
    }
    haar<true>(v, n);
    dct2<true>(a.C, v, n, buf, lane);
#pragma unroll
    for (int b = 0; b < kNmax; ++b)
      if (b < n) {
        atomicAdd(&accn[off[b]], w * v[b]);
        atomicAdd(&accd[off[b]], w);
      }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kFReg * kFReg; i += 64 * kFWaves) {
    const double dv = accd[i];
    if (dv == 0.0) continue;  // no block of the tile covers this pixel (and none outside the image does)
    const int y = oy + i / kFReg, x = ox + i % kFReg;
    const size_t o = slice * HW + (size_t)y * a.W + x;
    unsafeAtomicAdd(num + o, accn[i]);
    unsafeAtomicAdd(den + o, dv);
  }
}

__global__ __launch_bounds__(256) void fill_zero_d(double* p, size_t n) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) p[i] = 0.0;
}

__global__ __launch_bounds__(256) void bm3d_divide_basic(const double* __restrict__ num, const double* __restrict__ den,
                                                         double* __restrict__ basic, size_t n) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) basic[i] = num[i] / den[i];
}

__global__ __launch_bounds__(256) void bm3d_divide_out(const double* __restrict__ num, const double* __restrict__ den,
                                                       const float* __restrict__ f, float* __restrict__ u,
                                                       float* __restrict__ d_out, size_t n) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    const float uv = (float)(num[i] / den[i]);
    u[i] = uv;
    if (d_out) d_out[i] = f[i] - uv;
  }
}

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

struct Bm3dLayout {
  size_t matches, counts, num, den, basic, total;
};

Bm3dLayout bm3d_layout(const cspnp_plan& pl) {
  const auto& de = pl.desc;
  const size_t NR = (size_t)de.N * de.R;
  const size_t refs = NR * ref_count(de.H) * ref_count(de.W);
  const size_t vol = NR * de.H * de.W;
  Bm3dLayout L;
  size_t o = 0;
  L.matches = o; o += align_up(refs * kNmax * sizeof(int));
  L.counts = o; o += align_up(refs * sizeof(int));
  L.num = o; o += align_up(vol * sizeof(double));
  L.den = o; o += align_up(vol * sizeof(double));
  L.basic = o; o += align_up(vol * sizeof(double));
  L.total = o;
  return L;
}

}  // namespace

void make_dct_matrix(double* c) {
  for (int k = 0; k < kP; ++k) {
    const double a = k == 0 ? std::sqrt(1.0 / kP) : std::sqrt(2.0 / kP);
    for (int j = 0; j < kP; ++j) c[k * kP + j] = a * std::cos(M_PI * (2 * j + 1) * k / (2.0 * kP));
  }
}

size_t bm3d_workspace_bytes(const cspnp_plan& pl) { return bm3d_layout(pl).total; }

hipError_t launch_bm3d_stages(const cspnp_plan& pl, double sigma, const float* f, float* u, float* d_out, void* ws,
                              int stop_after, hipStream_t s) {
  const auto& de = pl.desc;
  const int NR = de.N * de.R;
  const Bm3dLayout L = bm3d_layout(pl);
  char* w = static_cast<char*>(ws);
  int* matches = reinterpret_cast<int*>(w + L.matches);
  int* counts = reinterpret_cast<int*>(w + L.counts);
  double* num = reinterpret_cast<double*>(w + L.num);
  double* den = reinterpret_cast<double*>(w + L.den);
  double* basic = reinterpret_cast<double*>(w + L.basic);
  const int nry = ref_count(de.H), nrx = ref_count(de.W);
  const size_t vol = (size_t)NR * de.H * de.W;
  const dim3 mgrid((nrx + kMRefs - 1) / kMRefs, (nry + kMWaves - 1) / kMWaves, NR);
  FilterArgs fa;
  fa.C = pl.dct;
  fa.sigma = sigma;
  fa.thr = kLambda3d * sigma;
  fa.H = de.H;
  fa.W = de.W;
  fa.nry = nry;
  fa.nrx = nrx;
  const dim3 fgrid((nrx + kFTile - 1) / kFTile, (nry + kFTile - 1) / kFTile, NR);
  // stage 1
  hipLaunchKernelGGL(bm3d_match<float>, mgrid, dim3(64 * kMWaves), 0, s, f, de.H, de.W, kTauHt, matches, counts);
  if (stop_after == 0) return hipGetLastError();
  hipLaunchKernelGGL(fill_zero_d, dim3(1024), dim3(256), 0, s, num, vol);
  hipLaunchKernelGGL(fill_zero_d, dim3(1024), dim3(256), 0, s, den, vol);
  fa.wiener = 0;
  hipLaunchKernelGGL(bm3d_filter, fgrid, dim3(64 * kFWaves), 0, s, fa, f, nullptr, matches, counts, num, den);
  hipLaunchKernelGGL(bm3d_divide_basic, dim3(1024), dim3(256), 0, s, num, den, basic, vol);
  if (stop_after == 1) return hipGetLastError();
  // stage 2
  hipLaunchKernelGGL(bm3d_match<double>, mgrid, dim3(64 * kMWaves), 0, s, basic, de.H, de.W, kTauWie, matches, counts);
  if (stop_after == 2) return hipGetLastError();
  hipLaunchKernelGGL(fill_zero_d, dim3(1024), dim3(256), 0, s, num, vol);
  hipLaunchKernelGGL(fill_zero_d, dim3(1024), dim3(256), 0, s, den, vol);
  fa.wiener = 1;
  hipLaunchKernelGGL(bm3d_filter, fgrid, dim3(64 * kFWaves), 0, s, fa, f, basic, matches, counts, num, den);
  hipLaunchKernelGGL(bm3d_divide_out, dim3(1024), dim3(256), 0, s, num, den, f, u, d_out, vol);
  return hipGetLastError();
}

hipError_t launch_bm3d(const cspnp_plan& pl, double sigma, const float* f, float* u, float* d_out, void* ws,
                       hipStream_t s) {
  return launch_bm3d_stages(pl, sigma, f, u, d_out, ws, 3, s);
}

}  // namespace cspnp

using namespace cspnp;

CSPNP_API int cspnp_bm3d_stage(const cspnp_plan* plan, const cspnp_params* params, const float* f, int stage,
                               void* ws, void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  if (plan->desc.denoiser != CSPNP_DENOISER_BM3D) return fail(CSPNP_EINVAL, "the plan's denoiser is not BM3D");
  if (check_ptr(f, "f")) return CSPNP_EINVAL;
  if (stage < 0 || stage > 2) return fail(CSPNP_EINVAL, "stage must be 0 (match 1), 1 (basic) or 2 (match 2)");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  CSPNP_HIP(launch_bm3d_stages(*plan, params->bm3d_sigma, f, nullptr, nullptr, ws, stage,
                               reinterpret_cast<hipStream_t>(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_bm3d_layout(const cspnp_plan* plan, size_t* matches_off, size_t* counts_off, size_t* basic_off,
                                int32_t* nry, int32_t* nrx) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (!matches_off || !counts_off || !basic_off || !nry || !nrx) return fail(CSPNP_EINVAL, "NULL output");
  const Bm3dLayout L = bm3d_layout(*plan);
  *matches_off = L.matches;
  *counts_off = L.counts;
  *basic_off = L.basic;
  *nry = ref_count(plan->desc.H);
  *nrx = ref_count(plan->desc.W);
  return CSPNP_OK;
}
