// Forward operator and adjoint of the DMD-coded acquisition (Sec. III-A,
// eq. (model-slice)), on packed masks.  HBM-bound streaming kernels: each thread
// owns VEC consecutive pixels of one row; 64-lane waves read 64*VEC consecutive
// floats per slice.  One shot (N = 1): the masks come as pixel-major words (all R
// bits of a pixel in one word).  N > 1: bit-planes, where the VEC mask bits of a
// slice share one 32-bit word.
#include "common.hpp"

namespace cspnp {

namespace {

constexpr int kOpThreads = 256;

template <int VEC>
struct Vec;
template <>
struct Vec<1> {
  using T = float;
  static __device__ float get(const T& v, int) { return v; }
  static __device__ void set(T& v, int, float x) { v = x; }
};
template <>
struct Vec<4> {
  using T = float4;
  static __device__ float get(const T& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
  static __device__ void set(T& v, int i, float x) {
    if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x;
  }
};

// streaming (nontemporal) stores of the adjoint's output volume; each volume is
// touched once per launch
using f4n = float __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void nt_store(float v, float* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(const float4& v, float* p) {
  const f4n w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<f4n*>(p));
}

// streaming (nontemporal) loads of the forward's input volume
__device__ __forceinline__ float nt_load(float, const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float4 nt_load(const float4&, const float* p) {
  const f4n w = __builtin_nontemporal_load(reinterpret_cast<const f4n*>(p));
  return make_float4(w.x, w.y, w.z, w.w);
}

// Slices are taken kChunk at a time with every load of a chunk issued before
// the first is used (slice indices clamped to R - 1, their mask words zeroed),
// so one wave keeps kChunk loads in flight instead of waiting once per slice.
constexpr int kChunk = 16;

// y[j][p] = sum_r bit_r(p) * x[j*R + r][p]   (summed in slice order)
template <int VEC>
__global__ __launch_bounds__(kOpThreads) void forward_kernel(const float* __restrict__ x,
                                                             float* __restrict__ y,
                                                             const uint32_t* __restrict__ bits,
                                                             int H, int W, int Wq, int R, int N) {
  using V = Vec<VEC>;
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w0 >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)h * W + w0;
  for (int j = 0; j < N; ++j) {
    float acc[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc[i] = 0.f;
    for (int r0 = 0; r0 < R; r0 += kChunk) {
      uint32_t word[kChunk];
      typename V::T xv[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const int r = min(r0 + q, R - 1);
        word[q] = r0 + q < R ? bits[((size_t)r * H + h) * Wq + (w0 >> 5)] >> (w0 & 31) : 0u;
        xv[q] = nt_load(xv[q], x + (size_t)(j * R + r) * HW + p);
      }
#pragma unroll
      for (int q = 0; q < kChunk; ++q)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[i] += ((word[q] >> i) & 1u) ? V::get(xv[q], i) : 0.f;
    }
    typename V::T out;
#pragma unroll
    for (int i = 0; i < VEC; ++i) V::set(out, i, acc[i]);
    *reinterpret_cast<typename V::T*>(y + (size_t)j * HW + p) = out;
  }
}

// The same for one shot (N = 1) with the plan's pixel-major mask words (MW =
// uint16 for R <= 16, else uint32; bit r of a pixel's word is mask r): a thread's
// VEC words come in one load instead of one bit-plane word per slice.  Two pixels
// per thread (2048 waves at 512x512) measured faster than four (1024 waves) and
// level with one.
// VEC consecutive mask words of one thread
template <typename MW, int VEC>
struct MaskWords {
  uint32_t w[VEC];
  __device__ explicit MaskWords(const MW* p) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) w[i] = p[i];
  }
};
template <>
struct Vec<2> {
  using T = float2;
  static __device__ float get(const T& v, int i) { return i == 0 ? v.x : v.y; }
  static __device__ void set(T& v, int i, float x) {
    if (i == 0) v.x = x; else v.y = x;
  }
};
__device__ __forceinline__ float2 nt_load(const float2&, const float* p) {
  typedef float f2n __attribute__((ext_vector_type(2)));
  const f2n w = __builtin_nontemporal_load(reinterpret_cast<const f2n*>(p));
  return make_float2(w.x, w.y);
}
__device__ __forceinline__ void nt_store(const float2& v, float* p) {
  typedef float f2n __attribute__((ext_vector_type(2)));
  const f2n w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<f2n*>(p));
}

template <typename MW, int VEC>
__global__ __launch_bounds__(kOpThreads) void forward_pm_kernel(const float* __restrict__ x, float* __restrict__ y,
                                                                const MW* __restrict__ pmask, int H, int W, int R) {
  using V = Vec<VEC>;
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w0 >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)h * W + w0;
  const MaskWords<MW, VEC> mk(pmask + p);
  const uint32_t* mw = mk.w;
  float acc[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) acc[i] = 0.f;
  for (int r0 = 0; r0 < R; r0 += kChunk) {
    typename V::T xv[kChunk];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) xv[q] = nt_load(xv[q], x + (size_t)min(r0 + q, R - 1) * HW + p);
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      if (r0 + q >= R) break;
#pragma unroll
      for (int i = 0; i < VEC; ++i) acc[i] += ((mw[i] >> (r0 + q)) & 1u) ? V::get(xv[q], i) : 0.f;
    }
  }
  typename V::T out;
#pragma unroll
  for (int i = 0; i < VEC; ++i) V::set(out, i, acc[i]);
  *reinterpret_cast<typename V::T*>(y + p) = out;
}

template <typename MW, int VEC>
__global__ __launch_bounds__(kOpThreads) void adjoint_pm_kernel(const float* __restrict__ y, float* __restrict__ x,
                                                                const MW* __restrict__ pmask, int H, int W, int R) {
  using V = Vec<VEC>;
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w0 >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)h * W + w0;
  const MaskWords<MW, VEC> mk(pmask + p);
  const uint32_t* mw = mk.w;
  const typename V::T yv = *reinterpret_cast<const typename V::T*>(y + p);
  for (int r = 0; r < R; ++r) {
    typename V::T out;
#pragma unroll
    for (int i = 0; i < VEC; ++i) V::set(out, i, ((mw[i] >> r) & 1u) ? V::get(yv, i) : 0.f);
    nt_store(out, x + (size_t)r * HW + p);
  }
}

// pixels per thread of the one-shot operator kernels
constexpr int kPmVec = 2;

// x[j*R + r][p] = bit_r(p) * y[j][p]
template <int VEC>
__global__ __launch_bounds__(kOpThreads) void adjoint_kernel(const float* __restrict__ y,
                                                             float* __restrict__ x,
                                                             const uint32_t* __restrict__ bits,
                                                             int H, int W, int Wq, int R, int N) {
  using V = Vec<VEC>;
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int h = blockIdx.y * blockDim.y + threadIdx.y;
  if (w0 >= W || h >= H) return;
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)h * W + w0;
  for (int j = 0; j < N; ++j) {
    const typename V::T yv = *reinterpret_cast<const typename V::T*>(y + (size_t)j * HW + p);
    for (int r0 = 0; r0 < R; r0 += kChunk) {
      uint32_t word[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const int r = min(r0 + q, R - 1);
        word[q] = bits[((size_t)r * H + h) * Wq + (w0 >> 5)] >> (w0 & 31);
      }
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        if (r0 + q >= R) break;
        typename V::T out;
#pragma unroll
        for (int i = 0; i < VEC; ++i) V::set(out, i, ((word[q] >> i) & 1u) ? V::get(yv, i) : 0.f);
        nt_store(out, x + (size_t)(j * R + r0 + q) * HW + p);
      }
    }
  }
}

bool vec4_ok(int W, const void* a, const void* b) {
  return (W % 4 == 0) && (reinterpret_cast<uintptr_t>(a) % 16 == 0) &&
         (reinterpret_cast<uintptr_t>(b) % 16 == 0);
}

// Block = (bx lanes along a row) x (rows): bx covers the row's W/VEC threads rounded up
// to a wave (at most the whole block), so narrow images do not launch idle lanes.
dim3 op_block(int W, int vec) {
  const int need = (W / vec + 63) / 64 * 64;
  const int bx = need < kOpThreads ? (need > 0 ? need : 64) : kOpThreads;
  return dim3(bx, kOpThreads / bx);
}

template <typename K>
void op_launch(K kernel, const cspnp_plan& pl, const float* in, float* out, hipStream_t s, int vec) {
  const auto& d = pl.desc;
  const dim3 block = op_block(d.W, vec);
  const dim3 grid((d.W / vec + block.x - 1) / block.x, (d.H + block.y - 1) / block.y);
  hipLaunchKernelGGL(kernel, grid, block, 0, s, in, out, pl.bits, d.H, d.W, pl.Wq, d.R, d.N);
}

}  // namespace

hipError_t launch_forward(const cspnp_plan& pl, const float* x, float* y, hipStream_t s) {
  if (pl.desc.N == 1 && vec4_ok(pl.desc.W, x, y)) {
    const auto& d = pl.desc;
    const dim3 block = op_block(d.W, kPmVec);
    const dim3 grid((d.W / kPmVec + block.x - 1) / block.x, (d.H + block.y - 1) / block.y);
    if (d.R <= 16)
      hipLaunchKernelGGL((forward_pm_kernel<uint16_t, kPmVec>), grid, block, 0, s, x, y, static_cast<const uint16_t*>(pl.pmask),
                         d.H, d.W, d.R);
    else
      hipLaunchKernelGGL((forward_pm_kernel<uint32_t, kPmVec>), grid, block, 0, s, x, y, static_cast<const uint32_t*>(pl.pmask),
                         d.H, d.W, d.R);
  } else if (vec4_ok(pl.desc.W, x, y)) op_launch(forward_kernel<4>, pl, x, y, s, 4);
  else op_launch(forward_kernel<1>, pl, x, y, s, 1);
  return hipGetLastError();
}

hipError_t launch_adjoint(const cspnp_plan& pl, const float* y, float* x, hipStream_t s) {
  if (pl.desc.N == 1 && vec4_ok(pl.desc.W, x, y)) {
    const auto& d = pl.desc;
    const dim3 block = op_block(d.W, kPmVec);
    const dim3 grid((d.W / kPmVec + block.x - 1) / block.x, (d.H + block.y - 1) / block.y);
    if (d.R <= 16)
      hipLaunchKernelGGL((adjoint_pm_kernel<uint16_t, kPmVec>), grid, block, 0, s, y, x, static_cast<const uint16_t*>(pl.pmask),
                         d.H, d.W, d.R);
    else
      hipLaunchKernelGGL((adjoint_pm_kernel<uint32_t, kPmVec>), grid, block, 0, s, y, x, static_cast<const uint32_t*>(pl.pmask),
                         d.H, d.W, d.R);
  } else if (vec4_ok(pl.desc.W, x, y)) op_launch(adjoint_kernel<4>, pl, y, x, s, 4);
  else op_launch(adjoint_kernel<1>, pl, y, x, s, 1);
  return hipGetLastError();
}

}  // namespace cspnp
