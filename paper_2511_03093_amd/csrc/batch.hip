// Batched solves: many independent snapshots of different sizes and depths
// reconstructed together.  Each ADMM iteration is one persistent grouped
// x-update launch per distinct R (a queue of 256-pixel blocks over all
// problems of that depth) and one persistent grouped TV launch (a queue of
// (problem, slice, tile) entries over all problems); the whole loop is one
// captured HIP graph.  Per-pixel and per-tile arithmetic is exactly that of
// the single-problem kernels, so every batched result equals its unbatched
// solve bit for bit.
//
// Workgroups walk the queues in an XCD-aware order: the hardware hands
// workgroup b to XCD b % 8, so each XCD is given a contiguous chunk of the
// queue (neighbouring tiles of a slice share their halo rows in that XCD's L2).
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include <type_traits>

#include "tv_impl.hpp"
#include "xupdate_impl.hpp"

using namespace cspnp;
using tvimpl::TvLaunch;

namespace {

constexpr int kXuThreads = 256;
constexpr int kNumXcd = 8;

struct XuProblem {
  ZSolve z;
  const void* pmask;  // the plan's pixel-major mask words (uint16 for R <= 16, else uint32)
  const float* y;
  const float* u;
  const float* d;
  float* x;
  float* f;
  int H, W;
};

// Pointers read from a problem record are generic; these are device (global)
// memory, and saying so turns flat accesses into global ones.
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) float gfloat_w;
__device__ __forceinline__ const gfloat* to_global(const float* p) { return (const gfloat*)p; }
__device__ __forceinline__ gfloat_w* to_global(float* p) { return (gfloat_w*)p; }

__device__ __forceinline__ bool next_entry(int& e, int& step, int n, bool first) {
  // XCD-aware static schedule over entries [0, n)
  const int G = gridDim.x;
  if (G < kNumXcd) {
    if (first) { e = blockIdx.x; step = G; } else { e += step; }
    return e < n;
  }
  const int xcd = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const int nblk = (G - xcd + kNumXcd - 1) / kNumXcd;
  const long lo = (long)n * xcd / kNumXcd, hi = (long)n * (xcd + 1) / kNumXcd;
  if (first) { e = (int)lo + j; step = nblk; } else { e += step; }
  return e < hi;
}

template <int R>
__global__ __launch_bounds__(kXuThreads) void batch_xupdate(const XuProblem* __restrict__ probs,
                                                            const int2* __restrict__ entries, int n, int emit_x,
                                                            int d_from_f) {
  int e, step;
  for (bool ok = next_entry(e, step, n, true); ok; ok = next_entry(e, step, n, false)) {
    const int2 en = entries[e];
    // the problem record by value: its pointers stay in registers (the stores
    // below cannot alias them), and the d source is chosen once, so every load
    // of the pixel is issued before the first is needed
    const XuProblem P = probs[en.x];
    const int HW = P.H * P.W;
    const int p = en.y * kXuThreads + threadIdx.x;
    if (p >= HW) continue;
    const int h = p / P.W, w = p - h * P.W;
    typedef typename std::conditional<(R <= 16), uint16_t, uint32_t>::type MW;
    const uint32_t m = ((__attribute__((address_space(1))) const MW*)P.pmask)[p];
    const double yv = (double)to_global(P.y)[p];
    const gfloat* __restrict__ us = to_global(P.u);
    const gfloat* __restrict__ ds = to_global(d_from_f ? P.f : P.d);
    double a[R];
    float dv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float ur = us[(size_t)r * HW + p];
      const float dr = ds[(size_t)r * HW + p];
      dv[r] = d_from_f ? dr - ur : dr;
      a[r] = P.z.rho * ((double)ur - (double)dv[r]);
      if ((m >> r) & 1u) a[r] += yv;
    }
    xuimpl::pixel_solve<R>(P.z, m, a);
    if (emit_x) {
      gfloat_w* xo = to_global(P.x);
#pragma unroll
      for (int r = 0; r < R; ++r) xo[(size_t)r * HW + p] = (float)a[r];
    }
    gfloat_w* fo = to_global(P.f);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // converted here, not kept as FP64 across the solve
      float dr = dv[r];
      asm volatile("" : "+v"(dr));
      fo[(size_t)r * HW + p] = (float)(a[r] + (double)dr);
    }
  }
}

template <int CX, int S, int NW>
__global__ __launch_bounds__(64 * NW) void batch_tv(const TvLaunch* __restrict__ probs, const int4* __restrict__ entries,
                                                    int n, int write_d) {
  __shared__ tvimpl::TvExchange<CX, NW> xch;
  __shared__ tvimpl::TvStage<CX, S, NW> fst;
  int e, step;
  for (bool ok = next_entry(e, step, n, true); ok; ok = next_entry(e, step, n, false)) {
    const int4 en = entries[e];
    TvLaunch a = probs[en.x];
    if (!write_d) a.d_out = nullptr;
    __syncthreads();  // the previous tile's epilogue has finished reading LDS
    tvimpl::tv_tile<CX, S, NW, false, true>(a, en.y, en.z, xch, fst);  // p_in is never set here
  }
}

struct BatchShape {
  int cx, s, nw;
  const void* kernel;
  hipError_t (*launch)(int grid, const TvLaunch*, const int4*, int, int, hipStream_t);
};

template <int CX, int S, int NW>
hipError_t launch_batch_tv(int grid, const TvLaunch* p, const int4* e, int n, int write_d, hipStream_t st) {
  hipLaunchKernelGGL((batch_tv<CX, S, NW>), dim3(grid), dim3(64 * NW), 0, st, p, e, n, write_d);
  return hipGetLastError();
}

#define CSPNP_BSHAPE(CX, S, NW) {CX, S, NW, reinterpret_cast<const void*>(&batch_tv<CX, S, NW>), &launch_batch_tv<CX, S, NW>}
const BatchShape kBShapes[] = {
    CSPNP_BSHAPE(2, 16, 8), CSPNP_BSHAPE(2, 16, 12), CSPNP_BSHAPE(2, 8, 16), CSPNP_BSHAPE(2, 12, 16),
    CSPNP_BSHAPE(3, 8, 16), CSPNP_BSHAPE(3, 12, 8),  CSPNP_BSHAPE(3, 16, 8), CSPNP_BSHAPE(1, 16, 8),
    CSPNP_BSHAPE(2, 8, 8),  CSPNP_BSHAPE(1, 8, 8),
};
#undef CSPNP_BSHAPE
constexpr int kNumBShapes = sizeof(kBShapes) / sizeof(kBShapes[0]);

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

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

template <typename T>
struct DevArray {
  T* p = nullptr;
  size_t n = 0;
  ~DevArray() { if (p) (void)hipFree(p); }
  hipError_t upload(const std::vector<T>& v, hipStream_t s) {
    if (v.size() > n) {
      if (p) { hipError_t e = hipFree(p); if (e != hipSuccess) return e; p = nullptr; }
      hipError_t e = hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T));
      if (e != hipSuccess) return e;
      n = v.size();
    }
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
  }
};

}  // namespace

struct cspnp_batch {
  std::vector<cspnp_plan*> plans;
  std::vector<int> rvals;  // distinct R, ascending
  int cus = 256;
  int tv_shape = 2;
  // device tables (host copies kept alive for the asynchronous uploads)
  std::vector<XuProblem> h_xu;
  std::vector<std::vector<int2>> h_xu_entries;  // per distinct R
  std::vector<TvLaunch> h_tv;
  std::vector<int4> h_tv_entries;
  DevArray<XuProblem> d_xu;
  std::vector<std::unique_ptr<DevArray<int2>>> d_xu_entries;
  DevArray<TvLaunch> d_tv;
  DevArray<int4> d_tv_entries;
  std::vector<int> xu_grid;
  int tv_grid = 0;
  std::vector<uint8_t> key;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~cspnp_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (auto* p : plans) cspnp_plan_destroy(p);
  }
  void drop_graph() {
    if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
    key.clear();
  }
};

namespace {

int validate_batch_params(const cspnp_batch& b, const cspnp_params* params) {
  if (!params) return fail(CSPNP_EINVAL, "params is NULL");
  for (size_t i = 0; i < b.plans.size(); ++i) {
    if (int s = validate_params(b.plans[i], &params[i])) return s;
    if (params[i].iters != params[0].iters) return fail(CSPNP_EINVAL, "all problems of a batch take the same iters");
    if (params[i].tv_inner > 16) return fail(CSPNP_EUNSUPPORTED, "batched TV supports tv_inner <= 16");
  }
  return CSPNP_OK;
}

size_t batch_ws_bytes(const cspnp_batch& b) {
  size_t n = 0;
  for (auto* p : b.plans) n += align_up((size_t)p->desc.R * p->desc.H * p->desc.W * sizeof(float));
  return n;
}

int occupancy_grid(const void* kernel, int threads, int cus, int n_entries) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return std::max(1, std::min(n_entries, per_cu * cus));
}

// Build the per-problem tables and queues for these pointers and parameters.
int prepare(cspnp_batch& b, const cspnp_params* params, const float* const* y, float* const* u, float* const* d,
            float* const* x, char* ws, hipStream_t st) {
  const int n = (int)b.plans.size();
  b.h_xu.assign(n, XuProblem{});
  b.h_tv.assign(n, TvLaunch{});
  b.h_xu_entries.assign(b.rvals.size(), {});
  b.h_tv_entries.clear();
  const BatchShape& sh = kBShapes[b.tv_shape];
  const int TW = 64 * sh.cx, TH = sh.nw * sh.s;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const cspnp_plan& pl = *b.plans[i];
    const auto& de = pl.desc;
    const size_t vol = (size_t)de.R * de.H * de.W;
    float* f = reinterpret_cast<float*>(ws + off);
    off += align_up(vol * sizeof(float));
    XuProblem& X = b.h_xu[i];
    X.z = make_zsolve(de.R, de.zbc, params[i].rho, params[i].gamma);
    X.pmask = pl.pmask;
    X.y = y[i];
    X.u = u[i];
    X.d = d[i];
    X.x = x[i];
    X.f = f;
    X.H = de.H;
    X.W = de.W;
    const int ri = (int)(std::find(b.rvals.begin(), b.rvals.end(), de.R) - b.rvals.begin());
    const int nblk = (de.H * de.W + kXuThreads - 1) / kXuThreads;
    for (int k = 0; k < nblk; ++k) b.h_xu_entries[ri].push_back(int2{i, k});
    TvLaunch& T = b.h_tv[i];
    const double theta = params[i].lambda / params[i].rho;
    const int inner = theta == 0.0 ? 0 : params[i].tv_inner;
    T.f = f;
    T.u = u[i];
    T.d_out = d[i];
    T.p_in = nullptr;
    T.p_out = nullptr;
    T.H = de.H;
    T.W = de.W;
    T.halo = inner;
    T.iters = inner;
    T.theta = (float)theta;
    T.inv_theta = theta > 0 ? (float)(1.0 / theta) : 0.f;
    T.tau = (float)params[i].tv_tau;
    T.vol = vol;
    T.IX = TW - 2 * inner;
    T.IY = TH - 2 * inner;
    if (T.IX < 1 || T.IY < 1) return fail(CSPNP_EUNSUPPORTED, "tv_inner too large for the batch's TV tile shape");
    T.tilesX = (de.W + T.IX - 1) / T.IX;
    const int tilesY = (de.H + T.IY - 1) / T.IY;
    for (int sl = 0; sl < de.R; ++sl)
      for (int t = 0; t < T.tilesX * tilesY; ++t) b.h_tv_entries.push_back(int4{i, t, sl, 0});
  }
  CSPNP_HIP(b.d_xu.upload(b.h_xu, st));
  b.d_xu_entries.resize(b.rvals.size());
  b.xu_grid.assign(b.rvals.size(), 1);
  for (size_t g = 0; g < b.rvals.size(); ++g) {
    if (!b.d_xu_entries[g]) b.d_xu_entries[g].reset(new DevArray<int2>());
    CSPNP_HIP(b.d_xu_entries[g]->upload(b.h_xu_entries[g], st));
    const void* kern = nullptr;
    AllR::dispatch(b.rvals[g], [&](auto rc) {
      kern = reinterpret_cast<const void*>(&batch_xupdate<decltype(rc)::value>);
      return hipSuccess;
    });
    b.xu_grid[g] = occupancy_grid(kern, kXuThreads, b.cus, (int)b.h_xu_entries[g].size());
  }
  CSPNP_HIP(b.d_tv.upload(b.h_tv, st));
  CSPNP_HIP(b.d_tv_entries.upload(b.h_tv_entries, st));
  b.tv_grid = occupancy_grid(sh.kernel, 64 * sh.nw, b.cus, (int)b.h_tv_entries.size());
  return CSPNP_OK;
}

hipError_t enqueue_batch_xu(cspnp_batch& b, int emit_x, int d_from_f, hipStream_t st) {
  for (size_t g = 0; g < b.rvals.size(); ++g) {
    const int n = (int)b.h_xu_entries[g].size();
    hipError_t e = AllR::dispatch(b.rvals[g], [&](auto rc) {
      hipLaunchKernelGGL(batch_xupdate<decltype(rc)::value>, dim3(b.xu_grid[g]), dim3(kXuThreads), 0, st, b.d_xu.p,
                         b.d_xu_entries[g]->p, n, emit_x, d_from_f);
      return hipGetLastError();
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_batch_tv(cspnp_batch& b, int write_d, hipStream_t st) {
  return kBShapes[b.tv_shape].launch(b.tv_grid, b.d_tv.p, b.d_tv_entries.p, (int)b.h_tv_entries.size(), write_d, st);
}

hipError_t enqueue_batch_iters(cspnp_batch& b, int iters, hipStream_t st) {
  // state carried as (u, f) between iterations, as in the single-problem solve
  for (int k = 0; k < iters; ++k) {
    hipError_t e = enqueue_batch_xu(b, k == iters - 1, k > 0, st);
    if (e != hipSuccess) return e;
    e = enqueue_batch_tv(b, k == iters - 1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
void append(std::vector<uint8_t>& k, const T& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

}  // namespace

CSPNP_API int cspnp_batch_create(int32_t n, const cspnp_desc* descs, const uint8_t* const* masks, void* stream,
                                 cspnp_batch** out) {
  clear_error();
  if (n < 1) return fail(CSPNP_EINVAL, "n must be >= 1");
  if (!descs || !masks || !out) return fail(CSPNP_EINVAL, "NULL argument");
  std::unique_ptr<cspnp_batch> b(new cspnp_batch());
  for (int i = 0; i < n; ++i) {
    if (descs[i].denoiser != CSPNP_DENOISER_TV) return fail(CSPNP_EUNSUPPORTED, "batched solves use the TV denoiser");
    if (descs[i].N != 1) return fail(CSPNP_EUNSUPPORTED, "batched solves take N = 1 shot per problem");
    cspnp_plan* p = nullptr;
    if (int s = cspnp_plan_create(&descs[i], masks[i], 0, stream, &p)) return s;
    b->plans.push_back(p);
    if (std::find(b->rvals.begin(), b->rvals.end(), descs[i].R) == b->rvals.end()) b->rvals.push_back(descs[i].R);
  }
  std::sort(b->rvals.begin(), b->rvals.end());
  hipDeviceProp_t prop;
  CSPNP_HIP(hipGetDeviceProperties(&prop, b->plans[0]->device));
  b->cus = prop.multiProcessorCount;
  CSPNP_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  *out = b.release();
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_destroy(cspnp_batch* b) {
  clear_error();
  delete b;
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_workspace_size(const cspnp_batch* b, size_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(CSPNP_EINVAL, "NULL argument");
  *bytes = batch_ws_bytes(*b);
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_set_tv_shape(cspnp_batch* b, int32_t shape) {
  clear_error();
  if (!b) return fail(CSPNP_EINVAL, "batch is NULL");
  if (shape < 0 || shape >= kNumBShapes) return fail(CSPNP_EINVAL, "tv shape out of range");
  b->tv_shape = shape;
  b->drop_graph();
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_get_tv_shape(const cspnp_batch* b, int32_t* shape) {
  clear_error();
  if (!b || !shape) return fail(CSPNP_EINVAL, "NULL argument");
  *shape = b->tv_shape;
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_solve(cspnp_batch* b, const cspnp_params* params, const float* const* y, float* const* u,
                                float* const* d, float* const* x, void* ws, void* stream) {
  clear_error();
  if (!b) return fail(CSPNP_EINVAL, "batch is NULL");
  if (int s = validate_batch_params(*b, params)) return s;
  if (!y || !u || !d || !x) return fail(CSPNP_EINVAL, "NULL pointer array");
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    if (check_ptr(y[i], "y[i]") || check_ptr(u[i], "u[i]") || check_ptr(d[i], "d[i]") || check_ptr(x[i], "x[i]"))
      return CSPNP_EINVAL;
    if (u[i] == d[i] || x[i] == u[i] || x[i] == d[i]) return fail(CSPNP_EINVAL, "u, d, x must be distinct");
  }
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be a 256-byte aligned buffer");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int iters = params[0].iters;
  if (iters == 0) return CSPNP_OK;
  std::vector<uint8_t> key;
  append(key, b->tv_shape);
  append(key, ws);
  for (int i = 0; i < n; ++i) {
    cspnp_params q = params[i];
    q.flags = 0;
    append(key, q);
    append(key, y[i]); append(key, u[i]); append(key, d[i]); append(key, x[i]);
  }
  const bool use_graph = !(params[0].flags & CSPNP_FLAG_NO_GRAPH);
  if (!(b->exec && key == b->key) || !use_graph) {
    b->drop_graph();
    if (int s = prepare(*b, params, y, u, d, x, static_cast<char*>(ws), st)) return s;
    // the tables are read by the kernels: make the uploads complete before any launch
    CSPNP_HIP(hipStreamSynchronize(st));
    if (!use_graph) {
      CSPNP_HIP(enqueue_batch_iters(*b, iters, st));
      return CSPNP_OK;
    }
    CSPNP_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_batch_iters(*b, iters, b->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e, "batched launch during capture"); }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e3, "hipGraphInstantiate"); }
    b->graph = g;
    b->exec = ex;
    b->key = key;
  }
  CSPNP_HIP(hipGraphLaunch(b->exec, st));
  return CSPNP_OK;
}

CSPNP_API int cspnp_batch_autotune(cspnp_batch* b, const cspnp_params* params, const float* const* y, float* const* u,
                                   float* const* d, float* const* x, void* ws, void* stream) {
  clear_error();
  if (!b) return fail(CSPNP_EINVAL, "batch is NULL");
  if (int s = validate_batch_params(*b, params)) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  CSPNP_HIP(hipEventCreate(&e0));
  CSPNP_HIP(hipEventCreate(&e1));
  double best = -1.0;
  int bi = b->tv_shape;
  for (int s = 0; s < kNumBShapes; ++s) {
    b->tv_shape = s;
    b->drop_graph();
    if (prepare(*b, params, y, u, d, x, static_cast<char*>(ws), st) != CSPNP_OK) { clear_error(); continue; }
    CSPNP_HIP(hipStreamSynchronize(st));
    CSPNP_HIP(enqueue_batch_tv(*b, 1, st));
    CSPNP_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) CSPNP_HIP(enqueue_batch_tv(*b, 1, st));
    CSPNP_HIP(hipEventRecord(e1, st));
    CSPNP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    CSPNP_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (best < 0 || ms < best) { best = ms; bi = s; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tv_shape = bi;
  b->drop_graph();
  return CSPNP_OK;
}
