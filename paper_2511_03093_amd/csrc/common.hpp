// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cspnp.h"

#define CSPNP_API extern "C" __attribute__((visibility("default")))

namespace cspnp {

constexpr int kMaxR = 32;

// Error text of the last failed call on this thread.
void set_error(const std::string& msg);
void clear_error();
int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define CSPNP_HIP(call)                                \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

// Per-pixel z-solve constants for T = rho I + gamma L_N (free-ends chain),
// LDL^T factored in FP64 on the host: T = L D L^T with unit lower bidiagonal L
// (sub-diagonal l[i], i >= 1) and D = diag(1/invd[i]).  For the periodic chain
// the wrap pair adds gamma w w^T with w = e_0 - e_{R-1}; c = T^{-1} w and
// wc = w^T c are precomputed for the rank-2 Woodbury correction.
struct ZSolve {
  double l[kMaxR];
  double invd[kMaxR];
  double c[kMaxR];
  double wc;
  double rho;
  double gamma;
  int32_t periodic;  // 1 when the wrap term is present (periodic, R >= 2, gamma > 0)
  int32_t pad;
};

ZSolve make_zsolve(int R, int zbc, double rho, double gamma);

// TV dual-projection settings for one launch.
struct TvArgs {
  float theta;    // lambda / rho
  float inv_theta;
  float tau;
  int32_t iters;  // inner iterations fused into this launch
};

struct TvShapeInfo {
  int cx, s, nw;  // lane columns, rows per lane, waves per workgroup
  int cols, rows; // tile size in pixels
};

// Appends the bytes of v to a graph-cache key.
template <typename T>
inline void key_append(std::vector<uint8_t>& k, const T& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

// Captured iteration graphs of a plan, keyed by (parameters, pointers); a few
// are kept (least recently used evicted) so alternating call patterns replay.
struct GraphEntry {
  std::vector<uint8_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

struct GraphCache {
  static constexpr size_t kMax = 4;
  std::vector<GraphEntry> entries;
  uint64_t clock = 0;
  GraphEntry* find(const std::vector<uint8_t>& key) {
    for (auto& e : entries)
      if (e.exec && e.key == key) {
        e.last_use = ++clock;
        return &e;
      }
    return nullptr;
  }
  // an empty entry (evicting the least recently used one when full)
  GraphEntry& slot() {
    if (entries.size() < kMax) {
      entries.emplace_back();
      return entries.back();
    }
    GraphEntry* lru = &entries[0];
    for (auto& e : entries)
      if (e.last_use < lru->last_use) lru = &e;
    release(*lru);
    return *lru;
  }
  static void release(GraphEntry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
    e.key.clear();
  }
  void clear() {
    for (auto& e : entries) release(e);
    entries.clear();
  }
  ~GraphCache() { clear(); }
};

}  // namespace cspnp

struct cspnp_plan {
  cspnp_desc desc;
  int device = 0;
  int Wq = 0;                    // 32-bit words per bit-plane row
  uint32_t* bits = nullptr;      // device uint32[R][H][Wq]
  // N = 1: the same masks pixel-major, bit r of pixel p = mask r at p; uint16[H][W]
  // when R <= 16, uint32[H][W] otherwise (one load per pixel in the x-step)
  void* pmask = nullptr;
  hipStream_t capture_stream = nullptr;
  cspnp::GraphCache graph;
  int tv_shape = 0;  // index into the TV tile-shape table
  int xu_block = 0;  // index into the x-update block-shape table
  double* dct = nullptr;  // device 8x8 DCT-II matrix (BM3D plans)
  double* ms_scratch = nullptr;  // FP64 scratch of the multi-shot x-step (N > 1)
  ~cspnp_plan();
};

namespace cspnp {

int validate_plan(const cspnp_plan* plan);
int validate_params(const cspnp_plan* plan, const cspnp_params* p);
int check_ptr(const void* p, const char* name);

// Kernel launchers (enqueue only; arguments already validated).
hipError_t launch_forward(const cspnp_plan& pl, const float* x, float* y, hipStream_t s);
hipError_t launch_adjoint(const cspnp_plan& pl, const float* y, float* x, hipStream_t s);
// x-step; writes x_out and/or f_out = x + d.  When tik_lam_over >= 0 the
// Tikhonov prox and d-step are fused: u_out = rho f/(2 lambda + rho), d_out = f - u.
// d_from_f: `d` holds the previous f and d = f - u is formed on the fly (f_out may alias it).
hipError_t launch_xupdate(const cspnp_plan& pl, const ZSolve& zs, const float* y, const float* u,
                          const float* d, float* x_out, float* f_out, hipStream_t s, bool d_from_f = false);
hipError_t launch_xupdate_tikhonov(const cspnp_plan& pl, const ZSolve& zs, double lambda,
                                   const float* y, float* u, float* d, float* x_out,
                                   hipStream_t s);
hipError_t launch_tikhonov(const cspnp_plan& pl, double lambda, double rho, const float* f,
                           float* u, float* d_out, hipStream_t s);
// TV prox of every slice of f; ws holds the dual field between passes when
// the inner iterations do not fit one fused launch.
size_t tv_workspace_bytes(const cspnp_plan& pl, int tv_inner);
// p^1..p^K of the Chambolle iteration of every slice of f (from p = 0) into the tape:
// px^t at tape + 2 t tape_stride, py^t at tape + (2 t + 1) tape_stride; 1 <= K <= 16.
hipError_t launch_tv_tape(const cspnp_plan& pl, double lambda, double rho, int tv_inner, double tau, const float* f,
                          float* tape, size_t tape_stride, hipStream_t st);
hipError_t launch_tv(const cspnp_plan& pl, double lambda, double rho, int tv_inner, double tau,
                     const float* f, float* u, float* d_out, void* ws, hipStream_t s);
// nslices > 0: denoise only the first nslices slices starting at f/u/d_out (default: all).
hipError_t launch_tv_shape(const cspnp_plan& pl, int shape, double lambda, double rho, int tv_inner,
                           double tau, const float* f, float* u, float* d_out, void* ws, hipStream_t s,
                           int nslices = 0);
size_t multishot_scratch_bytes(const cspnp_desc& de);
hipError_t launch_xupdate_multishot(const cspnp_plan& pl, double rho, double gamma, const float* y, const float* u,
                                    const float* d, bool d_from_f, float* x_out, float* f_out, hipStream_t s);
hipError_t launch_rel_change(const float* a, const float* b, size_t n, double* out, void* ws, hipStream_t s);
size_t rel_change_ws_bytes();
// Algorithm 1's own schedule (gamma on the u-block, Gauss-Seidel over slices).
size_t paper_workspace_bytes(const cspnp_plan& pl, int tv_inner);
hipError_t enqueue_paper_iterations(const cspnp_plan& pl, const cspnp_params& p, const float* y, float* u,
                                    float* d, float* x, void* ws, hipStream_t s);
size_t bm3d_workspace_bytes(const cspnp_plan& pl);
void make_dct_matrix(double* c);  // 64 entries, row k = frequency
hipError_t launch_bm3d(const cspnp_plan& pl, double sigma, const float* f, float* u, float* d_out, void* ws,
                       hipStream_t s);
int tv_num_shapes();
TvShapeInfo tv_shape_info(int i);
int tv_default_shape(int H, int W, int NR, int tv_inner);
int xu_num_blocks();
void xu_block_info(int i, int* bx, int* by);

}  // namespace cspnp
