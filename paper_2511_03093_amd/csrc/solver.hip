// C-ABI entry points for the operator, the ADMM pieces and the full solve
// (Algorithm 1 with the temporal term in the x-step).  The iteration loop of
// cspnp_solve is captured once into a HIP graph per (parameters, pointers)
// and replayed on the caller's stream.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

using namespace cspnp;

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align_up(size_t n) { return (n + 255) & ~size_t(255); }

size_t volume_elems(const cspnp_plan& pl) { return (size_t)pl.desc.N * pl.desc.R * pl.desc.H * pl.desc.W; }

size_t denoise_ws_bytes(const cspnp_plan& pl, const cspnp_params& p) {
  if (pl.desc.denoiser == CSPNP_DENOISER_TV) return align_up(tv_workspace_bytes(pl, p.tv_inner));
  if (pl.desc.denoiser == CSPNP_DENOISER_BM3D) return align_up(bm3d_workspace_bytes(pl));
  return 0;
}

size_t solve_ws_bytes(const cspnp_plan& pl, const cspnp_params& p) {
  if (p.flags & CSPNP_FLAG_PAPER_SCHEDULE) return paper_workspace_bytes(pl, p.tv_inner);
  if (pl.desc.denoiser == CSPNP_DENOISER_TIKHONOV && pl.desc.N == 1) return 0;
  // f = x + d between the x-step and the u-step, then the denoiser's own space
  return align_up(volume_elems(pl) * sizeof(float)) + denoise_ws_bytes(pl, p);
}

int check_ws(const cspnp_plan& pl, size_t need, const void* ws) {
  if (need == 0) return CSPNP_OK;
  if (ws == nullptr) return fail(CSPNP_EINVAL, "ws is NULL but the workspace size is not 0");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  return CSPNP_OK;
}

hipError_t enqueue_denoise(const cspnp_plan& pl, const cspnp_params& p, const float* f, float* u,
                           float* d_out, void* ws, hipStream_t s) {
  switch (pl.desc.denoiser) {
    case CSPNP_DENOISER_TIKHONOV: return launch_tikhonov(pl, p.lambda, p.rho, f, u, d_out, s);
    case CSPNP_DENOISER_TV: return launch_tv(pl, p.lambda, p.rho, p.tv_inner, p.tv_tau, f, u, d_out, ws, s);
    case CSPNP_DENOISER_BM3D: return launch_bm3d(pl, p.bm3d_sigma, f, u, d_out, ws, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t enqueue_iterations(const cspnp_plan& pl, const cspnp_params& p, const float* y, float* u,
                              float* d, float* x, void* ws, hipStream_t s) {
  if (p.flags & CSPNP_FLAG_PAPER_SCHEDULE) return enqueue_paper_iterations(pl, p, y, u, d, x, ws, s);
  const ZSolve zs = make_zsolve(pl.desc.R, pl.desc.zbc, p.rho, p.gamma);
  if (pl.desc.denoiser == CSPNP_DENOISER_TIKHONOV && pl.desc.N == 1) {
    for (int k = 0; k < p.iters; ++k) {
      hipError_t e = launch_xupdate_tikhonov(pl, zs, p.lambda, y, u, d, k == p.iters - 1 ? x : nullptr, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // Between iterations the state is carried as (u, f): the u-step writes only u, and the next
  // x-step forms d = f - u itself (the same FP32 subtraction the u-step would store).  The
  // caller's d is read by the first x-step and written by the last u-step.
  float* f = static_cast<float*>(ws);
  void* dws = static_cast<char*>(ws) + align_up(volume_elems(pl) * sizeof(float));
  for (int k = 0; k < p.iters; ++k) {
    const bool first = k == 0, last = k == p.iters - 1;
    hipError_t e = launch_xupdate(pl, zs, y, u, first ? d : f, last ? x : nullptr, f, s, !first);
    if (e != hipSuccess) return e;
    e = enqueue_denoise(pl, p, f, u, last ? d : nullptr, dws, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
void append(std::vector<uint8_t>& k, const T& v) {
  const uint8_t* b = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), b, b + sizeof(T));
}

int check_finite_x(const cspnp_plan& pl, const float* x, hipStream_t s) {
  const size_t n = volume_elems(pl);
  std::vector<float> host(n);
  CSPNP_HIP(hipMemcpyAsync(host.data(), x, n * sizeof(float), hipMemcpyDeviceToHost, s));
  CSPNP_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return fail(CSPNP_ENONFINITE, "non-finite value in x");
  return CSPNP_OK;
}

}  // namespace

CSPNP_API int cspnp_workspace_size(const cspnp_plan* plan, const cspnp_params* params, int mode,
                                   size_t* bytes) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  if (bytes == nullptr) return fail(CSPNP_EINVAL, "bytes is NULL");
  if (mode == CSPNP_WS_SOLVE) *bytes = solve_ws_bytes(*plan, *params);
  else if (mode == CSPNP_WS_SOLVE_TOL)
    *bytes = align_up(solve_ws_bytes(*plan, *params)) + align_up(volume_elems(*plan) * sizeof(float)) +
             rel_change_ws_bytes() + 256;
  else if (mode == CSPNP_WS_DENOISE) *bytes = denoise_ws_bytes(*plan, *params);
  else return fail(CSPNP_EINVAL, "unknown workspace mode");
  return CSPNP_OK;
}

CSPNP_API int cspnp_forward(const cspnp_plan* plan, const float* x, float* y, void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = check_ptr(x, "x")) return s;
  if (int s = check_ptr(y, "y")) return s;
  CSPNP_HIP(launch_forward(*plan, x, y, as_stream(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_adjoint(const cspnp_plan* plan, const float* y, float* x, void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = check_ptr(x, "x")) return s;
  if (int s = check_ptr(y, "y")) return s;
  CSPNP_HIP(launch_adjoint(*plan, y, x, as_stream(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_xupdate(const cspnp_plan* plan, const cspnp_params* params, const float* y,
                            const float* u, const float* d, float* x_out, float* f_out, void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  if (int s = check_ptr(y, "y")) return s;
  if (int s = check_ptr(u, "u")) return s;
  if (int s = check_ptr(d, "d")) return s;
  if (x_out == nullptr && f_out == nullptr) return fail(CSPNP_EINVAL, "x_out and f_out are both NULL");
  if (x_out && check_ptr(x_out, "x_out")) return CSPNP_EINVAL;
  if (f_out && check_ptr(f_out, "f_out")) return CSPNP_EINVAL;
  if (x_out == (float*)u || x_out == (float*)d || f_out == (float*)u || f_out == (float*)d || x_out == f_out)
    return fail(CSPNP_EINVAL, "outputs must not alias inputs or each other");
  const ZSolve zs = make_zsolve(plan->desc.R, plan->desc.zbc, params->rho, params->gamma);
  CSPNP_HIP(launch_xupdate(*plan, zs, y, u, d, x_out, f_out, as_stream(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_denoise(const cspnp_plan* plan, const cspnp_params* params, const float* f, float* u,
                            float* d_out, void* ws, void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  if (int s = check_ptr(f, "f")) return s;
  if (int s = check_ptr(u, "u")) return s;
  if (d_out && check_ptr(d_out, "d_out")) return CSPNP_EINVAL;
  if (u == f || d_out == f || (d_out && d_out == u)) return fail(CSPNP_EINVAL, "u/d_out must not alias f or each other");
  if (int s = check_ws(*plan, denoise_ws_bytes(*plan, *params), ws)) return s;
  CSPNP_HIP(enqueue_denoise(*plan, *params, f, u, d_out, ws, as_stream(stream)));
  return CSPNP_OK;
}

CSPNP_API int cspnp_solve(const cspnp_plan* cplan, const cspnp_params* params, const float* y, float* u,
                          float* d, float* x, void* ws, void* stream) {
  clear_error();
  if (int s = validate_plan(cplan)) return s;
  if (int s = validate_params(cplan, params)) return s;
  if (int s = check_ptr(y, "y")) return s;
  if (int s = check_ptr(u, "u")) return s;
  if (int s = check_ptr(d, "d")) return s;
  if (int s = check_ptr(x, "x")) return s;
  if (u == d || x == u || x == d) return fail(CSPNP_EINVAL, "u, d and x must be distinct buffers");
  if ((params->flags & CSPNP_FLAG_PAPER_SCHEDULE) && cplan->desc.denoiser == CSPNP_DENOISER_BM3D)
    return fail(CSPNP_EUNSUPPORTED, "the paper schedule is implemented for the TV and Tikhonov denoisers");
  if (int s = check_ws(*cplan, solve_ws_bytes(*cplan, *params), ws)) return s;
  cspnp_plan* plan = const_cast<cspnp_plan*>(cplan);  // the graph cache is mutable state
  hipStream_t st = as_stream(stream);
  if (params->iters == 0) return CSPNP_OK;
  if (params->flags & CSPNP_FLAG_NO_GRAPH) {
    CSPNP_HIP(enqueue_iterations(*plan, *params, y, u, d, x, ws, st));
  } else {
    std::vector<uint8_t> key;
    cspnp_params pk = *params;
    pk.flags &= CSPNP_FLAG_PAPER_SCHEDULE;  // the schedule changes the graph; other flags do not
    append(key, pk.flags);
    append(key, pk.lambda); append(key, pk.rho); append(key, pk.gamma); append(key, pk.iters);
    append(key, pk.tv_inner); append(key, pk.tv_tau); append(key, pk.bm3d_sigma);
    append(key, y); append(key, u); append(key, d); append(key, x); append(key, ws);
    GraphEntry* ge = plan->graph.find(key);
    if (!ge) {
      CSPNP_HIP(hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_iterations(*plan, *params, y, u, d, x, ws, plan->capture_stream);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(plan->capture_stream, &g);
      if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e, "kernel launch during capture"); }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      hipGraphExec_t ex = nullptr;
      hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (e3 != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e3, "hipGraphInstantiate"); }
      ge = &plan->graph.slot();
      ge->graph = g;
      ge->exec = ex;
      ge->key = key;
      ge->last_use = ++plan->graph.clock;
    }
    CSPNP_HIP(hipGraphLaunch(ge->exec, st));
  }
  if (params->flags & CSPNP_FLAG_CHECK_FINITE) return check_finite_x(*plan, x, st);
  return CSPNP_OK;
}

CSPNP_API int cspnp_solve_tol(const cspnp_plan* plan, const cspnp_params* params, double tol, int check_every,
                              const float* y, float* u, float* d, float* x, void* ws, void* stream,
                              int32_t* iters_done, double* last_rel) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  if (!(tol >= 0) || check_every < 1) return fail(CSPNP_EINVAL, "tol must be >= 0 and check_every >= 1");
  if (!iters_done || !last_rel) return fail(CSPNP_EINVAL, "iters_done and last_rel must not be NULL");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(CSPNP_EINVAL, "ws must be 256-byte aligned");
  hipStream_t st = as_stream(stream);
  const size_t vol = volume_elems(*plan);
  const size_t solve_ws = align_up(solve_ws_bytes(*plan, *params));
  char* w = static_cast<char*>(ws);
  float* x_prev = reinterpret_cast<float*>(w + solve_ws);
  char* red = w + solve_ws + align_up(vol * sizeof(float));
  double* rel_dev = reinterpret_cast<double*>(red + rel_change_ws_bytes());
  *iters_done = 0;
  *last_rel = -1.0;
  const int K = params->iters;
  int k = 0;
  cspnp_params p = *params;
  while (k < K) {
    const int n = std::min(check_every, K - k);
    if (n > 1) {
      p.iters = n - 1;
      if (int s = cspnp_solve(plan, &p, y, u, d, x, ws, stream)) return s;
    }
    const bool have_prev = k + n - 1 >= 1;  // x holds the previous x-step
    if (have_prev) CSPNP_HIP(hipMemcpyAsync(x_prev, x, vol * sizeof(float), hipMemcpyDeviceToDevice, st));
    p.iters = 1;
    if (int s = cspnp_solve(plan, &p, y, u, d, x, ws, stream)) return s;
    k += n;
    *iters_done = k;
    if (have_prev) {
      CSPNP_HIP(launch_rel_change(x, x_prev, vol, rel_dev, red, st));
      double rel = 0.0;
      CSPNP_HIP(hipMemcpyAsync(&rel, rel_dev, sizeof rel, hipMemcpyDeviceToHost, st));
      CSPNP_HIP(hipStreamSynchronize(st));
      *last_rel = rel;
      if (rel < tol) break;
    }
  }
  return CSPNP_OK;
}
