// Launch-shape selection: the TV tile shape and the x-update block shape of
// a plan, set directly or chosen by timing every candidate on the device
// (hipEvent timing on the caller's stream) and remembered in a JSON cache
// keyed by (device arch, H, W, R, N, z boundary, denoiser, TV inner count).
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "common.hpp"

using namespace cspnp;

namespace {

__global__ void fill_pattern(float* p, size_t n, uint32_t seed, float scale) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256ull) {
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = scale * (float)(h & 0xFFFFFF) * (1.0f / 16777216.0f);
  }
}

std::string cache_key(const cspnp_plan& pl, const cspnp_params& p) {
  hipDeviceProp_t prop;
  std::string arch = "gfx?";
  if (hipGetDeviceProperties(&prop, pl.device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
  }
  const auto& d = pl.desc;
  std::ostringstream o;
  o << arch << "/" << d.H << "x" << d.W << "/R" << d.R << "/N" << d.N << "/"
    << (d.zbc == CSPNP_ZBC_PERIODIC ? "periodic" : "neumann") << "/"
    << (d.denoiser == CSPNP_DENOISER_TV ? "tv" : d.denoiser == CSPNP_DENOISER_TIKHONOV ? "tikhonov" : "bm3d")
    << "/inner" << (d.denoiser == CSPNP_DENOISER_TV ? p.tv_inner : 0);
  return o.str();
}

// One entry per line:  "key": {"tv_shape": i, "xu_block": j, ...},
struct Entry {
  int tv_shape = -1, xu_block = -1;
  std::string line;
};

std::map<std::string, Entry> read_cache(const char* path) {
  std::map<std::string, Entry> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    if (q1 == std::string::npos) continue;
    Entry e;
    const std::string key = line.substr(q0 + 1, q1 - q0 - 1);
    auto grab = [&](const char* name) -> int {
      const size_t k = line.find(std::string("\"") + name + "\"", q1);
      if (k == std::string::npos) return -1;
      const size_t c = line.find(':', k);
      return c == std::string::npos ? -1 : std::atoi(line.c_str() + c + 1);
    };
    e.tv_shape = grab("tv_shape");
    e.xu_block = grab("xu_block");
    std::string body = line.substr(q1 + 1);
    while (!body.empty() && (body.back() == ',' || body.back() == ' ' || body.back() == '\r')) body.pop_back();
    e.line = body;
    if (e.tv_shape >= 0 && e.xu_block >= 0) m[key] = e;
  }
  return m;
}

int write_cache(const char* path, const std::map<std::string, Entry>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return fail(CSPNP_EINVAL, std::string("cannot write autotune cache ") + path);
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      f << "  \"" << kv.first << "\"" << kv.second.line << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(CSPNP_EINVAL, std::string("cannot replace ") + path);
  return CSPNP_OK;
}

void invalidate_graph(cspnp_plan& pl) { pl.graph.clear(); }

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

CSPNP_API int cspnp_tuning_candidates(int32_t* n_tv_shapes, int32_t* n_xu_blocks) {
  clear_error();
  if (!n_tv_shapes || !n_xu_blocks) return fail(CSPNP_EINVAL, "NULL output");
  *n_tv_shapes = tv_num_shapes();
  *n_xu_blocks = xu_num_blocks();
  return CSPNP_OK;
}

CSPNP_API int cspnp_tv_shape_info(int32_t index, int32_t* tile_cols, int32_t* tile_rows, int32_t* threads) {
  clear_error();
  if (index < 0 || index >= tv_num_shapes()) return fail(CSPNP_EINVAL, "TV shape index out of range");
  if (!tile_cols || !tile_rows || !threads) return fail(CSPNP_EINVAL, "NULL output");
  const TvShapeInfo s = tv_shape_info(index);
  *tile_cols = s.cols;
  *tile_rows = s.rows;
  *threads = 64 * s.nw;
  return CSPNP_OK;
}

CSPNP_API int cspnp_plan_get_tuning(const cspnp_plan* plan, cspnp_tuning* out) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (!out) return fail(CSPNP_EINVAL, "out is NULL");
  out->tv_shape = plan->tv_shape;
  out->xu_block = plan->xu_block;
  return CSPNP_OK;
}

CSPNP_API int cspnp_plan_set_tuning(cspnp_plan* plan, const cspnp_tuning* t) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (!t) return fail(CSPNP_EINVAL, "tuning is NULL");
  if (t->tv_shape < 0 || t->tv_shape >= tv_num_shapes()) return fail(CSPNP_EINVAL, "tv_shape out of range");
  if (t->xu_block < 0 || t->xu_block >= xu_num_blocks()) return fail(CSPNP_EINVAL, "xu_block out of range");
  plan->tv_shape = t->tv_shape;
  plan->xu_block = t->xu_block;
  invalidate_graph(*plan);
  return CSPNP_OK;
}

CSPNP_API int cspnp_autotune(cspnp_plan* plan, const cspnp_params* params, const char* cache_path, int force,
                             void* stream) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (int s = validate_params(plan, params)) return s;
  const std::string key = cache_key(*plan, *params);
  std::map<std::string, Entry> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (!force && it != cache.end() && it->second.tv_shape < tv_num_shapes() &&
        it->second.xu_block < xu_num_blocks()) {
      plan->tv_shape = it->second.tv_shape;
      plan->xu_block = it->second.xu_block;
      invalidate_graph(*plan);
      return CSPNP_OK;
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const auto& de = plan->desc;
  const size_t vol = (size_t)de.N * de.R * de.H * de.W;
  const size_t frame = (size_t)de.N * de.H * de.W;
  DevBuf y, u, d, f, o1, o2, ws;
  CSPNP_HIP(hipMalloc(&y.p, frame * 4));
  CSPNP_HIP(hipMalloc(&u.p, vol * 4));
  CSPNP_HIP(hipMalloc(&d.p, vol * 4));
  CSPNP_HIP(hipMalloc(&f.p, vol * 4));
  CSPNP_HIP(hipMalloc(&o1.p, vol * 4));
  CSPNP_HIP(hipMalloc(&o2.p, vol * 4));
  const size_t wsb = tv_workspace_bytes(*plan, params->tv_inner);
  if (wsb) CSPNP_HIP(hipMalloc(&ws.p, wsb));
  auto fill = [&](void* p, size_t n, uint32_t seed, float scale) {
    hipLaunchKernelGGL(fill_pattern, dim3(1024), dim3(256), 0, st, (float*)p, n, seed, scale);
  };
  fill(y.p, frame, 1u, (float)de.R * 0.5f);
  fill(u.p, vol, 2u, 1.0f);
  fill(d.p, vol, 3u, 0.1f);
  fill(f.p, vol, 4u, 1.0f);
  CSPNP_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  CSPNP_HIP(hipEventCreate(&e0));
  CSPNP_HIP(hipEventCreate(&e1));
  auto time_it = [&](auto&& launch) -> double {
    for (int i = 0; i < 2; ++i)
      if (launch() != hipSuccess) return -1.0;
    const int reps = 8;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.0;
    for (int i = 0; i < reps; ++i)
      if (launch() != hipSuccess) return -1.0;
    if (hipEventRecord(e1, st) != hipSuccess) return -1.0;
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return 1e3 * ms / reps;
  };
  const int old_xu = plan->xu_block, old_tv = plan->tv_shape;
  const ZSolve zs = make_zsolve(de.R, de.zbc, params->rho, params->gamma);
  double best_xu = -1.0;
  int bx = old_xu;
  for (int i = 0; i < xu_num_blocks(); ++i) {
    plan->xu_block = i;
    const double t = time_it([&] {
      return launch_xupdate(*plan, zs, (const float*)y.p, (const float*)u.p, (const float*)d.p, nullptr,
                            (float*)o1.p, st);
    });
    if (t > 0 && (best_xu < 0 || t < best_xu)) { best_xu = t; bx = i; }
  }
  plan->xu_block = bx;
  double best_tv = -1.0;
  int bt = old_tv;
  if (de.denoiser == CSPNP_DENOISER_TV) {
    for (int i = 0; i < tv_num_shapes(); ++i) {
      const double t = time_it([&] {
        return launch_tv_shape(*plan, i, params->lambda, params->rho, params->tv_inner, params->tv_tau,
                               (const float*)f.p, (float*)o1.p, (float*)o2.p, ws.p, st);
      });
      (void)hipGetLastError();  // shapes whose halo does not fit report an error: skip them
      if (t > 0 && (best_tv < 0 || t < best_tv)) { best_tv = t; bt = i; }
    }
  }
  plan->tv_shape = bt;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CSPNP_HIP(hipStreamSynchronize(st));
  invalidate_graph(*plan);
  if (cache_path) {
    char buf[256];
    std::snprintf(buf, sizeof buf, ": {\"tv_shape\": %d, \"xu_block\": %d, \"tv_us\": %.3f, \"xu_us\": %.3f}", bt, bx,
                  best_tv, best_xu);
    Entry e;
    e.tv_shape = bt;
    e.xu_block = bx;
    e.line = buf;
    cache[key] = e;
    if (int s = write_cache(cache_path, cache)) return s;
  }
  return CSPNP_OK;
}
