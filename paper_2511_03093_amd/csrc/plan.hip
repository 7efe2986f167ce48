// Plan creation (mask validation and bit-plane packing), z-solve constants,
// argument validation and error reporting.
#include <cmath>
#include <cstdio>

#include "common.hpp"

namespace cspnp {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

int fail(int status, const std::string& msg) {
  set_error(msg);
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  set_error(m);
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return CSPNP_ENODEV;
  if (e == hipErrorOutOfMemory) return CSPNP_ENOMEM;
  return CSPNP_EHIP;
}

int check_ptr(const void* p, const char* name) {
  if (p == nullptr) return fail(CSPNP_EINVAL, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) % 4 != 0)
    return fail(CSPNP_EINVAL, std::string(name) + " is not 4-byte aligned");
  return CSPNP_OK;
}

static int validate_desc(const cspnp_desc* d) {
  if (d == nullptr) return fail(CSPNP_EINVAL, "desc is NULL");
  if (d->H < 1 || d->W < 1) return fail(CSPNP_EINVAL, "H and W must be >= 1");
  if (d->R < 1 || d->R > kMaxR) return fail(CSPNP_EINVAL, "R must be in [1, 32]");
  if (d->N < 1) return fail(CSPNP_EINVAL, "N must be >= 1");
  if ((int64_t)d->N * d->R > 1024) return fail(CSPNP_EINVAL, "N*R must be <= 1024");
  if (d->zbc != CSPNP_ZBC_PERIODIC && d->zbc != CSPNP_ZBC_NEUMANN)
    return fail(CSPNP_EINVAL, "zbc must be CSPNP_ZBC_PERIODIC or CSPNP_ZBC_NEUMANN");
  if (d->denoiser != CSPNP_DENOISER_TIKHONOV && d->denoiser != CSPNP_DENOISER_TV &&
      d->denoiser != CSPNP_DENOISER_BM3D)
    return fail(CSPNP_EINVAL, "unknown denoiser");
  if (d->denoiser == CSPNP_DENOISER_BM3D && (d->H < 8 || d->W < 8))
    return fail(CSPNP_EINVAL, "the BM3D denoiser needs H, W >= 8 (8x8 blocks)");
  if ((int64_t)d->H * d->W > (int64_t(1) << 30))
    return fail(CSPNP_EINVAL, "H*W must be <= 2^30");
  return CSPNP_OK;
}

int validate_plan(const cspnp_plan* plan) {
  if (plan == nullptr) return fail(CSPNP_EINVAL, "plan is NULL");
  return CSPNP_OK;
}

int validate_params(const cspnp_plan* plan, const cspnp_params* p) {
  if (p == nullptr) return fail(CSPNP_EINVAL, "params is NULL");
  if (!(std::isfinite(p->rho) && p->rho > 0)) return fail(CSPNP_EINVAL, "rho must be finite and > 0");
  if (!(std::isfinite(p->lambda) && p->lambda >= 0))
    return fail(CSPNP_EINVAL, "lambda must be finite and >= 0");
  if (!(std::isfinite(p->gamma) && p->gamma >= 0))
    return fail(CSPNP_EINVAL, "gamma must be finite and >= 0");
  if (p->iters < 0) return fail(CSPNP_EINVAL, "iters must be >= 0");
  if (plan && plan->desc.denoiser == CSPNP_DENOISER_TV) {
    if (p->tv_inner < 0) return fail(CSPNP_EINVAL, "tv_inner must be >= 0");
    if (!(p->tv_tau > 0 && p->tv_tau <= 0.25)) return fail(CSPNP_EINVAL, "tv_tau must be in (0, 1/4]");
  }
  if (plan && plan->desc.denoiser == CSPNP_DENOISER_BM3D) {
    if (!(std::isfinite(p->bm3d_sigma) && p->bm3d_sigma > 0))
      return fail(CSPNP_EINVAL, "bm3d_sigma must be finite and > 0");
  }
  return CSPNP_OK;
}

ZSolve make_zsolve(int R, int zbc, double rho, double gamma) {
  ZSolve z;
  std::memset(&z, 0, sizeof(z));
  z.rho = rho;
  z.gamma = gamma;
  // T = rho I + gamma L_N: diagonal rho + gamma * (number of chain neighbours)
  double t[kMaxR], dd[kMaxR];
  for (int i = 0; i < R; ++i) {
    int deg = (R == 1) ? 0 : ((i == 0 || i == R - 1) ? 1 : 2);
    t[i] = rho + gamma * deg;
  }
  const double off = -gamma;
  dd[0] = t[0];
  z.l[0] = 0.0;
  for (int i = 1; i < R; ++i) {
    z.l[i] = off / dd[i - 1];
    dd[i] = t[i] - z.l[i] * off;
  }
  for (int i = 0; i < R; ++i) z.invd[i] = 1.0 / dd[i];
  z.periodic = (zbc == CSPNP_ZBC_PERIODIC && R >= 2 && gamma > 0) ? 1 : 0;
  if (z.periodic) {
    double w[kMaxR] = {0};
    w[0] = 1.0;
    w[R - 1] -= 1.0;
    double s[kMaxR];
    s[0] = w[0];
    for (int i = 1; i < R; ++i) s[i] = w[i] - z.l[i] * s[i - 1];
    z.c[R - 1] = s[R - 1] * z.invd[R - 1];
    for (int i = R - 2; i >= 0; --i) z.c[i] = s[i] * z.invd[i] - z.l[i + 1] * z.c[i + 1];
    z.wc = z.c[0] - z.c[R - 1];
  }
  return z;
}

static int ensure_device(int* dev_out) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(CSPNP_ENODEV, "no HIP device is available");
  int dev = 0;
  CSPNP_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  CSPNP_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CSPNP_ENODEV, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  *dev_out = dev;
  return CSPNP_OK;
}

}  // namespace cspnp

using namespace cspnp;

cspnp_plan::~cspnp_plan() {
  graph.clear();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (bits) (void)hipFree(bits);
  if (pmask) (void)hipFree(pmask);
  if (dct) (void)hipFree(dct);
  if (ms_scratch) (void)hipFree(ms_scratch);
}

CSPNP_API int cspnp_version(void) { return CSPNP_VERSION; }

CSPNP_API const char* cspnp_status_string(int s) {
  switch (s) {
    case CSPNP_OK: return "CSPNP_OK";
    case CSPNP_EINVAL: return "CSPNP_EINVAL: invalid argument";
    case CSPNP_ENOMEM: return "CSPNP_ENOMEM: out of memory";
    case CSPNP_EHIP: return "CSPNP_EHIP: HIP runtime error";
    case CSPNP_ENODEV: return "CSPNP_ENODEV: no usable gfx950 device";
    case CSPNP_EUNSUPPORTED: return "CSPNP_EUNSUPPORTED: not implemented";
    case CSPNP_ENONFINITE: return "CSPNP_ENONFINITE: non-finite value";
    default: return "unknown cspnp status";
  }
}

CSPNP_API const char* cspnp_last_error(void) { return g_last_error.c_str(); }

CSPNP_API int cspnp_plan_create(const cspnp_desc* desc, const uint8_t* masks, int masks_on_device,
                                void* stream, cspnp_plan** out) {
  clear_error();
  if (int s = validate_desc(desc)) return s;
  if (masks == nullptr) return fail(CSPNP_EINVAL, "masks is NULL");
  if (out == nullptr) return fail(CSPNP_EINVAL, "out is NULL");
  const int H = desc->H, W = desc->W, R = desc->R;
  const size_t nmask = (size_t)R * H * W;
  std::vector<uint8_t> host;
  const uint8_t* m = masks;
  int dev = 0;
  if (masks_on_device) {
    if (int s = ensure_device(&dev)) return s;
    host.resize(nmask);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CSPNP_HIP(hipMemcpyAsync(host.data(), masks, nmask, hipMemcpyDeviceToHost, st));
    CSPNP_HIP(hipStreamSynchronize(st));
    m = host.data();
  }
  // validate every byte before touching the device (host masks)
  for (size_t i = 0; i < nmask; ++i)
    if (m[i] > 1) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "mask byte %zu is %u; masks must be 0 or 1", i, (unsigned)m[i]);
      return fail(CSPNP_EINVAL, buf);
    }
  if (!masks_on_device)
    if (int s = ensure_device(&dev)) return s;
  const int Wq = (W + 31) / 32;
  std::vector<uint32_t> packed((size_t)R * H * Wq, 0u);
  for (int r = 0; r < R; ++r)
    for (int h = 0; h < H; ++h) {
      const uint8_t* row = m + ((size_t)r * H + h) * W;
      uint32_t* prow = packed.data() + ((size_t)r * H + h) * Wq;
      for (int w = 0; w < W; ++w) prow[w >> 5] |= uint32_t(row[w]) << (w & 31);
    }
  std::unique_ptr<cspnp_plan> plan(new cspnp_plan());
  plan->desc = *desc;
  plan->device = dev;
  plan->Wq = Wq;
  plan->tv_shape = tv_default_shape(H, W, desc->N * R, 10);
  plan->xu_block = 0;
  CSPNP_HIP(hipMalloc(&plan->bits, packed.size() * sizeof(uint32_t)));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  CSPNP_HIP(hipMemcpyAsync(plan->bits, packed.data(), packed.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, st));
  std::vector<uint16_t> pm16;
  std::vector<uint32_t> pm32;
  if (desc->N == 1) {
    const size_t HW = (size_t)H * W;
    if (R <= 16) pm16.assign(HW, 0); else pm32.assign(HW, 0u);
    for (int r = 0; r < R; ++r) {
      const uint8_t* mr = m + (size_t)r * HW;
      for (size_t i = 0; i < HW; ++i) {
        if (R <= 16) pm16[i] |= (uint16_t)(mr[i] << r);
        else pm32[i] |= uint32_t(mr[i]) << r;
      }
    }
    const size_t nb = R <= 16 ? HW * sizeof(uint16_t) : HW * sizeof(uint32_t);
    CSPNP_HIP(hipMalloc(&plan->pmask, nb));
    CSPNP_HIP(hipMemcpyAsync(plan->pmask, R <= 16 ? (const void*)pm16.data() : (const void*)pm32.data(), nb,
                             hipMemcpyHostToDevice, st));
  }
  if (desc->N > 1) CSPNP_HIP(hipMalloc(&plan->ms_scratch, multishot_scratch_bytes(*desc)));
  if (desc->denoiser == CSPNP_DENOISER_BM3D) {
    double c[64];
    make_dct_matrix(c);
    CSPNP_HIP(hipMalloc(&plan->dct, sizeof c));
    CSPNP_HIP(hipMemcpyAsync(plan->dct, c, sizeof c, hipMemcpyHostToDevice, st));
  }
  CSPNP_HIP(hipStreamSynchronize(st));
  CSPNP_HIP(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
  *out = plan.release();
  return CSPNP_OK;
}

CSPNP_API int cspnp_plan_destroy(cspnp_plan* plan) {
  clear_error();
  delete plan;
  return CSPNP_OK;
}

CSPNP_API int cspnp_plan_desc(const cspnp_plan* plan, cspnp_desc* out) {
  clear_error();
  if (int s = validate_plan(plan)) return s;
  if (out == nullptr) return fail(CSPNP_EINVAL, "out is NULL");
  *out = plan->desc;
  return CSPNP_OK;
}
