/*
 * cspnp -- plug-and-play ADMM reconstruction of a light-sheet z-stack from
 * DMD-coded snapshots, on AMD Instinct MI355X (gfx950).
 *
 * Problem (arXiv 2511.03093, Sec. III-A, eq. (model-slice); Sec. III-C):
 *   data b_j (j = 1..N shots, H x W pixels each) and R binary masks phi_r
 *   shared by every shot; unknown slices v_n, n = 1..N*R, with
 *   b_j = sum_r phi_r (.) v_{(j-1)R+r}.  The library minimises
 *     1/2 sum_j ||b_j - sum_r phi_r v_{(j-1)R+r}||^2 + lambda sum_n psi(v_n)
 *       + gamma/2 sum_{adjacent n} ||v_n - v_{n-1}||^2
 *   by ADMM with the splitting v = u and scaled dual d (eq. (ADMM)),
 *   Algorithm 1's loop: x-step, u-step (a plug-in denoiser), d-step.
 *
 * Memory layout (all row-major, contiguous, FP32 unless stated):
 *   volume  x, u, d, f : float[N*R][H][W]   (slice n = (j-1)R + r, 0-based j*R+r)
 *   frames  y          : float[N][H][W]
 *   masks   (input)    : uint8[R][H][W], values 0 or 1
 * Device pointers are HIP device (or managed) memory owned by the caller and
 * must stay alive until the stream has finished the enqueued work.  Float
 * pointers must be 4-byte aligned.  `stream` is a hipStream_t (NULL = the
 * default stream).  All compute calls are asynchronous on `stream`.
 *
 * Errors: every call returns a cspnp_status.  Arguments are validated on the
 * host before anything is enqueued; on error nothing is enqueued and
 * cspnp_last_error() gives a thread-local description.  A device fault
 * surfaces as CSPNP_EHIP from a later call.  The ABI never throws.
 *
 * Thread safety: distinct plans may be used concurrently; one plan must be
 * used by one host thread / stream at a time (it caches launch graphs).
 */
#ifndef CSPNP_H
#define CSPNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSPNP_VERSION 1

typedef enum cspnp_status {
  CSPNP_OK = 0,
  CSPNP_EINVAL = 1,       /* invalid argument (null/misaligned pointer, bad shape or parameter) */
  CSPNP_ENOMEM = 2,       /* host or device allocation failed */
  CSPNP_EHIP = 3,         /* a HIP runtime call failed (includes earlier asynchronous faults) */
  CSPNP_ENODEV = 4,       /* no usable gfx950 device */
  CSPNP_EUNSUPPORTED = 5, /* valid request this build does not implement (e.g. the backward with N > 1) */
  CSPNP_ENONFINITE = 6    /* non-finite value detected (only with CSPNP_FLAG_CHECK_FINITE) */
} cspnp_status;

/* z boundary of the temporal term.  PERIODIC is the paper's wrap
 * (Sec. III-C: u_0 = u_{NR}, u_{NR+1} = u_1), each adjacent pair counted once;
 * NEUMANN drops the wrap pair (free ends). */
enum { CSPNP_ZBC_PERIODIC = 0, CSPNP_ZBC_NEUMANN = 1 };

/* u-step denoisers (Sec. III-B, eq. (u-sub)). */
enum { CSPNP_DENOISER_TIKHONOV = 0, CSPNP_DENOISER_TV = 1, CSPNP_DENOISER_BM3D = 2 };

/* cspnp_params.flags */
enum {
  CSPNP_FLAG_NO_GRAPH = 1,     /* launch kernels one by one instead of replaying a captured graph */
  CSPNP_FLAG_CHECK_FINITE = 2, /* after a solve, synchronise and fail with ENONFINITE on NaN/Inf in x */
  /* cspnp_solve runs Algorithm 1's own schedule: the v-step without the temporal
   * term (eq. (v-update)), then one Gauss-Seidel sweep over the slices of
   * eq. (u-update) (datum (rho (v_n + d_n) + gamma (u_{n-1} + u_{n+1})) / (rho + 2 gamma),
   * strength lambda / (rho + 2 gamma), newest neighbour values, periodic wrap or
   * free ends), then d = d + v - u.  x returns v.  TV and Tikhonov denoisers. */
  CSPNP_FLAG_PAPER_SCHEDULE = 4
};

/* workspace modes for cspnp_workspace_size */
enum { CSPNP_WS_SOLVE = 0, CSPNP_WS_DENOISE = 1, CSPNP_WS_SOLVE_TOL = 2 };

/* Problem shape: H x W pixels, R masks/slices per shot, N shots (Sec. III-A). */
typedef struct cspnp_desc {
  int32_t H, W;
  int32_t R;        /* compression ratio, 1..32 */
  int32_t N;        /* shots per volume, N*R <= 1024 (N > 1: not batched; the x-step then
                       uses an FP64 scratch volume the plan owns, so calls on one such
                       plan must not overlap) */
  int32_t zbc;      /* CSPNP_ZBC_* */
  int32_t denoiser; /* CSPNP_DENOISER_* */
} cspnp_desc;

/* Algorithm 1's parameters (lambda, rho, gamma), the iteration count, and the
 * TV dual-projection settings (Chambolle's step tau <= 1/4; 1/8 is the proven
 * bound).  lambda >= 0, rho > 0, gamma >= 0, iters >= 0, tv_inner >= 0. */
typedef struct cspnp_params {
  double lambda;
  double rho;
  double gamma;
  int32_t iters;
  int32_t tv_inner;
  double tv_tau;
  double bm3d_sigma;
  int32_t flags;
} cspnp_params;

typedef struct cspnp_plan cspnp_plan;

/* Library ABI version (CSPNP_VERSION). */
int cspnp_version(void);
/* Static text for a status code. */
const char* cspnp_status_string(int status);
/* Thread-local detail of the last failed call on this thread ("" if none). */
const char* cspnp_last_error(void);

/* Create a plan for one problem shape and one mask set (Algorithm 1's
 * "Require" inputs: the masks phi_r and the shape).  `masks` is
 * uint8[R][H][W] with values in {0,1}, in host memory (masks_on_device = 0)
 * or device memory (1).  The plan validates every byte (EINVAL otherwise),
 * packs the masks into device bit-planes uint32[R][H][ceil(W/32)] (bit w%32
 * of word w/32), and owns them.  The call is synchronous.  *out receives the
 * plan on success and is untouched on error. */
int cspnp_plan_create(const cspnp_desc* desc, const uint8_t* masks, int masks_on_device,
                      void* stream, cspnp_plan** out);
/* Free a plan and everything it owns.  NULL is accepted. */
int cspnp_plan_destroy(cspnp_plan* plan);
/* The plan's shape. */
int cspnp_plan_desc(const cspnp_plan* plan, cspnp_desc* out);

/* Device workspace bytes that cspnp_solve (mode CSPNP_WS_SOLVE) or
 * cspnp_denoise (CSPNP_WS_DENOISE) needs for these parameters.  The caller
 * allocates it (256-byte aligned) and passes it as `ws`; it may be NULL when
 * the size is 0. */
int cspnp_workspace_size(const cspnp_plan* plan, const cspnp_params* params, int mode,
                         size_t* bytes);

/* Forward operator, Sec. III-A / eq. (model-slice):
 *   y[j][p] = sum_r phi_r[p] * x[j*R + r][p].
 * x: float[N*R][H][W] (device, read), y: float[N][H][W] (device, written). */
int cspnp_forward(const cspnp_plan* plan, const float* x, float* y, void* stream);

/* Adjoint operator (the Phi^T b of eq. (v-update)):
 *   x[j*R + r][p] = phi_r[p] * y[j][p].
 * y: float[N][H][W] (device, read), x: float[N*R][H][W] (device, written). */
int cspnp_adjoint(const cspnp_plan* plan, const float* y, float* x, void* stream);

/* x-step (eq. (v-update), with the temporal term of Sec. III-C carried by
 * the x-block): for every pixel p solve the N*R x N*R system
 *   (M_p^T M_p + gamma L + rho I) x_p = M_p^T y_p + rho (u_p - d_p)
 * with L the periodic or Neumann z-Laplacian, in FP64 registers (FP32 I/O).
 * y: frames; u, d: volumes (read).  x_out (may be NULL) receives x, f_out (may
 * be NULL) receives f = x + d, the datum of the next u-step.  At least one of
 * them must be non-NULL.  Neither output may alias an input. */
int cspnp_xupdate(const cspnp_plan* plan, const cspnp_params* params, const float* y,
                  const float* u, const float* d, float* x_out, float* f_out, void* stream);

/* u-step and d-step (eq. (u-sub) and the third line of eq. (ADMM)): every
 * slice of f is denoised independently,
 *   u = prox_{(lambda/rho) psi}(f),   d_out = f - u   (d_out may be NULL),
 * with the plan's denoiser: Tikhonov u = rho f / (2 lambda + rho); TV by
 * params->tv_inner iterations of Chambolle's dual projection with step
 * params->tv_tau from p = 0 (theta = lambda/rho).  f, u, d_out: volumes;
 * u and d_out must not alias f.  ws: cspnp_workspace_size(CSPNP_WS_DENOISE). */
int cspnp_denoise(const cspnp_plan* plan, const cspnp_params* params, const float* f, float* u,
                  float* d_out, void* ws, void* stream);

/* Algorithm 1: params->iters ADMM iterations from the caller's (u, d)
 * (zero them for a cold start; pass a previous state to resume exactly).
 * On return (stream-ordered) x holds the last x-step result, u and d the
 * final auxiliary and dual variables.  y: frames (read); u, d: volumes
 * (read-write); x: volume (written; untouched when iters = 0).
 * ws: cspnp_workspace_size(CSPNP_WS_SOLVE) bytes.  The first call with a
 * given (parameters, pointers) captures the iteration loop into a HIP graph
 * that later identical calls replay. */
int cspnp_solve(const cspnp_plan* plan, const cspnp_params* params, const float* y, float* u,
                float* d, float* x, void* ws, void* stream);

/* Algorithm 1 with a stopping rule (Sec. IV-B caps the iterations and uses a
 * relative tolerance it does not define; read here as
 * ||x^{k+1} - x^k|| / ||x^k|| < tol): at most params->iters iterations, the
 * relative change of consecutive x-steps tested every check_every iterations
 * (one host synchronisation per test).  *iters_done receives the iterations
 * run, *last_rel the last tested change (-1 if none).  Synchronous.
 * ws: cspnp_workspace_size(CSPNP_WS_SOLVE_TOL) bytes. */
int cspnp_solve_tol(const cspnp_plan* plan, const cspnp_params* params, double tol, int check_every,
                    const float* y, float* u, float* d, float* x, void* ws, void* stream, int32_t* iters_done,
                    double* last_rel);

/* ---- quality metrics (Sec. IV) --------------------------------------------
 * PSNR = 10 log10(n peak^2 / ||est - ref||^2) over n elements (3D: all voxels
 * as one array).  SSIM: window-weighted local statistics with an 11-tap
 * Gaussian (standard deviation 1.5, normalised) along W and H (dims = 2, per
 * slice) or W, H and D (dims = 3), c1 = (0.01 L)^2, c2 = (0.03 L)^2, averaged
 * over all positions where the window lies inside the data (needs H, W >= 11,
 * and D >= 11 for dims = 3).  cspnp_rel_change = ||a - b|| / ||b||.  Inputs are
 * device float arrays ([D][H][W] for SSIM); `out` is one device double,
 * written asynchronously; ws: cspnp_metrics_workspace_size(D, H, W, dims)
 * bytes (dims = 0 for PSNR and the relative change), 256-byte aligned. */
int cspnp_metrics_workspace_size(int32_t D, int32_t H, int32_t W, int32_t dims, size_t* bytes);
int cspnp_psnr(const float* est, const float* ref, size_t n, double peak, double* out, void* ws, void* stream);
int cspnp_ssim(const float* est, const float* ref, int32_t D, int32_t H, int32_t W, int32_t dims, double L,
               double* out, void* ws, void* stream);
int cspnp_rel_change(const float* a, const float* b, size_t n, double* out, void* ws, void* stream);

/* ---- BM3D stage inspection ------------------------------------------------
 * The BM3D u-step (plan denoiser CSPNP_DENOISER_BM3D, params->bm3d_sigma the
 * noise level) runs inside cspnp_denoise / cspnp_solve.  These calls expose
 * its intermediate results for verification: cspnp_bm3d_stage runs the
 * stage-1 block matching on f (stage 0), additionally the hard-threshold
 * stage producing the FP64 basic estimate (stage 1), or additionally the
 * stage-2 matching on the basic estimate (stage 2), into ws (the
 * CSPNP_WS_DENOISE workspace).  cspnp_bm3d_layout gives the byte offsets in
 * ws of the match lists int32[N*R][nry][nrx][16] (raster index y*W + x of
 * each block, reference first), of the group sizes int32[N*R][nry][nrx] and
 * of the basic estimate double[N*R][H][W], and the reference-grid size
 * (references at rows 0, 3, 6, ... and H-8; columns likewise). */
int cspnp_bm3d_stage(const cspnp_plan* plan, const cspnp_params* params, const float* f, int stage, void* ws,
                     void* stream);
int cspnp_bm3d_layout(const cspnp_plan* plan, size_t* matches_offset, size_t* counts_offset,
                      size_t* basic_offset, int32_t* nry, int32_t* nrx);

/* ---- differentiable solve (reverse mode through the unrolled iterations) --
 * Gradients of <x_bar, x^K>, x^K the last x-step of params->iters iterations
 * started from u = d = 0, with respect to the frames y and the scalars
 * rho, lambda, gamma.  (The paper defines no gradient: this differentiates the
 * iteration this library runs.)  TV (tv_inner <= 16) and Tikhonov denoisers,
 * any number of shots N (N > 1 uses the plan's block-elimination scratch, so
 * calls on such a plan must not overlap).
 * Other denoisers: CSPNP_EUNSUPPORTED. */

/* Bytes of the checkpoint buffer: ceil(iters/ckpt_every) x (u, d) volumes. */
int cspnp_ckpt_size(const cspnp_plan* plan, const cspnp_params* params, int ckpt_every, size_t* bytes);
/* Device workspace bytes of cspnp_solve_bwd (256-byte aligned by the caller). */
int cspnp_bwd_workspace_size(const cspnp_plan* plan, const cspnp_params* params, int ckpt_every,
                             size_t* bytes);
/* cspnp_solve from the caller's (u, d) (zero for the differentiable start),
 * storing (u, d) at iterations 0, ckpt_every, 2 ckpt_every, ... into ckpt
 * (float[ceil(iters/ckpt_every)][2][N*R][H][W], device).  ws as for cspnp_solve.
 * Launches kernels directly (no graph capture). */
int cspnp_solve_ckpt(const cspnp_plan* plan, const cspnp_params* params, const float* y, float* u,
                     float* d, float* x, int ckpt_every, float* ckpt, void* ws, void* stream);
/* Reverse pass: recomputes each segment from ckpt (as written by
 * cspnp_solve_ckpt with the same params and y) and accumulates
 *   y_bar (float[N][H][W], overwritten)  and
 *   param_bar (device double[3], overwritten) = d<x_bar,x^K>/d(rho, lambda, gamma).
 * x_bar: volume (read).  Deterministic (fixed-order FP64 reductions).
 * Captured into a HIP graph on the first call for a given (params,
 * ckpt_every, pointers) and replayed by later identical calls (the plan's
 * graph cache, shared with cspnp_solve); CSPNP_FLAG_NO_GRAPH launches
 * directly. */
int cspnp_solve_bwd(const cspnp_plan* plan, const cspnp_params* params, const float* y, int ckpt_every,
                    const float* ckpt, const float* x_bar, float* y_bar, double* param_bar, void* ws,
                    void* stream);

/* ---- batched solves ------------------------------------------------------
 * Many independent snapshots (each its own shape H x W x R, N = 1, masks and
 * parameters; TV denoiser) reconstructed by one graph of persistent grouped
 * launches: per ADMM iteration one x-update launch per distinct R and one TV
 * launch over all (problem, slice, tile).  Results equal the per-problem
 * cspnp_solve bit for bit. */
typedef struct cspnp_batch cspnp_batch;

/* n problems; descs[i] as for cspnp_plan_create (denoiser must be TV);
 * masks[i]: host uint8[R_i][H_i][W_i] in {0,1}.  Synchronous. */
int cspnp_batch_create(int32_t n, const cspnp_desc* descs, const uint8_t* const* masks, void* stream,
                       cspnp_batch** out);
int cspnp_batch_destroy(cspnp_batch* batch);
/* Device workspace bytes of cspnp_batch_solve (one f volume per problem). */
int cspnp_batch_workspace_size(const cspnp_batch* batch, size_t* bytes);
/* params[i] per problem (all with the same iters; tv_inner <= 16); y, u, d, x:
 * host arrays of n device pointers with the per-problem layouts of
 * cspnp_solve (u, d in/out, x out).  ws: 256-byte aligned workspace.  The
 * first call for a given (params, pointers, ws) uploads the problem tables
 * (synchronising the stream once) and captures the graph; later identical
 * calls replay it.  Flag CSPNP_FLAG_NO_GRAPH (params[0].flags) launches
 * directly. */
int cspnp_batch_solve(cspnp_batch* batch, const cspnp_params* params, const float* const* y, float* const* u,
                      float* const* d, float* const* x, void* ws, void* stream);
/* TV tile shape (index into the same table as cspnp_tv_shape_info) of the
 * grouped TV launch. */
int cspnp_batch_set_tv_shape(cspnp_batch* batch, int32_t shape);
int cspnp_batch_get_tv_shape(const cspnp_batch* batch, int32_t* shape);
/* Time every TV tile shape on the grouped launch (HIP events on `stream`,
 * synchronous) and keep the fastest.  Uses the given buffers as scratch:
 * u, d and ws are overwritten. */
int cspnp_batch_autotune(cspnp_batch* batch, const cspnp_params* params, const float* const* y,
                         float* const* u, float* const* d, float* const* x, void* ws, void* stream);

/* ---- launch-shape tuning ------------------------------------------------ */

/* A plan's launch shapes: an index into the TV tile-shape table and into the
 * x-update block-shape table.  Shapes change only speed, never results
 * beyond FP32 rounding order (the TV result is identical: every pixel's
 * arithmetic is the same whatever the tile). */
typedef struct cspnp_tuning {
  int32_t tv_shape;
  int32_t xu_block;
} cspnp_tuning;

/* Number of TV tile shapes and x-update block shapes. */
int cspnp_tuning_candidates(int32_t* n_tv_shapes, int32_t* n_xu_blocks);
/* Tile size (pixels) and workgroup size of TV shape `index`. */
int cspnp_tv_shape_info(int32_t index, int32_t* tile_cols, int32_t* tile_rows, int32_t* threads);
/* Read / set a plan's shapes (EINVAL for an index out of range).  Setting
 * drops the plan's cached solve graph. */
int cspnp_plan_get_tuning(const cspnp_plan* plan, cspnp_tuning* out);
int cspnp_plan_set_tuning(cspnp_plan* plan, const cspnp_tuning* tuning);
/* Choose the plan's shapes by timing every candidate with HIP events on
 * `stream` for these parameters (synchronous; allocates and frees scratch
 * volumes).  With cache_path != NULL a JSON file keyed by (device arch, H, W,
 * R, N, z boundary, denoiser, TV inner count) is read first (unless force is
 * non-zero) and updated afterwards. */
int cspnp_autotune(cspnp_plan* plan, const cspnp_params* params, const char* cache_path, int force,
                   void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CSPNP_H */
