/*
 * eecmg.h -- C ABI of the MI355X (gfx950) implementation of the extrapolation
 * economy cascadic multigrid (EECMG) image restoration method of Chu, Yan and
 * Li, "A New Extrapolation Economy Cascadic Multigrid Method for Image
 * Restoration Problems" (arXiv 2311.03010).
 *
 * Problem (Section 1, eq. 1-3, 7-9): restore u from g_delta = H u + e, where H
 * is the 2-D convolution with a point-spread function (PSF) under zero
 * boundary conditions and e is additive noise.  The cascade (Algorithm 2)
 * solves H_l u_l = g_l on nested grids from coarse to fine (Section 2,
 * eq. 11-14), smoothing each level with a CG-type iteration C_l^{m_l}, and
 * carries each result to the next level with the new extrapolation Pi and the
 * quadratic interpolation P (Section 3.2), the local weighted least-squares
 * smoothing S (Section 3.3, eq. 18-19) and the Perona-Malik denoising step D
 * (Section 4, eq. 20-26).
 *
 * Conventions for every entry point
 *   - Return value: an eecmg_status (0 = OK).  Outputs go through out-pointers
 *     only; nothing throws across the ABI.  On a non-OK status,
 *     eecmg_last_error() returns a thread-local message.
 *   - Images are dense row-major H x W arrays (H rows, W columns, no padding),
 *     each below 4 GiB (EINVAL otherwise: kernels index with 32-bit offsets);
 *     element type double when params->precision == EECMG_FP64, float otherwise.
 *     H and W are image sizes, not the blur operator.
 *   - PSF: (2r+1) x (2r+1) doubles, row-major, psf[(a+r)*(2r+1)+(b+r)] is the
 *     weight at offset (a, b): (H x)(i,j) = sum_{a,b} psf(a,b) x(i-a, j-b).
 *     The PSF is always given in FP64 on the host and copied by the call.
 *   - Levels: n_levels >= 1; level sizes halve per axis with rounding up
 *     (n_{l-1} = ceil(n_l / 2), Section 2), and every level must keep at
 *     least 3 nodes per axis.  iters_per_level: n_levels ints, coarsest first,
 *     each >= 0, the caps m_l; NULL selects the paper's economic rule
 *     (Section 2, after Algorithm 2).
 *   - k: the Perona-Malik threshold of eq. (6)/(21), > 0.
 *   - Host-pointer calls copy inputs before doing any work and write outputs
 *     only on EECMG_OK.  Device-pointer calls (_dev) take pointers to device
 *     memory on the current HIP device and a hipStream_t (NULL = default
 *     stream).  The restore calls run the cascade on that stream and return
 *     when it has completed (the level schedule follows the device's progress
 *     words, so it cannot run ahead of the device); output and stats are then
 *     final.  The single-operator calls (eecmg_op_*_dev) return once their
 *     kernels are enqueued and the caller synchronises the stream before
 *     reading the output.  The caller owns every buffer it passes and keeps
 *     device buffers alive until the work is complete.
 *   - Thread safety: every function may be called from any thread; calls that
 *     share a context or the process-wide plain-restore engine are serialised
 *     internally.
 */
#ifndef EECMG_H
#define EECMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EECMG_MAX_LEVELS 16
#define EECMG_MAX_RADIUS 12

typedef enum {
  EECMG_OK = 0,
  EECMG_PENDING = 1,     /* request not finished yet (eecmg_poll) */
  EECMG_EINVAL = -1,     /* invalid argument */
  EECMG_ENOMEM = -2,     /* device or host memory exhausted / over budget */
  EECMG_EAGAIN = -3,     /* queue full, try again later */
  EECMG_EDEVICE = -4,    /* HIP runtime error or HIP library missing */
  EECMG_ENOTFOUND = -5,  /* unknown request id */
  EECMG_ENUMERIC = -6,   /* non-finite value met in the smoother */
  EECMG_ECANCELED = -7   /* request was cancelled */
} eecmg_status;

typedef enum {
  EECMG_FP64 = 0,            /* all arithmetic and storage in FP64 */
  EECMG_FP32 = 1,            /* FP32 storage and stencils; FP64 inner products, scalars, extrapolation differences */
  EECMG_FP32_FP16COARSE = 2  /* refused (EINVAL): FP16 storage of coarse levels keeps the FP32 error bar
                                (relative L2 1e-4 against FP64) only on levels of at most 128^2 pixels,
                                whose time is launch latency, so it would add error and save nothing */
} eecmg_precision;

typedef enum {
  EECMG_CASCADE_EECMG = 0,   /* Algorithm 2: new extrapolation + quadratic interpolation */
  EECMG_CASCADE_IECMG_L = 1, /* Algorithm 1 with the linear prolongation of eq. (15) */
  EECMG_CASCADE_IECMG_P = 2  /* Algorithm 1 with the quadratic interpolation of Section 3.2 */
} eecmg_cascade;

typedef enum {
  EECMG_SMOOTHER_CGLS = 0, /* CG on the normal equations (the paper's "CG") */
  EECMG_SMOOTHER_MR = 1    /* minimal-residual iteration (the paper's "MR") */
} eecmg_smoother;

typedef enum {
  EECMG_STOP_NONE = 0,
  EECMG_STOP_DISCREPANCY = 1, /* ||g_l - H_l u|| <= c delta (Section 2 stopping rule, RMS norm of eq. 10) */
  EECMG_STOP_CAP = 2,         /* m_l iterations done */
  EECMG_STOP_GUARD = 3,       /* converged to rounding (gradient or residual vanished) */
  EECMG_STOP_NONFINITE = 4    /* a non-finite inner product was met */
} eecmg_stop_reason;

/* Per-call parameters.  Fill with eecmg_params_default() and override. */
typedef struct {
  uint32_t struct_size;     /* sizeof(eecmg_params) */
  int32_t precision;        /* eecmg_precision; default EECMG_FP32 */
  int32_t stop_rule;        /* 1: discrepancy principle on every level (Section 2); default 1 */
  double delta;             /* noise level ||e|| in the RMS norm of eq. (10), >= 0; default 1 */
  double c;                 /* discrepancy constant, > 1 when stop_rule = 1; default 1.1 */
  double tau;               /* explicit Perona-Malik step (eq. 25), 0 < tau <= 1/4; default 0.2 */
  int32_t pm_steps;         /* number of D steps per transfer, >= 0; default 1 */
  double smooth_h;          /* scale h of the S weights exp(-((u_c - u_n)/h)^2), > 0; default 1 */
  int32_t coarse_psf_mode;  /* scale of R H R^*: 0 sum-preserving, 1 x4, 2 x1; default 0 */
  double guard_eps;         /* convergence guard epsilon (>= 0); 0 = 1e-14 (FP64) or 1e-6 (FP32) */
  int32_t smoother;         /* eecmg_smoother; default CGLS */
  int32_t cascade;          /* eecmg_cascade; default EECMG */
  void* stats;              /* optional eecmg_stats* written on OK; NULL = none */
} eecmg_params;

/* Per-level record of a restore (coarsest level first). */
typedef struct {
  uint32_t struct_size;                   /* sizeof(eecmg_stats) */
  int32_t n_levels;
  int32_t level_h[EECMG_MAX_LEVELS];
  int32_t level_w[EECMG_MAX_LEVELS];
  int32_t psf_radius[EECMG_MAX_LEVELS];
  int32_t caps[EECMG_MAX_LEVELS];
  int32_t iters[EECMG_MAX_LEVELS];        /* smoother iterations run */
  int32_t stop_reason[EECMG_MAX_LEVELS];  /* eecmg_stop_reason */
  double final_rms[EECMG_MAX_LEVELS];     /* ||g_l - H_l u_l|| (eq. 10) when the smoother stopped */
} eecmg_stats;

/* Fill *p with the defaults listed above.  EINVAL if p is NULL. */
int eecmg_params_default(eecmg_params* p);

/* Restore one image, host buffers (Algorithm 2, or Algorithm 1 per
 * params->cascade).  g_delta: H x W input; u_out: H x W output; both of the
 * element type selected by params->precision.  params NULL = defaults.
 * Errors: EINVAL (sizes, levels, radius > EECMG_MAX_RADIUS, parameters),
 * ENOMEM, EDEVICE, ENUMERIC (non-finite input or divergence). */
int eecmg_restore(const void* g_delta, int H, int W, const double* psf, int psf_radius, int n_levels,
                  const int* iters_per_level, double k, const eecmg_params* params, void* u_out);

/* As eecmg_restore with device-resident g_delta_dev / u_out_dev (dense H x W)
 * enqueued on hip_stream.  Statistics (params->stats) are complete on return.
 * When a row of H x W is a multiple of 256 bytes and the two buffers are
 * 256-byte aligned and disjoint, the finest level reads g_delta_dev and
 * updates u_out_dev in place (no copies); u_out_dev may be the same buffer as
 * g_delta_dev.  On an error status the contents of u_out_dev are unspecified.
 * Additional error: EINVAL if a pointer is not device memory. */
int eecmg_restore_dev(const void* g_delta_dev, int H, int W, const double* psf, int psf_radius, int n_levels,
                      const int* iters_per_level, double k, const eecmg_params* params, void* u_out_dev,
                      void* hip_stream);

/* As eecmg_restore_dev, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): the call allocates
 * no device or pinned memory.  It works in a fixed device region of 64 MiB
 * that the library reserves per GPU (a device global, held until the process
 * ends) and that also holds its own engine's tables; the first call on a
 * device sets that engine up (the region's address, HIP events, host
 * tables).  A restore whose device footprint (about 9.7 times the finest
 * level's bytes: FP32 images up to about 1300 x 1300, FP64 up to about
 * 900 x 900) exceeds the region returns EINVAL and does nothing.  Calls on one
 * GPU share the region and are serialised (every call returns only after its
 * cascade completed); each call clears the solver state it reads, and the
 * region otherwise keeps the previous call's bytes.  Results and statistics
 * are bit for bit those of eecmg_restore_dev.  The level schedule follows the
 * device's progress by draining the stream (slower on levels with many
 * iterations); kernel timing (eecmg_profile_*) does not cover this call. */
int eecmg_restore_dev_noalloc(const void* g_delta_dev, int H, int W, const double* psf, int psf_radius,
                              int n_levels, const int* iters_per_level, double k, const eecmg_params* params,
                              void* u_out_dev, void* hip_stream);

/* Restore n_images independent images of possibly different sizes, PSFs and
 * level counts in one batched cascade: all images at a smoother or transfer
 * stage share each kernel launch.  Arrays are indexed by image; params is an
 * array of n_images (NULL = defaults for all), iters_per_level may be NULL
 * (rule for all) or hold NULL entries.  Every image's result equals its
 * eecmg_restore_dev result bit for bit.  All images must share one precision.
 * Returns the first failing image's status; results of other images are
 * still written. */
int eecmg_restore_batch_dev(int n_images, const void* const* g_delta_dev, const int* H, const int* W,
                            const double* const* psf, const int* psf_radius, const int* n_levels,
                            const int* const* iters_per_level, const double* k, const eecmg_params* params,
                            void* const* u_out_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Request loop with continuous batching.  A context owns a device memory
 * budget and a progress thread; submitted requests are admitted when their
 * device footprint fits the budget and a slot is free, and then advance in
 * the same kernel launches as every other admitted request.
 * ------------------------------------------------------------------------- */
typedef struct eecmg_ctx eecmg_ctx;

typedef struct {
  uint32_t struct_size;     /* sizeof(eecmg_ctx_config) */
  int32_t device;           /* HIP device ordinal; default 0 */
  size_t hbm_budget_bytes;  /* device memory the context may use; default 8 GiB */
  int32_t max_slots;        /* admitted requests at once, 1..EECMG_MAX_SLOTS; default 64 */
  int32_t max_queue;        /* submitted but not admitted, >= 1; default 4096 */
} eecmg_ctx_config;

#define EECMG_MAX_SLOTS 240

int eecmg_ctx_config_default(eecmg_ctx_config* cfg);
/* Create a context (allocates the budget up front).  EINVAL, ENOMEM, EDEVICE. */
int eecmg_create(const eecmg_ctx_config* cfg, eecmg_ctx** out);
/* Queue one restore; arguments as eecmg_restore (host buffers, copied before
 * return).  EAGAIN when the queue is full; ENOMEM when the request can never
 * fit the budget. */
int eecmg_submit(eecmg_ctx* ctx, const void* g_delta, int H, int W, const double* psf, int psf_radius,
                 int n_levels, const int* iters_per_level, double k, const eecmg_params* params,
                 uint64_t* request_id);
/* PENDING while running; on completion copies u (H x W) into u_out and the
 * statistics into stats_out (may be NULL), forgets the request and returns
 * its status.  ENOTFOUND for unknown or already collected ids. */
int eecmg_poll(eecmg_ctx* ctx, uint64_t request_id, void* u_out, eecmg_stats* stats_out);
/* As eecmg_poll but blocks until the request finishes. */
int eecmg_wait(eecmg_ctx* ctx, uint64_t request_id, void* u_out, eecmg_stats* stats_out);
/* Cancel a queued or running request; its poll then returns ECANCELED. */
int eecmg_cancel(eecmg_ctx* ctx, uint64_t request_id);
/* Requests queued / admitted right now, and device bytes in use. */
int eecmg_ctx_info(eecmg_ctx* ctx, int* queued, int* active, size_t* bytes_in_use);
/* Wait for in-flight work, free every device allocation, destroy. */
int eecmg_destroy(eecmg_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Operator entry points: the cascade's building blocks, one level each, on
 * dense device buffers (element type by precision) enqueued on hip_stream.
 * ------------------------------------------------------------------------- */

/* y = H x (transpose = 0) or y = H^T x (transpose = 1), zero boundary
 * (eq. 1, 9; Section 5).  x, y: H x W, must not alias. */
int eecmg_op_conv_dev(const void* x_dev, void* y_dev, int H, int W, const double* psf, int psf_radius,
                      int transpose, int precision, void* hip_stream);
/* One level of the smoother C_l^{m_l} (Section 2): u_dev holds u0 on entry and
 * the result on exit; g_dev the level's right-hand side.  params selects the
 * smoother, stopping rule and guard; stats_out (may be NULL) receives
 * iters[0], stop_reason[0] and final_rms[0]. Synchronous. */
int eecmg_op_smoother_dev(const void* g_dev, void* u_dev, int H, int W, const double* psf, int psf_radius,
                          int cap, const eecmg_params* params, eecmg_stats* stats_out, void* hip_stream);
/* Restriction of eq. (12-13): g_coarse(i,j) = g_fine(2i, 2j); coarse size is
 * ceil(Hf/2) x ceil(Wf/2). */
int eecmg_op_restrict_dev(const void* g_fine_dev, int Hf, int Wf, void* g_coarse_dev, int precision,
                          void* hip_stream);
/* Coarse PSF of eq. (14), host only: psf_coarse receives (2*(r/2)+1)^2
 * doubles.  mode as eecmg_params.coarse_psf_mode. */
int eecmg_op_coarse_psf(const double* psf, int psf_radius, int mode, double* psf_coarse);
/* New extrapolation Pi (Section 3.2): uA on level l-1 (ceil(HB/2) x
 * ceil(WB/2)) and uB on level l (HB x WB) -> ut on level l (HB x WB). */
int eecmg_op_extrapolate_dev(const void* uA_dev, const void* uB_dev, int HB, int WB, void* ut_dev, int precision,
                             void* hip_stream);
/* Quadratic interpolation P (Section 3.2): ut (ceil(HC/2) x ceil(WC/2)) ->
 * uC (HC x WC). */
int eecmg_op_prolong_quad_dev(const void* ut_dev, int HC, int WC, void* uC_dev, int precision, void* hip_stream);
/* Linear prolongation L of eq. (15): uB (ceil(HC/2) x ceil(WC/2)) -> uC. */
int eecmg_op_prolong_linear_dev(const void* uB_dev, int HC, int WC, void* uC_dev, int precision,
                                void* hip_stream);
/* Level transfer with its stages fused into one kernel (Sections 3.2-4):
 * the prolongation of uB (ceil(HC/2) x ceil(WC/2)) -- the quadratic
 * interpolation P of Section 3.2 when prolongation == 0, the linear
 * prolongation of eq. (15) when 1 -- then the smoothing S with parameter
 * smooth_h > 0, then pm_steps (0 or 1) Perona-Malik steps D with threshold
 * k > 0 and step 0 < tau <= 1/4, written to uC (HC x WC, must not alias uB).
 * Gives the values of the separate operator calls run in sequence; EINVAL for
 * pm_steps outside {0, 1}. */
int eecmg_op_transfer_dev(const void* uB_dev, int HC, int WC, void* uC_dev, int prolongation, double smooth_h,
                          int pm_steps, double k, double tau, int precision, void* hip_stream);
/* Local smoothing S (Section 3.3, eq. 18-19), out of place, H x W. */
int eecmg_op_local_smooth_dev(const void* u_dev, void* out_dev, int H, int W, double smooth_h, int precision,
                              void* hip_stream);
/* One Perona-Malik step D (Section 4, eq. 21, 23-25), out of place, H x W. */
int eecmg_op_pm_step_dev(const void* u_dev, void* out_dev, int H, int W, double k, double tau, int precision,
                         void* hip_stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (diagnostics).  While enabled, every launch of a smoother or
 * transfer stage whose grid has at least min_blocks blocks, and whose jobs'
 * levels hold at least the pixels set by eecmg_profile_min_pixels (default 0;
 * EINVAL if negative or NaN), is bracketed by HIP events on its launch stream; eecmg_profile_read waits for the recorded
 * events and returns, for one stage id, the number of launches, their summed
 * duration, and the pixels they covered (sum over the jobs of the level's
 * H x W); smoother passes that found their level already stopped are left
 * out.  Stage ids: 0 restriction (with the coarse levels, solved in one
 * block per image, in the same launch), 1 CGLS init r, 2 CGLS init s, 3 CGLS
 * init finalize, 4 CGLS pass A (q = H p), 5 its finalize, 6 CGLS pass B
 * (s = H^T r), 7 its finalize, 8 MR init, 9 its finalize, 10 MR pass, 11 its
 * finalize, 12 extrapolation, 13 quadratic interpolation, 14 linear
 * prolongation, 15 smoothing S, 16 denoising D, 17 output copy, 18 fused
 * prolongation + S (+ first D step), 19 the same on short tiles, 21 deferred
 * solution update (20 and 22 are unused).  eecmg_profile_read_level returns,
 * for the launches whose jobs all worked on level index `level` (0 =
 * coarsest; the restriction launch counts as level -1), the number of
 * launches of one stage (-1: every stage) and their summed duration,
 * including the passes that found their level stopped (they take time too).
 * Process-wide; not meant for concurrent contexts.
 * ------------------------------------------------------------------------- */
int eecmg_profile_enable(int enable, int min_blocks);
int eecmg_profile_min_pixels(double min_pixels);
int eecmg_profile_reset(void);
int eecmg_profile_read(int stage, int* launches, double* total_ms, double* total_pixels);
int eecmg_profile_read_level(int stage, int level, int* launches, double* total_ms);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* eecmg_last_error(void);
/* Library version string. */
const char* eecmg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EECMG_H */
