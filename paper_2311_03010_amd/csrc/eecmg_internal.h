// Internal structures shared by the HIP kernels and the host runtime of the
// EECMG library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eecmg {

constexpr int kMaxLevels = 16;
constexpr int kMaxRadius = 12;
constexpr int kMaxLaunchJobs = 240;
constexpr int kNPart = 4;  // doubles per tile in the partial-sum array

// Smoother tiles: one wave spans the tile width, four waves stack kV rows each.
constexpr int kTW = 64;
constexpr int kV = 8;
constexpr int kTH = 4 * kV;
// Transfer / element-wise tiles: 64 x 16 pixels per 256-thread block.
constexpr int kXW = 64;
constexpr int kXH = 16;
// Extrapolation (Pi) tiles: kPiTH x kXW nodes of the coarser grid per block.
constexpr int kPiTH = 4;

// Smoother and cascade ids (same values as eecmg_smoother / eecmg_cascade).
enum : int32_t { kSmootherCgls = 0, kSmootherMr = 1 };
enum : int32_t { kCascadeEecmg = 0, kCascadeIecmgL = 1, kCascadeIecmgP = 2 };

// Stop reasons (same values as eecmg_stop_reason).
enum : int32_t { kStopNone = 0, kStopDiscrepancy = 1, kStopCap = 2, kStopGuard = 3, kStopNonFinite = 4 };

// Device-resident smoother scalars of one job (one per slot).  Every scalar
// of the Krylov recurrences lives here in FP64 and is only touched by the
// finalize kernels, so the host never reads them during a level.
// Direction slots of a level whose CGLS solution update is deferred (lazy_u):
// p_k lives in slot (k + 1) mod kPRing, so the kPRing - 1 latest directions
// stay available and their updates are applied together (k_flush_u).
constexpr int kPRing = 8;

struct SolverState {
  double gamma, gamma0, alpha, beta;  // CGLS: <s,s>, initial <s,s>, step, direction update
  double rr, rr0, rq, eta;            // <r,r>, initial <r,r>, <r,q> (MR), <q,q>
  double alph[kPRing];                // CGLS: step alpha_k of iteration k, in slot k mod kPRing
  double gam[2];                      // CGLS: gamma_k = <s_k,s_k> of the last iteration k of each parity
  int32_t k;                          // iterations completed on this level
  int32_t done;                       // stop reason, 0 while running
  int32_t par;                        // ping-pong parity of r/p/q buffers
  int32_t level;                      // level the state belongs to
  int32_t pending;                    // MR: a step alpha is waiting to be applied
  int32_t seq;                        // finalize counter (diagnostics)
  int32_t na;                         // CGLS: iterations whose step alpha is known (pass B then runs)
  int32_t pad;
};


struct LevelRecord {
  int32_t iters, reason;
  double rms;
};

// Everything a kernel needs about one job at one level.  The host builds one
// descriptor per (slot, level) when a job is admitted and uploads the table
// once; kernels find theirs through the launch list.
struct JobDesc {
  // smoother on this level
  void* g;
  void* u;
  void* r[2];
  void* p[2];
  void* s;
  void* q[2];
  const void* taps;    // psf_l, element type of the precision, (2r+1)^2
  const void* taps_t;  // flipped psf_l (operator H^T)
  int32_t h, w, pitch, rad;
  int32_t tiles_x, ntiles;  // smoother tiles (kTH x kTW)
  int32_t cap, level;
  int32_t stop_rule, smoother;
  int32_t cascade, pm_steps;
  int32_t coarse_levels;  // level 0 only: leading levels solved by the restriction launch's head block
  int32_t zero_u;         // bit l: level l's smoother starts from zero (no transfer into it)
  int32_t lazy_u;         // CGLS: u updated by k_flush_u from a ring of kPRing directions (see k_cg_b)
  int32_t fold_a;         // CGLS pass B may compute alpha itself (when its launch says so)
  int32_t nstrips;       // streaming policies: strips of the level (ntiles counts blocks)
  int32_t pad2, pad3, pad4;
  double cdelta, eps2;
  SolverState* st;
  LevelRecord* rec;  // kMaxLevels records of this job
  double* partials;  // kNPart components, component c of tile t at partials[c * pstride + t]
  uint64_t* mirror;  // host-visible progress word of this job's slot (see mirror_word)
  uint32_t tag;      // (job id << 8) | level, echoed in the progress word
  int32_t pstride;
  // transfer into this level from level-2 (A) and level-1 (B)
  const void* uA;
  const void* uB;
  void* t1;
  void* t2;
  int32_t hA, wA, pA, hB, wB, pB;
  double pm_k, tau, smooth_h;
  // restriction of the dense input / copy of the dense output (finest level)
  const void* g_in;
  const void* u_in;  // optional initial guess on the finest level (operator calls)
  void* u_out;
  int32_t H, W, L, fine_pitch;
  void* g_lv[kMaxLevels];
  void* u_lv[kMaxLevels];
  int32_t lh[kMaxLevels], lw[kMaxLevels], lp[kMaxLevels];
  // bytes of the job's PSF-taps region (it starts at level 0's taps)
  int32_t taps_bytes;
  int32_t f64;  // element type double (else float)
};

static_assert(sizeof(JobDesc) % 4 == 0, "descriptors are copied as 32-bit words");

// Slots whose descriptors and taps k_upload copies from pinned host memory.
struct UploadList {
  int32_t n;
  int32_t slot[kMaxLaunchJobs];
};

// Progress word published by the finalize kernels into pinned host memory:
// [63:32] tag (job id << 8 | level), [31:8] iterations done, [7:0] stop reason.
__host__ __device__ inline uint64_t mirror_word(uint32_t tag, int32_t k, int32_t done) {
  return ((uint64_t)tag << 32) | ((uint64_t)(uint32_t)(k & 0xFFFFFF) << 8) | (uint64_t)(uint32_t)(done & 0xFF);
}

// Kernel-argument list of the jobs one launch covers.  Block b belongs to the
// entry e with start[e] <= b < start[e+1]; job[e] indexes the JobDesc table.
// Launch options (LaunchList::flags).
// kLaunchFoldA: pass B evaluates pass A's finalize; kLaunchFoldB: pass A of
// entry e evaluates the finalize still owed before iteration kf[e] (the
// previous pass B's, or at iteration 0 the initialisation's); kf[e] < 0: none
// is owed.  Both only for jobs whose level has fold_a set.
// kLaunchInitS: the initialisation's first launch also forms s = H^T r for
// the jobs whose level has a one-tap blur on the general tiles (their r needs
// no halo), which then skip the second launch.
enum : int32_t { kLaunchFoldA = 1, kLaunchFoldB = 2, kLaunchInitS = 4 };

struct LaunchList {
  int32_t n;
  int32_t total;
  int32_t flags;
  int32_t pad;
  int32_t job[kMaxLaunchJobs];
  int32_t start[kMaxLaunchJobs + 1];
  int32_t kf[kMaxLaunchJobs];  // per entry: iteration index of a folded finalize, or -1
};
static_assert(sizeof(LaunchList) + 64 <= 4096, "kernel arguments stay below 4 KiB");

// Stages launched by the runtime.
enum Stage : int32_t {
  kRestrict = 0,    // dense g -> level pyramid; zero u pyramid (or copy u_in); coarse levels solved
  kCgInit1,         // r = g - H u0
  kCgInit2,         // s = H^T r, p = s
  kCgFinInit,
  kCgA,             // p = s + beta p, q = H p
  kCgFinA,
  kCgB,             // r -= alpha q, s = H^T r, u += alpha p
  kCgFinB,
  kMrInit,          // r = g - H u0
  kMrFinInit,
  kMrPass,          // r -= alpha q, u += alpha r, q = H r
  kMrFin,
  kXfExtrap,        // Pi: (uA, uB) -> t2 on grid B
  kXfQuad,          // P: src (grid B) -> t1 (grid C)
  kXfLinear,        // L: uB -> t1
  kXfSmooth,        // S: src -> dst
  kXfPm,            // D: src -> dst
  kOutCopy,         // u (finest, pitched) -> dense u_out
  kXfFused,         // prolongation -> S (-> one D step), fused; variant bit 0 quadratic, bit 1 with D
  kXfFusedSmall,    // the same with short tiles, for small levels
  kReserved20,      // (unused id: the coarse levels are solved inside the restriction launch)
  kFlushU,          // apply a deferred CGLS solution update when a lazy_u level stops
  kReserved22,      // (unused id, kept so the stage numbers stay stable)
  kNumStages
};

// Buffer selectors of the transfer stages.
enum XBuf : int32_t { kBufU = 0, kBufT1 = 1, kBufT2 = 2, kBufUB = 3 };

// Blur-operator implementation families.  A variant id is kind * 100 + R
// (for kConvGeneral, R is the radius class 3, 6 or 12).
enum ConvKind : int32_t {
  kConvGeneral = 0,
  kConvSep = 1,
  kConvSymSquare = 2,
  kConvSymDisk = 3,
  kConvBoxDisk = 4,
  kConvGenShort = 5  // general policy on short tiles (small levels: more blocks per launch)
};
// Tile height of the short general tiles.
#ifndef EECMG_SHORT_TH
#define EECMG_SHORT_TH 16
#endif
constexpr int kTHShort = EECMG_SHORT_TH;

// Rows per unrolled group of the streaming (sliding-column) families: a
// multiple of 2R + 1 (the pending-output ring) of at least 4 rows (the
// prefetch ring).  Output rows per tile: the smallest height >= kTH whose
// input rows (height + 2R) fill whole groups, so the row loop has no partial
// group.
__host__ __device__ constexpr int strip_group(int R) {
  return (2 * R + 1) * ((4 + 2 * R) / (2 * R + 1));
}
// Tall strips (at least 2 kTH rows) serve large FP32 levels: half the halo
// rows per output and half the strips in flight per XCD.
constexpr int kTHTall = 2 * kTH;
// Short strips (at least kTH / 4 rows) serve streaming levels that give the
// chip too few strips of the usual height (mid-size levels, which the
// Infinity Cache holds, so the extra halo rows cost little).
constexpr int kTHShortStrip = kTH / 4;
// Streaming strips per block (one per wave): the blocks of a pass, and so the
// partial sums of its inner products, are a quarter of its strips, which keeps
// the finalize that every block of the next pass may evaluate cheap.
constexpr int kStripsPerBlock = 4;
// Strip mode: 0 usual height, 1 tall, 2 short.
__host__ __device__ constexpr int strip_th(int R, int mode = 0) {
  return strip_group(R) *
             (((mode == 1 ? kTHTall : mode == 2 ? kTHShortStrip : kTH) + 2 * R + strip_group(R) - 1) / strip_group(R)) -
         2 * R;
}
// A variant id is kind * 100 + R, plus kTallVariant (kShortVariant) for a
// streaming kind on tall (short) strips.
constexpr int kTallVariant = 10000;
constexpr int kShortVariant = 20000;
__host__ __device__ constexpr int variant_kind(int variant) { return (variant % kTallVariant) / 100; }
__host__ __device__ constexpr int variant_r(int variant) { return variant % 100; }
__host__ __device__ constexpr int variant_strip_mode(int variant) { return variant / kTallVariant; }
__host__ __device__ constexpr bool variant_tall(int variant) { return variant_strip_mode(variant) == 1; }
__host__ __device__ constexpr int tile_h_for_variant(int variant) {
  return variant_kind(variant) == kConvGeneral    ? kTH
         : variant_kind(variant) == kConvGenShort ? kTHShort
                                                  : strip_th(variant_r(variant), variant_strip_mode(variant));
}

// Host-side launchers (defined in eecmg_kernels.hip).
hipError_t launch_stage(Stage st, bool f64, int variant, const LaunchList& ll, const JobDesc* descs, int src,
                        int dst, hipStream_t stream);
int rmax_class_for(int r);
int blocks_for_stage(Stage st, const JobDesc& d);

// Copy the listed slots' descriptors (host table hdesc, kMaxLevels per slot)
// and PSF taps (htaps, taps_stride bytes per slot), both in device-visible
// pinned host memory, to ddesc and to each job's taps region.
hipError_t launch_upload(const UploadList& ul, const JobDesc* hdesc, JobDesc* ddesc, const char* htaps,
                         size_t taps_stride, hipStream_t s);

// Set n 32-bit words at p to zero with a kernel on stream s.
hipError_t launch_zero_words(void* p, size_t n, hipStream_t s);

// Operator kernels on dense buffers (one image, no job table).
hipError_t op_conv(const void* x, void* y, int H, int W, const void* taps, int variant, int radius, bool f64,
                   hipStream_t s);
hipError_t op_restrict(const void* gf, int Hf, int Wf, void* gc, bool f64, hipStream_t s);
hipError_t op_extrapolate(const void* uA, const void* uB, int HB, int WB, void* ut, bool f64, hipStream_t s);
hipError_t op_prolong_quad(const void* ut, int HC, int WC, void* uC, bool f64, hipStream_t s);
hipError_t op_prolong_linear(const void* uB, int HC, int WC, void* uC, bool f64, hipStream_t s);
hipError_t op_local_smooth(const void* u, void* out, int H, int W, double h, bool f64, hipStream_t s);
hipError_t op_pm_step(const void* u, void* out, int H, int W, double k, double tau, bool f64, hipStream_t s);
hipError_t op_fused_transfer(const void* uB, int HC, int WC, void* uC, bool quad, double smooth_h, bool denoise,
                             double k, double tau, bool f64, hipStream_t s);

}  // namespace eecmg
