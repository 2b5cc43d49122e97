// Host runtime of the EECMG library: level plans, a device memory arena, the
// job engine that drives every restore (plain, batched and served requests
// all run through it), the request loop with continuous batching, and the C
// ABI declared in include/eecmg.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/eecmg.h"
#include "eecmg_internal.h"

namespace eecmg {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define EECMG_HIP(call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(EECMG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Host copy of a served request's image into or out of its pinned staging
// buffer; large images are split over a few threads (one thread's memcpy
// reaches only a fraction of the host's memory bandwidth).
static void staging_copy(void* dst, const void* src, size_t bytes) {
  constexpr size_t kChunk = (size_t)8 << 20;
  constexpr int kMaxThreads = 8;
  const int n = (int)std::min<size_t>(kMaxThreads, bytes / kChunk);
  if (n < 2) {
    std::memcpy(dst, src, bytes);
    return;
  }
  const size_t part = align_up((bytes + n - 1) / n, 4096);
  std::vector<std::thread> th;
  for (int i = 1; i < n; ++i) {
    const size_t o = part * (size_t)i;
    if (o >= bytes) break;
    th.emplace_back([=] { std::memcpy((char*)dst + o, (const char*)src + o, std::min(part, bytes - o)); });
  }
  std::memcpy(dst, src, std::min(part, bytes));
  for (auto& t : th) t.join();
}

constexpr size_t kTapsSlotBytes = 32 << 10;  // pinned staging of one job's PSF pyramid

// ---------------------------------------------------------------------------
// Level plan (Section 2: nested grids, m_l rule; eq. 12-14: restriction and
// coarse operators)
// ---------------------------------------------------------------------------
struct LevelPlan {
  int h = 0, w = 0, pitch = 0, rad = 0, cap = 0, ntiles = 0, tiles_x = 0;
  int nstrips = 0;  // smoother tiles (general) or strips (streaming); ntiles counts blocks
  int variant = 0;                    // blur-operator kernel family (ConvKind * 100 + R)
  bool lazy = false;                  // CGLS solution updates deferred (k_flush_u)
  bool fold_a = false;                // CGLS pass B evaluates pass A's finalize itself
  std::vector<double> psf;            // (2 rad + 1)^2, FP64
  std::vector<double> taps, taps_t;   // the variant's tap layout for H and H^T
};

// Largest b with a^2 + b^2 <= R^2 (disk support), or R (square support); the
// same layout rule as the symmetric device policy.
static int sym_span_h(int R, bool disk, int a) {
  if (!disk) return R;
  int b = 0;
  while ((b + 1) * (b + 1) + a * a <= R * R) ++b;
  return b;
}

// Pick the blur-operator kernel family for one level's PSF and lay out its
// taps (FP64; converted to the element type at upload):
//   rank one (to 8 ulp)                 -> separable: row(-R..R), col(-R..R)
//   symmetric in both axes, disk support -> row-filter kernel on the quadrant
//   symmetric in both axes               -> same with square support (R <= 6)
//   otherwise                            -> general (all taps)
// Small levels with small radii always take the general kernels on short
// tiles: their whole-tile loads (four waves per tile, all rows at once) have
// far less latency per launch than one wave streaming down each strip, and
// short tiles give a small level enough blocks to fill the chip.  From 1024^2
// pixels the streaming kernels (four strips per block, short strips) are
// faster: the 4096^2 restore -1.8%, four of them in a batch -2.1%.
constexpr long kSmallLevelPixels = 512L * 512L;
// Levels up to this many pixels (the leading ones of a cascade) are solved
// by one block per job in a single launch (EECMG_COARSE_MAX_PIXELS moves the
// limit; 32^2, 64^2 and 128^2 measured, 64^2 best on the 4096^2 restore).
constexpr long kCoarsePixels = 64L * 64L;
static long coarse_max_pixels() {
  const char* e = std::getenv("EECMG_COARSE_MAX_PIXELS");
  return e ? std::atol(e) : kCoarsePixels;
}
// CGLS levels of at least this many pixels defer their solution updates
// (k_cg_b's lazy_u mode): pass B moves no u or p, and k_flush_u applies the
// terms of up to kPRing - 1 iterations in one pass (reading u and their
// directions once) -- 4 + 8 / (kPRing - 1) instead of 12 bytes per pixel and
// iteration, for kPRing - 2 more direction buffers of the finest level's size.
constexpr long kLazyPixels = 1024L * 1024L;
// The threshold can be moved with EECMG_LAZY_MIN_PIXELS (tests use it to run
// both update schedules on small images).
static long lazy_min_pixels() {
  const char* e = std::getenv("EECMG_LAZY_MIN_PIXELS");
  return e ? std::atol(e) : kLazyPixels;
}
// CGLS levels with at most this many blocks per pass let every block of
// pass B sum pass A's partials itself, and every block of pass A the previous
// pass B's (the same fixed order as the finalize kernel, so alpha and beta
// are bit-identical), which saves two launches per iteration.  Each block
// reads every partial of the pass before, so the cost grows with the square
// of the block count; with four strips per streaming block even the 4096^2
// level (1008 blocks) gains (restore -2.5% against no fold on the two largest
// levels).  EECMG_FOLD_MAX_TILES and EECMG_FOLD_MAX_TILES_STREAM move the
// limits (0 turns folding off).
constexpr long kFoldMaxTiles = 4096;
constexpr long kFoldMaxTilesStream = 1L << 30;
// Launches of at most this many jobs fold (EECMG_FOLD_MAX_JOBS moves it).
constexpr int kFoldMaxJobs = 1;
static int fold_max_jobs() {
  const char* e = std::getenv("EECMG_FOLD_MAX_JOBS");
  return e ? std::max(0, std::atoi(e)) : kFoldMaxJobs;
}
// Levels whose tall-strip tiles number at least this many (two waves per
// SIMD of the 1024 on the chip) use tall strips; EECMG_TALL_MIN_TILES moves
// the limit and EECMG_TALL_STRIPS=0 keeps every level on short strips.
constexpr long kTallMinTiles = 2048;
static bool tall_strips_enabled() {
  const char* e = std::getenv("EECMG_TALL_STRIPS");
  return !(e && e[0] == '0');
}
static long tall_min_tiles() {
  const char* e = std::getenv("EECMG_TALL_MIN_TILES");
  return e ? std::atol(e) : kTallMinTiles;
}
// FP32 streaming levels whose usual strips number fewer than this (one wave
// per SIMD of the chip) use short strips (EECMG_SHORT_MAX_TILES; 0 turns
// them off).  Measured against 2048 with 16-row short strips: the uneven
// batch -8.5%, the 4096^2 restore -0.6% (its 2048^2 level keeps the usual
// strips, its 1024^2 level gets four times as many waves).
constexpr long kShortMaxTiles = 1024;
static long short_max_tiles() {
  const char* e = std::getenv("EECMG_SHORT_MAX_TILES");
  return e ? std::atol(e) : kShortMaxTiles;
}
static long fold_max_tiles() {
  const char* e = std::getenv("EECMG_FOLD_MAX_TILES");
  return e ? std::atol(e) : kFoldMaxTiles;
}
static long fold_max_tiles_stream() {
  const char* e = std::getenv("EECMG_FOLD_MAX_TILES_STREAM");
  return e ? std::atol(e) : kFoldMaxTilesStream;
}
static void choose_variant(LevelPlan& lp, bool f64, bool by_size) {
  const int R = lp.rad, n = 2 * R + 1;
  const std::vector<double>& P = lp.psf;
  auto at = [&](int a, int b) { return P[(a + R) * n + (b + R)]; };
  if (by_size && (long)lp.h * lp.w <= kSmallLevelPixels && R <= 3) {
    lp.variant = kConvGenShort * 100 + rmax_class_for(R);
    lp.taps = P;
    lp.taps_t.assign(P.rbegin(), P.rend());
    return;
  }
  int a0 = 0, b0 = 0;
  double mx = 0.0;
  for (int a = -R; a <= R; ++a)
    for (int b = -R; b <= R; ++b)
      if (std::fabs(at(a, b)) > mx) {
        mx = std::fabs(at(a, b));
        a0 = a;
        b0 = b;
      }
  if (mx > 0.0) {
    std::vector<double> col(n), row(n);
    for (int k = -R; k <= R; ++k) {
      col[k + R] = at(k, b0);
      row[k + R] = at(a0, k) / at(a0, b0);
    }
    double err = 0.0;
    for (int a = -R; a <= R; ++a)
      for (int b = -R; b <= R; ++b) err = std::max(err, std::fabs(at(a, b) - col[a + R] * row[b + R]));
    if (err <= 8.0 * 2.220446049250313e-16 * mx) {
      lp.variant = kConvSep * 100 + R;
      lp.taps.assign(row.begin(), row.end());
      lp.taps.insert(lp.taps.end(), col.begin(), col.end());
      lp.taps_t.assign(row.rbegin(), row.rend());
      lp.taps_t.insert(lp.taps_t.end(), col.rbegin(), col.rend());
      return;
    }
  }
  bool sym = true, disk = true, uniform = R >= 1 && at(0, 0) != 0.0;
  for (int a = -R; a <= R; ++a)
    for (int b = -R; b <= R; ++b) {
      if (at(a, b) != at(-a, b) || at(a, b) != at(a, -b)) sym = false;
      if (a * a + b * b > R * R && at(a, b) != 0.0) disk = false;
      if (a * a + b * b <= R * R && at(a, b) != at(0, 0)) uniform = false;
    }
  // FP64 disk kernels above R = 6 would spill registers: general kernel instead
  const int disk_max = f64 ? 6 : 8;
  if (sym && disk && uniform && R <= disk_max) {
    // uniform disk: one weight, row filters are plain sums over nested spans
    lp.variant = kConvBoxDisk * 100 + R;
    lp.taps.assign(1, at(0, 0));
    lp.taps_t = lp.taps;
    return;
  }
  if (sym && ((disk && R <= disk_max) || R <= 6)) {
    const bool use_disk = disk && R <= disk_max;
    lp.variant = (use_disk ? kConvSymDisk : kConvSymSquare) * 100 + R;
    lp.taps.clear();
    for (int a = 0; a <= R; ++a)
      for (int b = 0; b <= sym_span_h(R, use_disk, a); ++b) lp.taps.push_back(at(a, b));
    lp.taps_t = lp.taps;  // H^T = H for a PSF symmetric in both axes
    return;
  }
  lp.variant = kConvGeneral * 100 + rmax_class_for(R);
  lp.taps = P;
  lp.taps_t.assign(P.rbegin(), P.rend());
}

struct Plan {
  int H = 0, W = 0, L = 0;
  bool f64 = false;
  size_t esz = 4;
  eecmg_params prm{};
  double k = 10.0;
  double eps2 = 0.0;
  LevelPlan lv[kMaxLevels];
  std::vector<int> order;  // 0-based levels in solve order
  bool own_gin = false, own_uout = false;
  // device layout (byte offsets inside the job allocation)
  size_t off_gin = 0, off_uout = 0, off_part = 0, taps_bytes = 0;  // taps region at offset 0
  size_t off_g[kMaxLevels] = {}, off_u[kMaxLevels] = {}, off_taps[kMaxLevels] = {}, off_tapst[kMaxLevels] = {};
  size_t off_work[7] = {};  // r0 r1 p0 p1 s q0 q1 (p0, p1: the first direction slots)
  size_t bytes = 0;
  int max_tiles = 0;
  int coarse = 0;  // leading levels solved by the restriction launch (one block per job)
};

// Economic iteration counts (Section 2): for l > L/2,
// ceil((L - L/2)^2 4^(L-l)); otherwise ceil((L - 1.5 l) 4^(l-1)); at least 1.
static int economic_cap(int L, int l) {
  const double half = 0.5 * L;
  double t;
  if (l > half)
    t = (L - half) * (L - half) * std::ldexp(1.0, 2 * (L - l));
  else
    t = (L - 1.5 * l) * std::ldexp(1.0, 2 * (l - 1));
  const double c = std::ceil(t);
  return c < 1.0 ? 1 : (int)c;
}

// psf_c(a, b) = s psf(2a, 2b), radius r/2; s per coarse_psf_mode.
static int decimate_psf(const std::vector<double>& psf, int r, int mode, std::vector<double>& out) {
  const int n = 2 * r + 1, rc = r / 2, nc = 2 * rc + 1;
  double tot = 0.0, sub = 0.0;
  for (double v : psf) tot += v;
  for (int a = -rc; a <= rc; ++a)
    for (int b = -rc; b <= rc; ++b) sub += psf[(2 * a + r) * n + (2 * b + r)];
  double s;
  if (mode == 0) {
    if (sub == 0.0) return fail(EECMG_EINVAL, "coarse PSF: the decimated taps sum to zero (use coarse_psf_mode 1 or 2)");
    s = tot / sub;
  } else if (mode == 1) {
    s = 4.0;
  } else if (mode == 2) {
    s = 1.0;
  } else {
    return fail(EECMG_EINVAL, "coarse_psf_mode must be 0, 1 or 2");
  }
  out.assign((size_t)nc * nc, 0.0);
  for (int a = -rc; a <= rc; ++a)
    for (int b = -rc; b <= rc; ++b) out[(a + rc) * nc + (b + rc)] = s * psf[(2 * a + r) * n + (2 * b + r)];
  return EECMG_OK;
}

static void default_params(eecmg_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(eecmg_params);
  p->precision = EECMG_FP32;
  p->stop_rule = 1;
  p->delta = 1.0;
  p->c = 1.1;
  p->tau = 0.2;
  p->pm_steps = 1;
  p->smooth_h = 1.0;
  p->coarse_psf_mode = 0;
  p->guard_eps = 0.0;
  p->smoother = EECMG_SMOOTHER_CGLS;
  p->cascade = EECMG_CASCADE_EECMG;
  p->stats = nullptr;
}

// defer_updates = false: no level defers its CGLS solution updates (two
// direction buffers instead of kPRing; the results are the same bits).
static int build_plan(int H, int W, const double* psf, int r, int L, const int* caps, double k,
                      const eecmg_params* params, bool own_io, Plan& P, bool defer_updates = true) {
  eecmg_params prm;
  if (params) {
    if (params->struct_size != sizeof(eecmg_params)) return fail(EECMG_EINVAL, "params->struct_size mismatch");
    prm = *params;
  } else {
    default_params(&prm);
  }
  if (prm.precision == EECMG_FP32_FP16COARSE)
    return fail(EECMG_EINVAL,
                "FP16 storage of coarse levels is not provided: it stays within the FP32 error bar only on levels "
                "of at most 128^2 pixels, which are launch-bound, so it would add error and save no time");
  if (prm.precision < 0 || prm.precision > 1) return fail(EECMG_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (L < 1 || L > kMaxLevels) return fail(EECMG_EINVAL, "n_levels must be in [1, 16]");
  if (H < 3 || W < 3) return fail(EECMG_EINVAL, "image must be at least 3 x 3");
  if ((long long)H * W > (1LL << 31)) return fail(EECMG_EINVAL, "image too large");
  if (r < 0 || r > kMaxRadius) return fail(EECMG_EINVAL, "psf_radius must be in [0, 12]");
  if (!psf) return fail(EECMG_EINVAL, "psf is NULL");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(EECMG_EINVAL, "k must be > 0");
  if (!(prm.tau > 0.0 && prm.tau <= 0.25)) return fail(EECMG_EINVAL, "tau must be in (0, 1/4]");
  if (prm.pm_steps < 0 || prm.pm_steps > 64) return fail(EECMG_EINVAL, "pm_steps must be in [0, 64]");
  if (!(prm.smooth_h > 0.0) || !std::isfinite(prm.smooth_h)) return fail(EECMG_EINVAL, "smooth_h must be > 0");
  if (!(prm.delta >= 0.0) || !std::isfinite(prm.delta)) return fail(EECMG_EINVAL, "delta must be >= 0");
  if (prm.stop_rule && !(prm.c > 1.0)) return fail(EECMG_EINVAL, "c must be > 1 with the stopping rule");
  if (!(prm.guard_eps >= 0.0) || prm.guard_eps >= 1.0) return fail(EECMG_EINVAL, "guard_eps must be in [0, 1)");
  if (prm.smoother < 0 || prm.smoother > 1) return fail(EECMG_EINVAL, "smoother must be 0 (CGLS) or 1 (MR)");
  if (prm.cascade < 0 || prm.cascade > 2) return fail(EECMG_EINVAL, "cascade must be 0, 1 or 2");
  const int n = 2 * r + 1;
  for (int i = 0; i < n * n; ++i)
    if (!std::isfinite(psf[i])) return fail(EECMG_EINVAL, "psf has a non-finite tap");

  P = Plan();
  P.H = H;
  P.W = W;
  P.L = L;
  P.f64 = prm.precision == EECMG_FP64;
  P.esz = P.f64 ? 8 : 4;
  P.prm = prm;
  P.prm.stats = nullptr;
  P.k = k;
  const double eps = prm.guard_eps > 0.0 ? prm.guard_eps : (P.f64 ? 1e-14 : 1e-6);
  P.eps2 = eps * eps;
  P.own_gin = P.own_uout = own_io;
  // level sizes, coarsest first
  int hh = H, ww = W;
  for (int l = L - 1; l >= 0; --l) {
    P.lv[l].h = hh;
    P.lv[l].w = ww;
    hh = (hh + 1) / 2;
    ww = (ww + 1) / 2;
  }
  for (int l = 0; l < L; ++l)
    if (P.lv[l].h < 3 || P.lv[l].w < 3)
      return fail(EECMG_EINVAL, "too many levels: every level needs at least 3 nodes per axis");
  // caps
  for (int l = 0; l < L; ++l) {
    const int c = caps ? caps[l] : economic_cap(L, l + 1);
    if (c < 0) return fail(EECMG_EINVAL, "iters_per_level entries must be >= 0");
    P.lv[l].cap = c;
  }
  // PSF pyramid, finest first
  P.lv[L - 1].rad = r;
  P.lv[L - 1].psf.assign(psf, psf + (size_t)n * n);
  for (int l = L - 2; l >= 0; --l) {
    const int rc = decimate_psf(P.lv[l + 1].psf, P.lv[l + 1].rad, prm.coarse_psf_mode, P.lv[l].psf);
    if (rc != EECMG_OK) return rc;
    P.lv[l].rad = P.lv[l + 1].rad / 2;
  }
  // solve order
  P.order.clear();
  for (int l = 0; l < L; ++l) P.order.push_back(l);
  // leading small levels go to the one-block coarse cascade (full taps)
  P.coarse = 0;
  const long coarse_px = coarse_max_pixels();
  while (P.coarse < L && (long)P.lv[P.coarse].h * P.lv[P.coarse].w <= coarse_px) P.coarse += 1;
  // tiles and layout
  const size_t pitch_elems = P.f64 ? 32 : 64;  // 256-byte rows
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  for (int l = 0; l < L; ++l) {
    if (l < P.coarse) {
      LevelPlan& lp = P.lv[l];
      lp.variant = kConvGeneral * 100 + rmax_class_for(lp.rad);
      lp.taps = lp.psf;
      lp.taps_t.assign(lp.psf.rbegin(), lp.psf.rend());
    } else {
      choose_variant(P.lv[l], P.f64, true);
      P.lv[l].lazy = defer_updates && P.prm.smoother == EECMG_SMOOTHER_CGLS &&
                     (long)P.lv[l].h * P.lv[l].w >= lazy_min_pixels();
    }
    P.off_taps[l] = take(P.lv[l].taps.size() * P.esz);
    P.off_tapst[l] = take(P.lv[l].taps_t.size() * P.esz);
  }
  P.taps_bytes = off;
  if (P.taps_bytes > kTapsSlotBytes) return fail(EECMG_EINVAL, "PSF pyramid too large");
  if (P.own_gin) P.off_gin = take((size_t)H * W * P.esz);
  if (P.own_uout) P.off_uout = take((size_t)H * W * P.esz);
  for (int l = 0; l < L; ++l) {
    LevelPlan& lp = P.lv[l];
    lp.pitch = (int)align_up((size_t)lp.w, pitch_elems);
    if ((size_t)lp.h * lp.pitch * P.esz >= ((size_t)1 << 32))
      return fail(EECMG_EINVAL, "a level array would exceed 4 GiB (32-bit offsets)");
    lp.tiles_x = (lp.w + kTW - 1) / kTW;
    const int kind = variant_kind(lp.variant);
    const bool general = kind == kConvGeneral || kind == kConvGenShort;
    // FP32 streaming kernels walk tall strips on levels that still give the
    // chip enough of them (the choice depends on the level's shape only, so
    // an image gets the same kernels alone and in a batch)
    auto strips = [&](int mode) {
      const int th = strip_th(variant_r(lp.variant), mode);
      return (long)lp.tiles_x * ((lp.h + th - 1) / th);
    };
    if (!general && !P.f64 && tall_strips_enabled() && strips(1) >= tall_min_tiles())
      lp.variant += kTallVariant;
    else if (!general && !P.f64 && strips(0) < short_max_tiles())
      lp.variant += kShortVariant;
    const int th = tile_h_for_variant(lp.variant);
    lp.nstrips = lp.tiles_x * ((lp.h + th - 1) / th);
    // smoother blocks (= partial-sum slots): one tile, or kStripsPerBlock strips
    lp.ntiles = general ? lp.nstrips : (lp.nstrips + kStripsPerBlock - 1) / kStripsPerBlock;
    lp.fold_a = l >= P.coarse && P.prm.smoother == EECMG_SMOOTHER_CGLS &&
                lp.ntiles <= (general ? fold_max_tiles() : fold_max_tiles_stream());
    P.max_tiles = std::max(P.max_tiles, lp.ntiles);
    P.off_g[l] = take((size_t)lp.h * lp.pitch * P.esz);
    P.off_u[l] = take((size_t)lp.h * lp.pitch * P.esz);
  }
  const size_t fine = (size_t)P.lv[L - 1].h * P.lv[L - 1].pitch * P.esz;
  // r, r', s, q, q', then the direction slots, evenly spaced: two, or
  // kPRing when a level defers its solution updates
  for (int i : {0, 1, 4, 5, 6}) P.off_work[i] = take(fine);
  bool any_lazy = false;
  for (int l = 0; l < L; ++l) any_lazy = any_lazy || P.lv[l].lazy;
  P.off_work[2] = take(fine);
  P.off_work[3] = take(fine);
  for (int i = 2; i < (any_lazy ? kPRing : 2); ++i) take(fine);
  P.off_part = take((size_t)P.max_tiles * kNPart * sizeof(double));
  P.bytes = off;
  return EECMG_OK;
}

// ---------------------------------------------------------------------------
// Device arena: one slab, first-fit free list with coalescing.
// ---------------------------------------------------------------------------
class Arena {
 public:
  ~Arena() {}
  int reserve(size_t bytes) {
    if (bytes <= size_) return EECMG_OK;
    if (!owned_) return fail(EECMG_ENOMEM, "the arena is a fixed region and cannot grow");
    if (used_ != 0) return fail(EECMG_ENOMEM, "arena busy, cannot grow");
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
    size_ = 0;
    free_.clear();
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(EECMG_ENOMEM, "hipMalloc of the device arena failed (" + std::to_string(bytes) + " bytes)");
    }
    base_ = (char*)p;
    size_ = bytes;
    free_[0] = bytes;
    return EECMG_OK;
  }
  void release() {
    if (base_ && owned_) (void)hipFree(base_);
    base_ = nullptr;
    size_ = used_ = 0;
    free_.clear();
  }
  // Use [base, base + bytes) of memory the arena does not own (never grown
  // or freed by it).
  void adopt(void* base, size_t bytes) {
    base_ = (char*)base;
    size_ = bytes;
    used_ = 0;
    owned_ = false;
    free_.clear();
    free_[0] = bytes;
  }
  void* alloc(size_t n) {
    n = align_up(n, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        used_ += n;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void free(void* p, size_t n) {
    n = align_up(n, 256);
    size_t off = (char*)p - base_;
    used_ -= n;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  bool owned_ = true;
  std::map<size_t, size_t> free_;
};


// ---------------------------------------------------------------------------
// Kernel timing (diagnostics): HIP events around selected launches.
// ---------------------------------------------------------------------------
struct Profiler {
  std::mutex mu;
  std::atomic<bool> on{false};
  int min_blocks = 0;
  double min_pixels = 0.0;
  struct Tag {
    uint32_t uid;
    int level, kidx;
    bool mr;
  };
  struct Rec {
    int stage;
    hipEvent_t a, b;
    double pixels;
    std::vector<Tag> tags;  // smoother passes: which iteration each job runs
    int level;              // level index shared by every job of the launch, or -1
  };
  std::vector<Rec> pending;
  std::map<uint64_t, int> final_iters;  // (uid, level) -> iterations run
  std::vector<hipEvent_t> pool;
  int launches[kNumStages] = {};
  double ms[kNumStages] = {};
  double pixels[kNumStages] = {};
  // every launch (also those that found their level stopped) by level and stage
  int lv_launches[kMaxLevels][kNumStages] = {};
  double lv_ms[kMaxLevels][kNumStages] = {};

  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // A smoother pass launched after its level had already stopped returns at
  // once; such launches are not counted.  CGLS iteration k runs both passes
  // iff k < iterations run; MR pass k runs iff k <= iterations run.
  bool real(const Rec& r) const {
    if (r.tags.empty()) return true;
    for (const Tag& t : r.tags) {
      auto it = final_iters.find(((uint64_t)t.uid << 8) | (uint64_t)t.level);
      if (it == final_iters.end()) return true;
      if (t.mr ? t.kidx <= it->second : t.kidx < it->second) return true;
    }
    return false;
  }
  void harvest() {
    for (auto& r : pending) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        if (real(r)) {
          launches[r.stage] += 1;
          ms[r.stage] += t;
          pixels[r.stage] += r.pixels;
        }
        if (r.level >= 0 && r.level < kMaxLevels) {
          lv_launches[r.level][r.stage] += 1;
          lv_ms[r.level][r.stage] += t;
        }
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
};

static Profiler& profiler() {
  static Profiler* p = new Profiler();
  return *p;
}

static bool profiled_stage(Stage st) { return st >= 0 && st < kNumStages; }

// ---------------------------------------------------------------------------
// Jobs and the engine
// ---------------------------------------------------------------------------
constexpr int kMaxSlots = EECMG_MAX_SLOTS;
static_assert(kMaxSlots <= kMaxLaunchJobs, "one launch must be able to cover every slot");

// An event owned by every job that waits for it.
struct HipEvent {
  hipEvent_t e = nullptr;
  HipEvent() { (void)hipEventCreateWithFlags(&e, hipEventDisableTiming); }
  ~HipEvent() {
    if (e) (void)hipEventDestroy(e);
  }
  HipEvent(const HipEvent&) = delete;
  HipEvent& operator=(const HipEvent&) = delete;
};

struct Job {
  Plan plan;
  int slot = -1;
  char* mem = nullptr;
  const void* g_in_dev = nullptr;
  const void* u_init_dev = nullptr;
  void* u_out_dev = nullptr;
  enum Phase { kNew, kStartLevel, kIter, kOutput, kWaitOut, kFinished } phase = kNew;
  int oi = 0;
  int issued = 0;
  int next_chunk = 1;
  int confirmed = 0;
  bool level_done_seen = false;
  uint32_t uid = 0;           // engine-assigned id, part of the progress tag
  std::shared_ptr<struct HipEvent> done_ev;  // output complete (shared by jobs finishing in one step)
  bool needs_upload = false;                  // descriptors and taps still in pinned host memory
  // a finalize the job still owes on its level (see kLaunchFoldB): that of
  // its initialisation or of its last issued pass B
  enum Owed { kOwesNone = 0, kOwesInit = 1, kOwesB = 2 } owed = kOwesNone;
  // served requests: the input copy runs on the context's copy stream; the
  // first kernel of the job waits for in_ev, the output copy for comp_ev
  hipEvent_t in_ev = nullptr, comp_ev = nullptr;
  bool in_wait = false;
  int status = EECMG_OK;
  LevelRecord rec[kMaxLevels];
  // served-request extras
  uint64_t id = 0;
  void* host_in = nullptr;   // pinned staging of g
  void* host_out = nullptr;  // pinned staging of u
  size_t host_bytes = 0;
  std::atomic<bool> cancelled{false};
  double t_submit = 0.0, t_done = 0.0;
  // the finest level reads g_in_dev / writes u_out_dev in place (see alias_io)
  bool alias_in = false, alias_out = false;
  // valid while the job is on a level (phases kStartLevel and kIter)
  int cur_level() const { return oi < (int)plan.order.size() ? plan.order[oi] : -1; }
};

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

class Engine {
 public:
  explicit Engine(int device) : device_(device) {}
  ~Engine() {}

  int init(hipStream_t stream) {
    EECMG_HIP(hipSetDevice(device_));
    stream_ = stream;
    EECMG_HIP(hipMalloc(&d_desc_, sizeof(JobDesc) * kMaxSlots * kMaxLevels));
    EECMG_HIP(hipMalloc(&d_state_, sizeof(SolverState) * kMaxSlots));
    EECMG_HIP(hipMalloc(&d_rec_, sizeof(LevelRecord) * kMaxSlots * kMaxLevels));
    EECMG_HIP(hipMemset(d_state_, 0, sizeof(SolverState) * kMaxSlots));
    // descriptors and taps are staged in fine-grained pinned memory that
    // k_upload reads directly (no stale device-cached copies)
    EECMG_HIP(hipHostMalloc((void**)&h_desc_, sizeof(JobDesc) * kMaxSlots * kMaxLevels, hipHostMallocCoherent));
    EECMG_HIP(hipHostGetDevicePointer((void**)&dv_desc_, (void*)h_desc_, 0));
    EECMG_HIP(hipHostMalloc((void**)&h_rec_, sizeof(LevelRecord) * kMaxSlots * kMaxLevels, hipHostMallocDefault));
    EECMG_HIP(hipHostMalloc((void**)&h_taps_, kTapsSlotBytes * kMaxSlots, hipHostMallocCoherent));
    EECMG_HIP(hipHostGetDevicePointer((void**)&dv_taps_, (void*)h_taps_, 0));
    EECMG_HIP(hipHostMalloc((void**)&h_mirror_, sizeof(uint64_t) * kMaxSlots, hipHostMallocCoherent));
    std::memset((void*)h_mirror_, 0, sizeof(uint64_t) * kMaxSlots);
    EECMG_HIP(hipHostGetDevicePointer((void**)&d_mirror_, (void*)h_mirror_, 0));
    for (auto& e : step_ev_) EECMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    slots_.assign(kMaxSlots, nullptr);
    return EECMG_OK;
  }

  // An engine that allocates no device or pinned memory: its descriptor
  // table, solver state, level records, progress words and job arena are
  // carved from the device region [dev, dev + bytes) (256-byte aligned), its
  // host-side tables are ordinary host memory, and it serves one job at a
  // time.  The progress words then live in device memory: the engine reads
  // them with a copy after draining its stream (wait_some), so a level's
  // schedule advances in steps of at most two iterations per drain.
  // Returns EINVAL when the region cannot hold the tables.
  int init_noalloc(char* dev, size_t bytes) {
    EECMG_HIP(hipSetDevice(device_));
    noalloc_ = true;
    n_slots_ = 1;
    size_t off = 0;
    auto carve = [&](size_t n) {
      char* p = dev + off;
      off = align_up(off + n, 256);
      return p;
    };
    d_desc_ = (JobDesc*)carve(sizeof(JobDesc) * kMaxLevels);
    d_state_ = (SolverState*)carve(sizeof(SolverState));
    d_rec_ = (LevelRecord*)carve(sizeof(LevelRecord) * kMaxLevels);
    d_mirror_ = (uint64_t*)carve(sizeof(uint64_t));
    if (off >= bytes) return fail(EECMG_EINVAL, "scratch region too small for the engine tables");
    arena_.adopt(dev + off, bytes - off);
    noalloc_tables_.assign(sizeof(JobDesc) * kMaxLevels + sizeof(LevelRecord) * kMaxLevels + kTapsSlotBytes +
                               sizeof(uint64_t) + 3 * 256,
                           0);
    char* h = noalloc_tables_.data();
    h = (char*)align_up((uintptr_t)h, 256);
    h_desc_ = (JobDesc*)h;
    h += align_up(sizeof(JobDesc) * kMaxLevels, 256);
    h_rec_ = (LevelRecord*)h;
    h += align_up(sizeof(LevelRecord) * kMaxLevels, 256);
    h_taps_ = h;
    h += kTapsSlotBytes;
    h_mirror_ = (volatile uint64_t*)h;
    dv_desc_ = nullptr;  // k_upload is never used (one job: two copies)
    dv_taps_ = nullptr;
    for (auto& e : step_ev_) EECMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    out_ev_ = std::make_shared<HipEvent>();
    slots_.assign(n_slots_, nullptr);
    return EECMG_OK;
  }
  size_t arena_capacity() const { return arena_.size(); }
  // Clear the solver state and progress word of the engine's one slot (a
  // fill kernel on the stream: the region keeps the previous call's bytes).
  int clear_noalloc_state() {
    EECMG_HIP(launch_zero_words(d_state_, sizeof(SolverState) / 4, stream_));
    EECMG_HIP(launch_zero_words(d_mirror_, sizeof(uint64_t) / 4, stream_));
    h_mirror_[0] = 0;
    return EECMG_OK;
  }

  // Free the engine's own device and pinned memory (the arena is released
  // separately).  No job may be active.
  void shutdown() {
    if (d_desc_) (void)hipFree(d_desc_);
    if (d_state_) (void)hipFree(d_state_);
    if (d_rec_) (void)hipFree(d_rec_);
    if (h_desc_) (void)hipHostFree(h_desc_);
    if (h_rec_) (void)hipHostFree(h_rec_);
    if (h_taps_) (void)hipHostFree(h_taps_);
    if (h_mirror_) (void)hipHostFree((void*)h_mirror_);
    h_mirror_ = nullptr;
    for (auto& e : step_ev_) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
    d_desc_ = nullptr;
    d_state_ = nullptr;
    d_rec_ = nullptr;
    h_desc_ = nullptr;
    h_rec_ = nullptr;
    h_taps_ = nullptr;
  }

  void set_stream(hipStream_t s) { stream_ = s; }
  // Host<->device copies of served requests go to this stream (NULL: the
  // compute stream), so they overlap other requests' kernels.
  void set_copy_stream(hipStream_t s) { copy_ = s; }
  // The job's input was enqueued on stream s: its first kernel waits for it.
  int mark_input(Job* j, hipStream_t s) {
    if (!j->in_ev && hipEventCreateWithFlags(&j->in_ev, hipEventDisableTiming) != hipSuccess) return EECMG_EDEVICE;
    if (hipEventRecord(j->in_ev, s) != hipSuccess) return EECMG_EDEVICE;
    j->in_wait = true;
    return EECMG_OK;
  }
  // First HIP error met by an asynchronous call (sticky), and its reset.
  hipError_t error() const { return err_; }
  void clear_error() { err_ = hipSuccess; }
  hipStream_t stream() const { return stream_; }
  Arena& arena() { return arena_; }
  int active() const { return n_active_; }

  // Give the job a slot and device memory; upload its per-level descriptors.
  // EAGAIN when no slot or memory is free right now.
  int admit(Job* j) {
    int slot = -1;
    for (int i = 0; i < n_slots_; ++i)
      if (!slots_[i]) {
        slot = i;
        break;
      }
    if (slot < 0) return EECMG_EAGAIN;
    char* mem = (char*)arena_.alloc(j->plan.bytes);
    if (!mem) return EECMG_EAGAIN;
    j->slot = slot;
    j->mem = mem;
    j->uid = (next_uid_++) & 0xFFFFFF;
    // the slot's previous occupant has no kernels left (its completion event
    // was seen): clear its progress word so that a stale word with the same
    // tag can never be taken for this job's
    __atomic_store_n(&h_mirror_[slot], (uint64_t)0, __ATOMIC_RELEASE);
    slots_[slot] = j;
    ++n_active_;
    j->phase = Job::kNew;
    j->oi = 0;
    // taps (element type of the precision, and flipped for H^T), staged in
    // this slot's pinned buffer and copied with the descriptors
    const Plan& P = j->plan;
    char* tb = h_taps_ + (size_t)slot * kTapsSlotBytes;
    for (int l = 0; l < P.L; ++l) {
      const LevelPlan& lp = P.lv[l];
      for (size_t k = 0; k < lp.taps.size(); ++k) {
        if (P.f64) {
          ((double*)(tb + P.off_taps[l]))[k] = lp.taps[k];
          ((double*)(tb + P.off_tapst[l]))[k] = lp.taps_t[k];
        } else {
          ((float*)(tb + P.off_taps[l]))[k] = (float)lp.taps[k];
          ((float*)(tb + P.off_tapst[l]))[k] = (float)lp.taps_t[k];
        }
      }
    }
    if (P.own_gin) j->g_in_dev = mem + P.off_gin;
    if (P.own_uout) j->u_out_dev = mem + P.off_uout;
    alias_io(j);
    JobDesc* hd = h_desc_ + (size_t)slot * kMaxLevels;
    for (int l = 0; l < P.L; ++l) fill_desc(j, l, hd[l]);
    j->needs_upload = true;  // copied by the next step's k_upload
    return EECMG_OK;
  }

  // Issue one round of work for every active job.  Returns true if anything
  // was launched.
  bool step(std::vector<Job*>& finished) {
    if (paced()) {
      // the device still has pace_ steps queued: only report finished jobs
      finished.clear();
      for (Job* j : slots_)
        if (j && j->phase == Job::kWaitOut && event_done(j->done_ev->e)) {
          finish(j);
          finished.push_back(j);
        }
      return false;
    }
    const bool idle_before = !step_pending_;  // everything enqueued so far had completed
    const uint64_t progress_before = progress_sum();
    poll_mirror();
    finished.clear();
    if (fail_step_ > 0 && ++steps_ == fail_step_ && err_ == hipSuccess) {
      // test hook (EECMG_TEST_FAIL_STEP): a HIP error reported by this step,
      // without any kernel being affected
      err_ = hipErrorUnknown;
      return false;
    }
    // action lists
    std::vector<Job*> restrict_l, out_l;
    std::vector<std::pair<Job*, int>> xfer_l;  // job, level
    std::vector<Job*> init_l;
    std::vector<std::pair<Job*, int>> iter_l;  // job, chunk
    std::vector<std::pair<Job*, int>> flush_l;  // job, level left with a possibly deferred update
    std::vector<std::pair<Job*, int>> finb_l;   // job, level left with its last finalize still to run
    std::vector<std::pair<Job*, int>> fini_l;   // job, level left before its first iteration, init owed
    bool launched = false;
    for (int s = 0; s < n_slots_; ++s) {
      Job* j = slots_[s];
      if (!j) continue;
      bool again = true, started = false;
      while (again) {
        again = false;
        switch (j->phase) {
          case Job::kNew:
            restrict_l.push_back(j);
            j->phase = Job::kStartLevel;
            j->oi = 0;
            if (j->plan.coarse > 0) {
              // the leading small levels are solved by the restriction
              // launch, stream-ordered before everything issued for the
              // levels after them
              j->oi = j->plan.coarse;
              if (j->oi >= (int)j->plan.order.size()) {
                out_l.push_back(j);
                j->phase = Job::kOutput;
                break;
              }
            }
            again = true;
            break;
          case Job::kStartLevel: {
            // at most one level start per job and step: the launches of one
            // step are grouped by stage, so a second level would run its
            // transfer before the first level's initialisation
            if (started) break;
            started = true;
            const int l = j->cur_level();
            if (needs_transfer(j, l)) xfer_l.push_back({j, l});
            init_l.push_back(j);
            j->issued = 0;
            j->confirmed = 0;
            j->next_chunk = 1;
            j->level_done_seen = false;
            j->phase = Job::kIter;
            again = true;
            break;
          }
          case Job::kIter: {
            // launches per level: CGLS needs cap iterations; MR needs one
            // more pass, because its first pass only forms q = H r
            const int limit = j->plan.lv[j->cur_level()].cap + (j->plan.prm.smoother == EECMG_SMOOTHER_MR ? 1 : 0);
            if (j->cancelled || j->level_done_seen || j->issued >= limit) {
              // the last pass B's finalize is still owed -- unless the stop was
              // already seen: that finalize would then find the level stopped
              // and do nothing
              if (j->owed == Job::kOwesB && !j->level_done_seen) finb_l.push_back({j, j->cur_level()});
              if (j->owed == Job::kOwesInit && !j->cancelled) fini_l.push_back({j, j->cur_level()});
              j->owed = Job::kOwesNone;
              if (lazy_level(j, j->cur_level())) flush_l.push_back({j, j->cur_level()});
              if (!j->cancelled && j->oi + 1 < (int)j->plan.order.size()) {
                j->oi += 1;
                j->phase = Job::kStartLevel;
                again = !started;
              } else {
                out_l.push_back(j);
                j->phase = Job::kOutput;
              }
              break;
            }
            // keep at most kMaxAhead unconfirmed iterations queued: enough to
            // hide the host's reaction time, few enough that a data-dependent
            // stop leaves almost no empty launches behind
            const int ahead = j->issued - j->confirmed;
            const int chunk = std::min(limit - j->issued, max_ahead_ - ahead);
            if (chunk > 0) {
              iter_l.push_back({j, chunk});
              j->issued += chunk;
            }
            break;
          }
          case Job::kWaitOut:
            if (event_done(j->done_ev->e)) {
              finish(j);
              finished.push_back(j);
            }
            break;
          default: break;
        }
      }
    }
    // launches, in dependency order; first the newly admitted jobs' tables:
    // one job's by two copies, several jobs' by one upload kernel
    {
      UploadList ul;
      ul.n = 0;
      for (int s = 0; s < n_slots_; ++s)
        if (slots_[s] && slots_[s]->needs_upload) {
          slots_[s]->needs_upload = false;
          ul.slot[ul.n++] = s;
        }
      if (ul.n == 1) {
        const Job* j = slots_[ul.slot[0]];
        const size_t so = (size_t)j->slot;
        chk(hipMemcpyAsync(j->mem, h_taps_ + so * kTapsSlotBytes, j->plan.taps_bytes, hipMemcpyHostToDevice,
                           stream_));
        chk(hipMemcpyAsync(d_desc_ + so * kMaxLevels, h_desc_ + so * kMaxLevels, sizeof(JobDesc) * j->plan.L,
                           hipMemcpyHostToDevice, stream_));
      } else if (ul.n > 1) {
        chk(launch_upload(ul, dv_desc_, d_desc_, dv_taps_, kTapsSlotBytes, stream_));
      }
    }
    if (!restrict_l.empty()) {
      for (Job* j : restrict_l)
        if (j->in_wait) {
          chk(hipStreamWaitEvent(stream_, j->in_ev, 0));
          j->in_wait = false;
        }
      // one launch per precision restricts every level and solves the
      // leading coarse levels (level 0's descriptor: the restriction fields
      // are the same on every level, and a job whose levels are all coarse
      // has no current level)
      for (int f64 = 0; f64 < 2; ++f64) {
        std::vector<Job*> js;
        for (Job* j : restrict_l)
          if ((int)j->plan.f64 == f64) js.push_back(j);
        if (!js.empty()) launch_group(kRestrict, js, 0, f64 != 0, 0, -1, -1);
      }
      launched = true;
    }
    for (auto* fl : {&fini_l, &finb_l}) {
      // the finalize of each level's last pass B (its records, stop reason and
      // iteration count; a level that already stopped leaves it unchanged),
      // or of an initialisation no iteration followed
      if (fl->empty()) continue;
      std::vector<Job*> js;
      std::vector<int> lv;
      for (auto& x : *fl) {
        js.push_back(x.first);
        lv.push_back(x.second);
      }
      launch_group(fl == &fini_l ? kCgFinInit : kCgFinB, js, -1, false, 0, -1, -1, nullptr, &lv);
      launched = true;
    }
    if (!flush_l.empty()) {
      // stream-ordered after the level's last pass, before anything reads u
      for (int f64 = 0; f64 < 2; ++f64) {
        std::vector<Job*> js;
        std::vector<int> lv;
        for (auto& x : flush_l)
          if ((int)x.first->plan.f64 == f64) {
            js.push_back(x.first);
            lv.push_back(x.second);
          }
        if (!js.empty()) launch_group(kFlushU, js, -1, f64 != 0, 0, -1, -1, nullptr, &lv);
      }
      launched = true;
    }
    if (!xfer_l.empty()) {
      issue_transfers(xfer_l);
      launched = true;
    }
    if (!init_l.empty()) {
      issue_inits(init_l);
      launched = true;
    }
    if (!iter_l.empty()) {
      issue_iterations(iter_l);
      launched = true;
    }
    if (!out_l.empty()) {
      // outputs of every job finishing in this step: one copy launch per
      // precision, one read-back of the level records, one shared event
      // (served requests copy their results on the copy stream instead)
      int lo = n_slots_, hi = -1;
      for (int f64 = 0; f64 < 2; ++f64) {
        std::vector<Job*> js;
        std::vector<int> lv;
        for (Job* j : out_l)
          if ((int)j->plan.f64 == f64 && !j->alias_out) {
            js.push_back(j);
            lv.push_back(j->plan.L - 1);
          }
        if (!js.empty()) launch_group(kOutCopy, js, -1, f64 != 0, 0, -1, -1, nullptr, &lv);
      }
      for (Job* j : out_l) {
        lo = std::min(lo, j->slot);
        hi = std::max(hi, j->slot);
      }
      chk(hipMemcpyAsync(h_rec_ + (size_t)lo * kMaxLevels, d_rec_ + (size_t)lo * kMaxLevels,
                         sizeof(LevelRecord) * kMaxLevels * (size_t)(hi - lo + 1), hipMemcpyDeviceToHost, stream_));
      std::shared_ptr<HipEvent> shared;
      for (Job* j : out_l) {
        const size_t out_bytes = (size_t)j->plan.H * j->plan.W * j->plan.esz;
        if (j->host_out && copy_) {
          if (!j->comp_ev) chk(hipEventCreateWithFlags(&j->comp_ev, hipEventDisableTiming));
          chk(hipEventRecord(j->comp_ev, stream_));
          chk(hipStreamWaitEvent(copy_, j->comp_ev, 0));
          chk(hipMemcpyAsync(j->host_out, j->u_out_dev, out_bytes, hipMemcpyDeviceToHost, copy_));
          j->done_ev = std::make_shared<HipEvent>();
          chk(hipEventRecord(j->done_ev->e, copy_));
        } else {
          if (j->host_out) chk(hipMemcpyAsync(j->host_out, j->u_out_dev, out_bytes, hipMemcpyDeviceToHost, stream_));
          if (!shared) shared = noalloc_ ? out_ev_ : std::make_shared<HipEvent>();
          j->done_ev = shared;
        }
        j->phase = Job::kWaitOut;
      }
      if (shared) chk(hipEventRecord(shared->e, stream_));
      launched = true;
    }
    if (launched) {
      step_cur_ = (step_cur_ + 1) % kStepEvents;
      chk(hipEventRecord(step_ev_[step_cur_], stream_));
      step_pending_ = true;
      n_out_ = std::min(n_out_ + 1, kStepEvents - 1);
    }
    note_progress(launched || !finished.empty() || progress_sum() != progress_before || !idle_before);
    return launched;
  }

  // Wait until the device reports progress for some job (through the pinned
  // progress words) or all enqueued work has completed.
  void wait_some() {
    if (noalloc_) {
      // progress words in device memory: read them behind everything
      // enqueued, on the engine's stream, and drain it
      chk(hipMemcpyAsync((void*)h_mirror_, d_mirror_, sizeof(uint64_t) * n_slots_, hipMemcpyDeviceToHost, stream_));
      chk(hipStreamSynchronize(stream_));
      step_pending_ = false;
      return;
    }
    if (paced()) {
      // wait for the oldest queued step (or a job's output) instead of the
      // next progress word: the jobs confirmed meanwhile then share launches
      for (long spin = 0; paced() && err_ == hipSuccess; ++spin) {
        for (Job* j : slots_)
          if (j && j->phase == Job::kWaitOut && event_done(j->done_ev->e)) return;
        if (spin > 2000) std::this_thread::yield();
      }
      return;
    }
    const std::vector<uint64_t> before = snapshot();
    for (long spin = 0;; ++spin) {
      if (snapshot() != before) return;
      for (Job* j : slots_)
        if (j && j->phase == Job::kWaitOut && event_done(j->done_ev->e)) return;
      if (!step_pending_ || event_done(step_ev_[step_cur_])) {
        step_pending_ = false;
        return;
      }
      if (err_ != hipSuccess) return;
      if (spin > 2000) std::this_thread::yield();
    }
  }

  // Release a finished job's slot and memory.
  void release(Job* j) {
    if (j->slot >= 0) {
      slots_[j->slot] = nullptr;
      --n_active_;
    }
    if (j->mem) arena_.free(j->mem, j->plan.bytes);
    j->mem = nullptr;
    j->slot = -1;
    j->done_ev.reset();
    for (hipEvent_t* e : {&j->in_ev, &j->comp_ev}) {
      if (*e) (void)hipEventDestroy(*e);
      *e = nullptr;
    }
    j->in_wait = false;
  }

  int device() const { return device_; }

 private:
  // Unconfirmed iterations a job may have queued.  At least 2: with folded
  // finalizes, iteration k's progress word is published by iteration k + 1's
  // pass A, so a single iteration in flight would wait for itself.  Deeper
  // run-ahead only adds empty launches after a level stops (measured slower).
  // EECMG_MAX_AHEAD moves it (1..8); 1 stalls on levels with folded
  // finalizes, which the stall guard then reports (its test uses that).
  static constexpr int kMaxAhead = 2;
  static_assert(kMaxAhead >= 2, "folded finalizes confirm an iteration only from the next one");

 public:
  // Re-read the environment knobs of the scheduler (once per driver call).
  void read_knobs() {
    const char* e = std::getenv("EECMG_MAX_AHEAD");
    max_ahead_ = e ? std::min(8, std::max(1, std::atoi(e))) : kMaxAhead;
    e = std::getenv("EECMG_STALL_STEPS");
    stall_steps_ = e ? std::max(0L, std::atol(e)) : kStallSteps;
    e = std::getenv("EECMG_STALL_MS");
    stall_ms_ = e ? std::max(0.0, std::atof(e)) : kStallMs;
    e = std::getenv("EECMG_TEST_FAIL_STEP");
    fail_step_ = e ? std::atol(e) : 0;
    fold_max_jobs_ = fold_max_jobs();
    e = std::getenv("EECMG_PACE_STEPS");
    pace_ = e ? std::min(kStepEvents - 1, std::max(0, std::atoi(e))) : kPaceSteps;
    steps_ = 0;
  }
  // The engine can make no further progress: a HIP error was reported, or the
  // stall guard tripped.  Returns the status and message for the callers.
  bool failed() const { return err_ != hipSuccess || stalled_; }
  std::string failure() const {
    if (err_ != hipSuccess) return std::string("HIP error in the cascade: ") + hipGetErrorString(err_);
    return "scheduler stall: no kernel to launch, no progress and the device idle for " +
           std::to_string(idle_steps_) + " steps";
  }
  // After failed(): wait for the device to finish (or fail) everything
  // enqueued, mark every admitted job that has not finished with `status`,
  // free their slots and memory and append them to `out`, and clear the error
  // state so that the engine can be used again.
  void abort_all(int status, std::vector<Job*>& out) {
    (void)hipStreamSynchronize(stream_);
    if (copy_) (void)hipStreamSynchronize(copy_);
    (void)hipGetLastError();
    for (Job* j : slots_) {
      if (!j || j->phase == Job::kFinished) continue;  // finished ones are the caller's to release
      j->status = status;
      j->phase = Job::kFinished;
      j->t_done = now_s();
      release(j);
      out.push_back(j);
    }
    for (int i = 0; i < n_slots_; ++i) __atomic_store_n(&h_mirror_[i], (uint64_t)0, __ATOMIC_RELEASE);
    err_ = hipSuccess;
    stalled_ = false;
    step_pending_ = false;
    n_out_ = 0;
    idle_steps_ = 0;
  }

 private:
  // A job cannot advance when nothing was launched, no job finished, no
  // progress word changed and the device had completed all enqueued work
  // before the step.  In a correct schedule that resolves at once (the
  // progress words of completed work are visible), so it persisting for
  // stall_steps_ consecutive steps and stall_ms_ milliseconds is a stall.
  static constexpr long kStallSteps = 1000;
  static constexpr double kStallMs = 1000.0;
  void note_progress(bool progress) {
    // a job waiting for its output copy waits for an event that completes
    for (const Job* j : slots_)
      if (j && j->phase == Job::kWaitOut) progress = true;
    if (progress || n_active_ == 0) {
      idle_steps_ = 0;
      return;
    }
    if (idle_steps_++ == 0) idle_since_ = now_s();
    if (idle_steps_ >= stall_steps_ && (now_s() - idle_since_) * 1e3 >= stall_ms_) stalled_ = true;
  }
  uint64_t progress_sum() const {
    uint64_t h = 0;
    for (int i = 0; i < n_slots_; ++i) h = h * 1000003u + __atomic_load_n(&h_mirror_[i], __ATOMIC_ACQUIRE);
    return h;
  }
  // hipEventQuery: complete, not yet, or an error (recorded as the engine's
  // error, which the drivers then report).
  bool event_done(hipEvent_t e) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) return true;
    if (r != hipErrorNotReady) chk(r);
    return false;
  }

  static constexpr int kStepEvents = 4;

  // Step pacing.  Every step that launches records one of kStepEvents
  // events; n_out_ counts those not yet seen complete (they complete in
  // order, so only the oldest is polled).  While pace_ steps are queued on
  // the device, no new step launches: jobs confirmed in the meantime are
  // issued together in the next step, one launch per stage for all of them,
  // instead of one small launch each time a progress word changes.  The
  // queued steps keep the device busy while the host builds the next one.
  // Without it a batch of many jobs splits into groups that drift apart and
  // the host spends its time issuing launches of one or two jobs.
  // EECMG_PACE_STEPS moves the depth (0 = off, at most kStepEvents - 1).
  static constexpr int kPaceSteps = 2;
  int outstanding() {
    while (n_out_ > 0) {
      const int oldest = ((step_cur_ - n_out_ + 1) % kStepEvents + kStepEvents) % kStepEvents;
      if (!event_done(step_ev_[oldest])) break;
      --n_out_;
    }
    return n_out_;
  }
  bool paced() { return pace_ > 0 && !noalloc_ && n_out_ >= pace_ && outstanding() >= pace_; }

  std::vector<uint64_t> snapshot() const {
    std::vector<uint64_t> v(n_slots_);
    for (int i = 0; i < n_slots_; ++i) v[i] = __atomic_load_n(&h_mirror_[i], __ATOMIC_ACQUIRE);
    return v;
  }

  static uint32_t level_tag(const Job* j, int level) { return (j->uid << 8) | (uint32_t)level; }

  // Read the progress words the finalize kernels publish; a word counts only
  // if its tag names this job and its current level.
  void poll_mirror() {
    for (Job* j : slots_) {
      if (!j || j->phase != Job::kIter) continue;
      const uint64_t w = __atomic_load_n(&h_mirror_[j->slot], __ATOMIC_ACQUIRE);
      if ((uint32_t)(w >> 32) != level_tag(j, j->cur_level())) continue;
      const int k = (int)((w >> 8) & 0xFFFFFF), done = (int)(w & 0xFF);
      const int passes = j->plan.prm.smoother == EECMG_SMOOTHER_MR ? k + 1 : k;
      j->confirmed = std::max(j->confirmed, std::min(passes, j->issued));
      if (done != 0) {
        j->level_done_seen = true;
        j->confirmed = j->issued;
      }
    }
  }

  static bool lazy_level(const Job* j, int l) { return j->plan.lv[l].lazy; }

  bool needs_transfer(const Job* j, int l) const {
    return j->plan.prm.cascade == EECMG_CASCADE_EECMG ? l >= 2 : l >= 1;
  }

  // The finest level's right-hand side and solution live in the caller's
  // dense input and output when those already have the level's row pitch and
  // alignment and do not overlap (saves the pitched copy in and out).  An
  // initial guess keeps the separate solution buffer.
  static void alias_io(Job* j) {
    const Plan& P = j->plan;
    const size_t n = (size_t)P.H * P.W * P.esz;
    const char* g = (const char*)j->g_in_dev;
    const char* u = (const char*)j->u_out_dev;
    const bool dense = P.lv[P.L - 1].pitch == P.W;
    const bool disjoint = g && u && (g + n <= u || u + n <= g);
    j->alias_in = dense && disjoint && ((uintptr_t)g & 255) == 0;
    j->alias_out = dense && disjoint && ((uintptr_t)u & 255) == 0 && !j->u_init_dev;
  }

  void fill_desc(const Job* j, int l, JobDesc& d) {
    const Plan& P = j->plan;
    const LevelPlan& lp = P.lv[l];
    char* m = j->mem;
    const int Lf = P.L - 1;
    auto g_at = [&](int k) -> void* {
      return k == Lf && j->alias_in ? const_cast<void*>(j->g_in_dev) : (void*)(m + P.off_g[k]);
    };
    auto u_at = [&](int k) -> void* { return k == Lf && j->alias_out ? j->u_out_dev : (void*)(m + P.off_u[k]); };
    std::memset(&d, 0, sizeof(d));
    d.g = g_at(l);
    d.u = u_at(l);
    d.r[0] = m + P.off_work[0];
    d.r[1] = m + P.off_work[1];
    d.p[0] = m + P.off_work[2];
    d.p[1] = m + P.off_work[3];
    d.s = m + P.off_work[4];
    d.q[0] = m + P.off_work[5];
    d.q[1] = m + P.off_work[6];
    d.taps = m + P.off_taps[l];
    d.taps_t = m + P.off_tapst[l];
    d.h = lp.h;
    d.w = lp.w;
    d.pitch = lp.pitch;
    d.rad = lp.rad;
    d.tiles_x = lp.tiles_x;
    d.ntiles = lp.ntiles;
    d.cap = lp.cap;
    d.level = l;
    d.stop_rule = P.prm.stop_rule;
    d.smoother = P.prm.smoother;
    d.cascade = P.prm.cascade;
    d.pm_steps = P.prm.pm_steps;
    d.coarse_levels = l == 0 ? P.coarse : 0;
    d.lazy_u = lazy_level(j, l) ? 1 : 0;
    d.fold_a = lp.fold_a ? 1 : 0;
    d.nstrips = lp.nstrips;
    for (int k = 0; k < P.L; ++k)
      if (!needs_transfer(j, k)) d.zero_u |= 1 << k;
    d.cdelta = P.prm.c * P.prm.delta;
    d.eps2 = P.eps2;
    d.st = d_state_ + j->slot;
    d.rec = d_rec_ + (size_t)j->slot * kMaxLevels;
    d.partials = (double*)(m + P.off_part);
    d.pstride = P.max_tiles;
    d.mirror = d_mirror_ + j->slot;
    d.tag = level_tag(j, l);
    d.taps_bytes = (int32_t)P.taps_bytes;
    d.f64 = P.f64 ? 1 : 0;
    if (l >= 1) {
      d.uB = u_at(l - 1);
      d.hB = P.lv[l - 1].h;
      d.wB = P.lv[l - 1].w;
      d.pB = P.lv[l - 1].pitch;
    }
    if (l >= 2) {
      d.uA = u_at(l - 2);
      d.hA = P.lv[l - 2].h;
      d.wA = P.lv[l - 2].w;
      d.pA = P.lv[l - 2].pitch;
    }
    // transfer temporaries: the smoother's direction buffers are free then
    d.t1 = m + P.off_work[2];
    d.t2 = m + P.off_work[3];
    d.pm_k = P.k;
    d.tau = P.prm.tau;
    d.smooth_h = P.prm.smooth_h;
    d.g_in = j->g_in_dev;
    d.u_in = j->u_init_dev;
    d.u_out = j->u_out_dev;
    d.H = P.H;
    d.W = P.W;
    d.L = P.L;
    d.fine_pitch = P.lv[P.L - 1].pitch;
    for (int k = 0; k < P.L; ++k) {
      d.g_lv[k] = g_at(k);
      d.u_lv[k] = u_at(k);
      d.lh[k] = P.lv[k].h;
      d.lw[k] = P.lv[k].w;
      d.lp[k] = P.lv[k].pitch;
    }
  }

  // Launch `stage` for jobs at the given level (-1: each job's current level),
  // splitting by nothing: caller groups jobs of one precision / variant.
  void launch_group(Stage st, const std::vector<Job*>& jobs, int level, bool f64, int variant, int src, int dst,
                    const std::vector<int>* kidx = nullptr, const std::vector<int>* levels = nullptr,
                    int flags = 0, const std::vector<int>* kfold = nullptr) {
    LaunchList ll;
    ll.n = 0;
    ll.total = 0;
    ll.flags = flags;
    ll.pad = 0;
    auto level_of = [&](size_t i) { return levels ? (*levels)[i] : level >= 0 ? level : jobs[i]->cur_level(); };
    for (size_t i = 0; i < jobs.size(); ++i) {
      Job* j = jobs[i];
      const int l = level_of(i);
      if (l < 0 || l >= j->plan.L) {  // never launch with a descriptor that does not exist
        if (err_ == hipSuccess) err_ = hipErrorInvalidValue;
        return;
      }
      const int di = j->slot * kMaxLevels + l;
      const JobDesc& hd = h_desc_[di];
      ll.job[ll.n] = di;
      ll.kf[ll.n] = kfold ? (*kfold)[i] : -1;
      ll.start[ll.n] = ll.total;
      ll.total += blocks_for_stage(st, hd);
      ll.n += 1;
      f64 = j->plan.f64;
    }
    ll.start[ll.n] = ll.total;
    // (the restriction launch also has one head block per job)
    if (ll.total <= 0 && !(st == kRestrict && ll.n > 0)) return;
    Profiler& pr = profiler();
    double px = 0.0;
    const bool prof = !noalloc_ && pr.on.load(std::memory_order_relaxed) && profiled_stage(st) &&
                      ll.total >= pr.min_blocks;
    if (prof)
      for (size_t i = 0; i < jobs.size(); ++i) {
        const Job* j = jobs[i];
        const int l = level_of(i);
        px += st == kXfExtrap ? (double)j->plan.lv[l - 1].h * j->plan.lv[l - 1].w
                              : (double)j->plan.lv[l].h * j->plan.lv[l].w;
      }
    if (prof && px >= pr.min_pixels) {
      std::lock_guard<std::mutex> g(pr.mu);
      hipEvent_t a = pr.ev(), b = pr.ev();
      chk(hipEventRecord(a, stream_));
      chk(launch_stage(st, f64, variant, ll, d_desc_, src, dst, stream_));
      chk(hipEventRecord(b, stream_));
      // the level the launch works on (restriction and output copy: none)
      int lvl = (st == kRestrict || st == kOutCopy || jobs.empty()) ? -1 : level_of(0);
      for (size_t i = 1; i < jobs.size() && lvl >= 0; ++i)
        if (level_of(i) != lvl) lvl = -1;
      Profiler::Rec rec{(int)st, a, b, px, {}, lvl};
      if (kidx)
        for (size_t i = 0; i < jobs.size(); ++i)
          rec.tags.push_back({jobs[i]->uid, jobs[i]->cur_level(), (*kidx)[i], st == kMrPass});
      pr.pending.push_back(std::move(rec));
      return;
    }
    chk(launch_stage(st, f64, variant, ll, d_desc_, src, dst, stream_));
  }

  static int variant_key(const Job* j) {
    const int l = j->cur_level();
    return (j->plan.f64 ? 100000 : 0) + j->plan.lv[l].variant;
  }

  void issue_transfers(const std::vector<std::pair<Job*, int>>& xs) {
    // group by (precision, cascade, pm_steps, small level)
    std::map<std::tuple<int, int, int, int>, std::vector<Job*>> groups;
    for (auto& x : xs) {
      const Job* j = x.first;
      const LevelPlan& lv = j->plan.lv[j->cur_level()];
      const bool small = ((lv.h + 31) / 32) * ((lv.w + 63) / 64) < 256;
      groups[{j->plan.f64, j->plan.prm.cascade, j->plan.prm.pm_steps, small}].push_back(x.first);
    }
    for (auto& kv : groups) {
      const bool f64 = std::get<0>(kv.first);
      const int cascade = std::get<1>(kv.first), n = std::get<2>(kv.first);
      const Stage fused = std::get<3>(kv.first) ? kXfFusedSmall : kXfFused;
      auto& js = kv.second;
      // EECMG: Pi into t2, then P, S and the first D step fused (t2 -> u);
      // IECMG-P / IECMG-L prolong the level below directly.  Further D
      // steps ping-pong between the two work buffers and end in u.
      if (cascade == EECMG_CASCADE_EECMG) launch_group(kXfExtrap, js, -1, f64, 0, -1, kBufT2);
      const int fsrc = cascade == EECMG_CASCADE_EECMG ? kBufT2 : kBufUB;
      const int fvar = (cascade != EECMG_CASCADE_IECMG_L ? 1 : 0) | (n >= 1 ? 2 : 0);
      int cur = n <= 1 ? kBufU : (fsrc == kBufT2 ? kBufT1 : kBufT2);
      launch_group(fused, js, -1, f64, fvar, fsrc, cur);
      for (int s = 1; s < n; ++s) {
        const int nxt = (s == n - 1) ? kBufU : (cur == kBufT1 ? kBufT2 : kBufT1);
        launch_group(kXfPm, js, -1, f64, 0, cur, nxt);
        cur = nxt;
      }
    }
  }

  void launch_fin(Stage st, const std::vector<Job*>& jobs) {
    if (!jobs.empty()) launch_group(st, jobs, -1, jobs.front()->plan.f64, 0, -1, -1);
  }

  // The initialisation of each group's level, then one finalize launch for
  // the jobs whose level cannot fold it into its first pass A (see
  // issue_iterations); the others owe it.
  void issue_inits(const std::vector<Job*>& js) {
    std::map<std::pair<int, int>, std::vector<Job*>> groups;  // (smoother, variant)
    for (Job* j : js) groups[{j->plan.prm.smoother, variant_key(j)}].push_back(j);
    std::vector<Job*> fin_cg, fin_mr;
    for (auto& kv : groups) {
      const bool f64 = kv.first.second >= 100000;
      const int rc = kv.first.second % 100000;
      if (kv.first.first == EECMG_SMOOTHER_CGLS) {
        // a one-tap blur on the general tiles forms s in the first launch
        const int kind = variant_kind(rc);
        const bool general = kind == kConvGeneral || kind == kConvGenShort;
        std::vector<Job*> need_s;
        for (Job* j : kv.second)
          if (!general || j->plan.lv[j->cur_level()].rad != 0) need_s.push_back(j);
        launch_group(kCgInit1, kv.second, -1, f64, rc, -1, -1, nullptr, nullptr, general ? kLaunchInitS : 0);
        if (!need_s.empty()) launch_group(kCgInit2, need_s, -1, f64, rc, -1, -1);
        for (Job* j : kv.second) {
          const LevelPlan& lp = j->plan.lv[j->cur_level()];
          if (lp.fold_a && lp.cap >= 1)
            j->owed = Job::kOwesInit;
          else
            fin_cg.push_back(j);
        }
      } else {
        launch_group(kMrInit, kv.second, -1, f64, rc, -1, -1);
        fin_mr.insert(fin_mr.end(), kv.second.begin(), kv.second.end());
      }
    }
    launch_fin(kCgFinInit, fin_cg);
    launch_fin(kMrFinInit, fin_mr);
  }

  // One round of iterations per chunk index.  Jobs are grouped by smoother
  // and blur kernel.  A CGLS group of a single job on a fold_a level folds
  // its finalizes into the passes: its pass B evaluates pass A's finalize,
  // and its next pass A the one it owes (the previous pass B's, or at
  // iteration 0 the initialisation's).  A launch shared by several jobs does
  // not fold (every block would repeat its job's whole partial sum, which
  // costs more than the one finalize launch all of them share): the
  // finalizes such jobs owe are launched first, then every group's pass A,
  // one finalize launch for the groups that do not fold, every pass B and
  // again one finalize launch.  The finalize kernels are precision- and
  // kernel-independent, so one launch serves jobs of every group.
  void issue_iterations(const std::vector<std::pair<Job*, int>>& its) {
    int maxc = 0;
    for (auto& x : its) maxc = std::max(maxc, x.second);
    for (int it = 0; it < maxc; ++it) {
      struct Group {
        std::vector<Job*> js;
        std::vector<int> ks;  // iteration index per job
        bool fold = false;
      };
      std::map<std::pair<int, int>, Group> groups;  // (smoother, variant)
      for (auto& x : its)
        if (x.second > it) {
          Group& g = groups[{x.first->plan.prm.smoother, variant_key(x.first)}];
          g.js.push_back(x.first);
          g.ks.push_back(x.first->issued - x.second + it);
        }
      std::vector<Job*> owe_init, owe_b;
      for (auto& kv : groups) {
        Group& g = kv.second;
        g.fold = kv.first.first == EECMG_SMOOTHER_CGLS && (int)g.js.size() <= fold_max_jobs_;
        for (Job* j : g.js) g.fold = g.fold && j->plan.lv[j->cur_level()].fold_a;
        if (g.fold) continue;
        for (Job* j : g.js) {
          if (j->owed == Job::kOwesInit) owe_init.push_back(j);
          if (j->owed == Job::kOwesB) owe_b.push_back(j);
          j->owed = Job::kOwesNone;
        }
      }
      launch_fin(kCgFinInit, owe_init);
      launch_fin(kCgFinB, owe_b);
      std::vector<Job*> fin_a, fin_b, fin_m;
      for (auto& kv : groups) {
        if (kv.first.first != EECMG_SMOOTHER_CGLS) continue;
        const bool f64 = kv.first.second >= 100000;
        const int rc = kv.first.second % 100000;
        Group& g = kv.second;
        if (g.fold) {
          std::vector<int> kf(g.js.size());
          for (size_t i = 0; i < g.js.size(); ++i) {
            kf[i] = g.js[i]->owed == Job::kOwesNone ? -1 : g.ks[i];
            g.js[i]->owed = Job::kOwesNone;  // evaluated by this pass A
          }
          launch_group(kCgA, g.js, -1, f64, rc, -1, -1, &g.ks, nullptr, kLaunchFoldB, &kf);
        } else {
          launch_group(kCgA, g.js, -1, f64, rc, -1, -1, &g.ks);
          fin_a.insert(fin_a.end(), g.js.begin(), g.js.end());
        }
      }
      launch_fin(kCgFinA, fin_a);
      for (auto& kv : groups) {
        if (kv.first.first != EECMG_SMOOTHER_CGLS) continue;
        const bool f64 = kv.first.second >= 100000;
        const int rc = kv.first.second % 100000;
        Group& g = kv.second;
        launch_group(kCgB, g.js, -1, f64, rc, -1, -1, &g.ks, nullptr, g.fold ? kLaunchFoldA : 0);
        if (g.fold)
          for (Job* j : g.js) j->owed = Job::kOwesB;  // the next pass A, or the level end, runs it
        else
          fin_b.insert(fin_b.end(), g.js.begin(), g.js.end());
      }
      launch_fin(kCgFinB, fin_b);
      // a deferred-update level whose iteration closes a group of kPRing - 1
      // terms applies them before the next pass A reuses the oldest slot
      for (int f64 = 0; f64 < 2; ++f64) {
        std::vector<Job*> fj;
        std::vector<int> fk;
        for (auto& kv : groups) {
          if (kv.first.first != EECMG_SMOOTHER_CGLS || (kv.first.second >= 100000) != (f64 != 0)) continue;
          const Group& g = kv.second;
          for (size_t i = 0; i < g.js.size(); ++i)
            if (lazy_level(g.js[i], g.js[i]->cur_level()) && g.ks[i] % (kPRing - 1) == kPRing - 2) {
              fj.push_back(g.js[i]);
              fk.push_back(g.ks[i]);
            }
        }
        if (!fj.empty()) launch_group(kFlushU, fj, -1, f64 != 0, 0, -1, -1, nullptr, nullptr, 0, &fk);
      }
      for (auto& kv : groups) {
        if (kv.first.first == EECMG_SMOOTHER_CGLS) continue;
        const bool f64 = kv.first.second >= 100000;
        const int rc = kv.first.second % 100000;
        launch_group(kMrPass, kv.second.js, -1, f64, rc, -1, -1, &kv.second.ks);
        fin_m.insert(fin_m.end(), kv.second.js.begin(), kv.second.js.end());
      }
      launch_fin(kMrFin, fin_m);
    }
  }

  void finish(Job* j) {
    std::memcpy(j->rec, h_rec_ + (size_t)j->slot * kMaxLevels, sizeof(LevelRecord) * kMaxLevels);
    {
      Profiler& pr = profiler();
      std::lock_guard<std::mutex> g(pr.mu);
      // (only while profiling: a long-running context would grow the map)
      if (pr.on.load(std::memory_order_relaxed) || !pr.pending.empty())
        for (int l = 0; l < j->plan.L; ++l) pr.final_iters[((uint64_t)j->uid << 8) | (uint64_t)l] = j->rec[l].iters;
    }
    int st = EECMG_OK;
    for (int l = 0; l < j->plan.L; ++l)
      if (j->rec[l].reason == kStopNonFinite) st = EECMG_ENUMERIC;
    if (j->cancelled) st = EECMG_ECANCELED;
    j->status = st;
    j->phase = Job::kFinished;
    j->t_done = now_s();
  }

  void chk(hipError_t e) {
    if (e != hipSuccess && err_ == hipSuccess) err_ = e;
  }

  int device_;
  hipError_t err_ = hipSuccess;
  hipStream_t stream_ = nullptr;
  hipStream_t copy_ = nullptr;
  Arena arena_;
  JobDesc* d_desc_ = nullptr;
  JobDesc* h_desc_ = nullptr;
  SolverState* d_state_ = nullptr;
  LevelRecord* d_rec_ = nullptr;
  LevelRecord* h_rec_ = nullptr;
  char* h_taps_ = nullptr;
  const JobDesc* dv_desc_ = nullptr;  // device view of h_desc_
  const char* dv_taps_ = nullptr;     // device view of h_taps_
  volatile uint64_t* h_mirror_ = nullptr;
  uint64_t* d_mirror_ = nullptr;
  hipEvent_t step_ev_[kStepEvents] = {};
  int step_cur_ = 0;
  bool step_pending_ = false;
  int n_out_ = 0;                        // queued steps, see paced()
  int fold_max_jobs_ = kFoldMaxJobs;
  int pace_ = kPaceSteps;
  int max_ahead_ = kMaxAhead;
  bool noalloc_ = false;                 // see init_noalloc
  int n_slots_ = kMaxSlots;
  std::vector<char> noalloc_tables_;     // host tables of a no-alloc engine
  std::shared_ptr<HipEvent> out_ev_;     // its output event (one job at a time)
  long stall_steps_ = kStallSteps, idle_steps_ = 0, fail_step_ = 0, steps_ = 0;
  double stall_ms_ = kStallMs, idle_since_ = 0.0;
  bool stalled_ = false;
  uint32_t next_uid_ = 1;
  std::vector<Job*> slots_;
  int n_active_ = 0;
};

static void fill_stats(const Job* j, eecmg_stats* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->struct_size = sizeof(eecmg_stats);
  s->n_levels = j->plan.L;
  for (int l = 0; l < j->plan.L; ++l) {
    s->level_h[l] = j->plan.lv[l].h;
    s->level_w[l] = j->plan.lv[l].w;
    s->psf_radius[l] = j->plan.lv[l].rad;
    s->caps[l] = j->plan.lv[l].cap;
    s->iters[l] = j->rec[l].iters;
    s->stop_reason[l] = j->rec[l].reason;
    s->final_rms[l] = j->rec[l].rms;
  }
}

// Run a set of jobs to completion on an engine (admitting as room frees).
// On a HIP error or a scheduler stall every admitted job is aborted (the
// device drained first, slots and memory freed) before EDEVICE is returned,
// so the engine holds no job of this call afterwards.
static int run_jobs(Engine& E, std::vector<Job*>& jobs) {
  size_t next = 0, done = 0;
  std::vector<Job*> fin;
  E.read_knobs();
  while (done < jobs.size()) {
    while (next < jobs.size()) {
      const int rc = E.admit(jobs[next]);
      if (rc == EECMG_EAGAIN) break;
      if (rc != EECMG_OK) {
        std::vector<Job*> ab;
        E.abort_all(rc, ab);
        return rc;
      }
      ++next;
    }
    if (E.active() == 0 && next < jobs.size())
      return fail(EECMG_ENOMEM, "a job does not fit the device arena");
    const bool launched = E.step(fin);
    for (Job* j : fin) {
      E.release(j);
      ++done;
    }
    if (!launched && fin.empty() && !E.failed()) E.wait_some();
    if (E.failed()) {
      const std::string msg = E.failure();
      std::vector<Job*> ab;
      E.abort_all(EECMG_EDEVICE, ab);
      return fail(EECMG_EDEVICE, msg);
    }
  }
  return EECMG_OK;
}

// ---------------------------------------------------------------------------
// Process-wide engines for the plain / batched / operator calls
// ---------------------------------------------------------------------------
struct PlainEngine {
  std::mutex mu;
  std::unique_ptr<Engine> eng;
};

static PlainEngine* plain_engine(int device, int* rc) {
  static std::mutex mu;
  static std::map<int, PlainEngine*> engines;  // never destroyed: outlives static teardown order
  std::lock_guard<std::mutex> g(mu);
  auto it = engines.find(device);
  if (it != engines.end()) return it->second;
  PlainEngine* pe = new PlainEngine();
  pe->eng.reset(new Engine(device));
  *rc = pe->eng->init(nullptr);
  if (*rc != EECMG_OK) {
    delete pe;
    return nullptr;
  }
  engines[device] = pe;
  return pe;
}

static int current_device(int* dev) {
  EECMG_HIP(hipGetDevice(dev));
  return EECMG_OK;
}

static int check_dev_ptr(const void* p, const char* what) {
  if (!p) return fail(EECMG_EINVAL, std::string(what) + " is NULL");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(EECMG_EINVAL, std::string(what) + " is not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(EECMG_EINVAL, std::string(what) + " is not device memory");
  return EECMG_OK;
}

// ---------------------------------------------------------------------------
// Restores that allocate nothing: one fixed device region per GPU
// ---------------------------------------------------------------------------
// The region holds the no-alloc engine's tables (descriptors, solver state,
// level records, progress word: about 12 KiB) and the job arena.  A job needs
// about 9.7 times its finest level's bytes (seven work vectors, the
// right-hand-side and solution pyramids, PSF taps and tile partials), so
// 64 MiB serves FP32 images up to about 1300 x 1300 and FP64 ones up to
// about 900 x 900.  Each GPU the library runs on holds its own copy until
// the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

struct NoAllocEngine {
  std::mutex mu;  // calls on one GPU share its region: they run one at a time
  std::unique_ptr<Engine> eng;
  char* base = nullptr;  // this GPU's device address of `scratch`
};

// Set-up on the first call on a device (with that device current): the
// region's device address from hipGetSymbolAddress (the host-side name of
// the array is only a stand-in and never reaches a kernel), the engine's
// events and host tables.  No device or pinned memory is allocated.
static NoAllocEngine* noalloc_engine(int device, int* rc) {
  static std::mutex mu;
  static std::map<int, NoAllocEngine*> engines;  // never destroyed, like the region itself
  std::lock_guard<std::mutex> g(mu);
  auto it = engines.find(device);
  if (it != engines.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    *rc = fail(EECMG_EDEVICE, std::string("hipGetSymbolAddress of the scratch region: ") + hipGetErrorString(e));
    return nullptr;
  }
  std::unique_ptr<NoAllocEngine> ne(new NoAllocEngine());
  ne->base = (char*)ptr;
  ne->eng.reset(new Engine(device));
  *rc = ne->eng->init_noalloc(ne->base, kScratchBytes);
  if (*rc != EECMG_OK) return nullptr;
  engines[device] = ne.get();
  return ne.release();
}

static size_t arena_target(size_t need) {
  // keep at least 256 MiB so small calls do not reallocate
  return std::max(need, (size_t)256 << 20);
}

static int restore_jobs_on(PlainEngine* pe, std::vector<Job*>& jobs, hipStream_t stream) {
  Engine& E = *pe->eng;
  E.set_stream(stream);
  size_t total = 0, biggest = 0;
  for (Job* j : jobs) {
    total += align_up(j->plan.bytes, 256);
    biggest = std::max(biggest, j->plan.bytes);
  }
  // the free-memory query (about 15-20 us) only when the arena must grow:
  // an arena that holds every job already is what reserve() would keep
  if (E.arena().size() < arena_target(total)) {
    size_t free_b = 0, tot_b = 0;
    if (hipMemGetInfo(&free_b, &tot_b) != hipSuccess) free_b = (size_t)4 << 30;
    const size_t cap = (size_t)(0.6 * (double)(free_b + E.arena().size()));
    const size_t want = std::min(total, std::max(cap, biggest));
    const int rc = E.arena().reserve(arena_target(want));
    if (rc != EECMG_OK) return rc;
  }
  return run_jobs(E, jobs);
}

// Lanes of a batched call.  A batch of many images is split into K groups
// of about equal pixel count (longest first onto the least loaded lane),
// each driven by its own engine, HIP stream and host thread.  The lanes'
// launches run side by side on the device: the many small launches of a
// batch of small images (one per blur kernel and stage) no longer leave the
// chip idle between them, and the host issues them in parallel.  Each job's
// arithmetic does not depend on what shares its launches, so the results
// are the same bits as on one lane.  EECMG_BATCH_LANES sets K (1 = off);
// a lane gets at least kMinJobsPerLane images.  Measured on the uneven set
// (256 images): 1, 2, 3, 4 lanes take 26.7, 21.5, 20.2, 26.6 ms; four
// lanes and the caller's stream exceed the process's four hardware queues.
constexpr int kBatchLanes = 3, kMaxBatchLanes = 4, kMinJobsPerLane = 4;

static int batch_lane_count() {
  const char* e = std::getenv("EECMG_BATCH_LANES");
  return e ? std::min(kMaxBatchLanes, std::max(1, std::atoi(e))) : kBatchLanes;
}

struct BatchLanes {
  std::mutex mu;  // one lane-split batch at a time per device
  std::vector<std::unique_ptr<PlainEngine>> pes;
  std::vector<hipStream_t> streams;
  hipEvent_t start = nullptr;
};

static BatchLanes* batch_lanes(int device, int k, int* rc) {
  static std::mutex mu;
  static std::map<int, BatchLanes*> all;  // never destroyed, as the plain engines
  std::lock_guard<std::mutex> g(mu);
  BatchLanes*& bl = all[device];
  if (!bl) {
    bl = new BatchLanes();
    if (hipEventCreateWithFlags(&bl->start, hipEventDisableTiming) != hipSuccess) {
      *rc = fail(EECMG_EDEVICE, "hipEventCreate failed");
      delete bl;
      bl = nullptr;
      return nullptr;
    }
  }
  while ((int)bl->pes.size() < k) {
    std::unique_ptr<PlainEngine> pe(new PlainEngine());
    pe->eng.reset(new Engine(device));
    *rc = pe->eng->init(nullptr);
    if (*rc != EECMG_OK) return nullptr;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      *rc = fail(EECMG_EDEVICE, "hipStreamCreate failed");
      return nullptr;
    }
    bl->pes.push_back(std::move(pe));
    bl->streams.push_back(s);
  }
  return bl;
}

static int restore_jobs_lanes(int device, std::vector<Job*>& jobs, hipStream_t stream, int K) {
  int rc = EECMG_OK;
  BatchLanes* bl = batch_lanes(device, K, &rc);
  if (!bl) return rc;
  std::lock_guard<std::mutex> g(bl->mu);
  std::vector<Job*> order = jobs;
  std::stable_sort(order.begin(), order.end(), [](const Job* a, const Job* b) {
    return (long)a->plan.H * a->plan.W > (long)b->plan.H * b->plan.W;
  });
  std::vector<std::vector<Job*>> parts(K);
  std::vector<double> load(K, 0.0);
  for (Job* j : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    parts[k].push_back(j);
    load[k] += (double)j->plan.H * j->plan.W;
  }
  // every lane starts after the work the caller enqueued on its stream
  EECMG_HIP(hipEventRecord(bl->start, stream));
  std::vector<int> rcs(K, EECMG_OK);
  std::vector<std::string> errs(K);
  auto lane = [&](int k) {
    if (hipSetDevice(device) != hipSuccess || hipStreamWaitEvent(bl->streams[k], bl->start, 0) != hipSuccess) {
      rcs[k] = EECMG_EDEVICE;
      errs[k] = "lane set-up failed";
      return;
    }
    PlainEngine* pe = bl->pes[k].get();
    std::lock_guard<std::mutex> lk(pe->mu);
    rcs[k] = restore_jobs_on(pe, parts[k], bl->streams[k]);
    if (rcs[k] != EECMG_OK) errs[k] = g_err;
  };
  std::vector<std::thread> th;
  for (int k = 1; k < K; ++k) th.emplace_back(lane, k);
  lane(0);
  for (auto& t : th) t.join();
  for (int k = 0; k < K; ++k)
    if (rcs[k] != EECMG_OK) return fail(rcs[k], errs[k]);
  return EECMG_OK;
}

}  // namespace eecmg

using namespace eecmg;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* eecmg_last_error(void) { return g_err.c_str(); }

const char* eecmg_version(void) { return "eecmg-mi355x 0.1 (gfx950)"; }

int eecmg_profile_enable(int enable, int min_blocks) {
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  p.min_blocks = min_blocks < 0 ? 0 : min_blocks;
  p.on.store(enable != 0);
  return EECMG_OK;
}

int eecmg_profile_min_pixels(double min_pixels) {
  if (!(min_pixels >= 0.0)) return fail(EECMG_EINVAL, "min_pixels must be >= 0");
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  p.min_pixels = min_pixels;
  return EECMG_OK;
}

int eecmg_profile_reset(void) {
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  p.harvest();
  for (int i = 0; i < kNumStages; ++i) {
    p.launches[i] = 0;
    p.ms[i] = 0.0;
    p.pixels[i] = 0.0;
  }
  for (int l = 0; l < kMaxLevels; ++l)
    for (int i = 0; i < kNumStages; ++i) {
      p.lv_launches[l][i] = 0;
      p.lv_ms[l][i] = 0.0;
    }
  p.final_iters.clear();
  return EECMG_OK;
}

int eecmg_profile_read_level(int stage, int level, int* launches, double* total_ms) {
  if (stage < -1 || stage >= kNumStages) return fail(EECMG_EINVAL, "unknown stage id");
  if (level < 0 || level >= kMaxLevels) return fail(EECMG_EINVAL, "level out of range");
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  p.harvest();
  int n = 0;
  double ms = 0.0;
  for (int i = 0; i < kNumStages; ++i)
    if (stage == -1 || stage == i) {
      n += p.lv_launches[level][i];
      ms += p.lv_ms[level][i];
    }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  return EECMG_OK;
}

int eecmg_profile_read(int stage, int* launches, double* total_ms, double* total_pixels) {
  if (stage < 0 || stage >= kNumStages) return fail(EECMG_EINVAL, "unknown stage id");
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  p.harvest();
  if (launches) *launches = p.launches[stage];
  if (total_ms) *total_ms = p.ms[stage];
  if (total_pixels) *total_pixels = p.pixels[stage];
  return EECMG_OK;
}

int eecmg_params_default(eecmg_params* p) {
  if (!p) return fail(EECMG_EINVAL, "params is NULL");
  default_params(p);
  return EECMG_OK;
}

int eecmg_restore_dev(const void* g_delta_dev, int H, int W, const double* psf, int psf_radius, int n_levels,
                      const int* iters_per_level, double k, const eecmg_params* params, void* u_out_dev,
                      void* hip_stream) {
  g_err.clear();
  int rc = check_dev_ptr(g_delta_dev, "g_delta_dev");
  if (rc) return rc;
  rc = check_dev_ptr(u_out_dev, "u_out_dev");
  if (rc) return rc;
  Job job;
  rc = build_plan(H, W, psf, psf_radius, n_levels, iters_per_level, k, params, false, job.plan);
  if (rc) return rc;
  int dev = 0;
  rc = current_device(&dev);
  if (rc) return rc;
  PlainEngine* pe = plain_engine(dev, &rc);
  if (!pe) return rc;
  std::lock_guard<std::mutex> g(pe->mu);
  job.g_in_dev = g_delta_dev;
  job.u_out_dev = u_out_dev;
  std::vector<Job*> jobs{&job};
  rc = restore_jobs_on(pe, jobs, (hipStream_t)hip_stream);
  if (rc) return rc;
  if (params && params->stats) fill_stats(&job, (eecmg_stats*)params->stats);
  if (job.status != EECMG_OK) return fail(job.status, "non-finite value in the smoother");
  return EECMG_OK;
}

int eecmg_restore_dev_noalloc(const void* g_delta_dev, int H, int W, const double* psf, int psf_radius,
                              int n_levels, const int* iters_per_level, double k, const eecmg_params* params,
                              void* u_out_dev, void* hip_stream) {
  g_err.clear();
  int rc = check_dev_ptr(g_delta_dev, "g_delta_dev");
  if (rc) return rc;
  rc = check_dev_ptr(u_out_dev, "u_out_dev");
  if (rc) return rc;
  Job job;
  rc = build_plan(H, W, psf, psf_radius, n_levels, iters_per_level, k, params, false, job.plan);
  if (rc) return rc;
  int dev = 0;
  rc = current_device(&dev);
  if (rc) return rc;
  NoAllocEngine* ne = noalloc_engine(dev, &rc);
  if (!ne) return rc;
  std::lock_guard<std::mutex> g(ne->mu);
  Engine& E = *ne->eng;
  // without the direction ring if that is what makes the restore fit
  if (job.plan.bytes > E.arena_capacity()) {
    rc = build_plan(H, W, psf, psf_radius, n_levels, iters_per_level, k, params, false, job.plan, false);
    if (rc) return rc;
  }
  if (job.plan.bytes > E.arena_capacity())
    return fail(EECMG_EINVAL, "the restore needs " + std::to_string(job.plan.bytes) +
                                  " bytes of device scratch, more than the fixed region's " +
                                  std::to_string(E.arena_capacity()) + " (use eecmg_restore_dev)");
  E.set_stream((hipStream_t)hip_stream);
  rc = E.clear_noalloc_state();
  if (rc) return rc;
  job.g_in_dev = g_delta_dev;
  job.u_out_dev = u_out_dev;
  std::vector<Job*> jobs{&job};
  rc = run_jobs(E, jobs);
  if (rc) return rc;
  if (params && params->stats) fill_stats(&job, (eecmg_stats*)params->stats);
  if (job.status != EECMG_OK) return fail(job.status, "non-finite value in the smoother");
  return EECMG_OK;
}

int eecmg_restore(const void* g_delta, int H, int W, const double* psf, int psf_radius, int n_levels,
                  const int* iters_per_level, double k, const eecmg_params* params, void* u_out) {
  g_err.clear();
  if (!g_delta || !u_out) return fail(EECMG_EINVAL, "g_delta / u_out is NULL");
  Job job;
  int rc = build_plan(H, W, psf, psf_radius, n_levels, iters_per_level, k, params, true, job.plan);
  if (rc) return rc;
  int dev = 0;
  rc = current_device(&dev);
  if (rc) return rc;
  PlainEngine* pe = plain_engine(dev, &rc);
  if (!pe) return rc;
  std::lock_guard<std::mutex> g(pe->mu);
  Engine& E = *pe->eng;
  E.set_stream(nullptr);
  rc = E.arena().reserve(arena_target(job.plan.bytes));
  if (rc) return rc;
  // admit first so the job's own input buffer exists, then copy the input in
  if (E.admit(&job) != EECMG_OK) return fail(EECMG_ENOMEM, "job does not fit the device arena");
  const size_t bytes = (size_t)H * W * job.plan.esz;
  hipError_t he = hipMemcpy((void*)job.g_in_dev, g_delta, bytes, hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    E.release(&job);
    return fail(EECMG_EDEVICE, std::string("hipMemcpy H2D: ") + hipGetErrorString(he));
  }
  std::vector<Job*> fin;
  E.read_knobs();
  while (job.phase != Job::kFinished) {
    const bool launched = E.step(fin);
    if (!launched && fin.empty() && !E.failed()) E.wait_some();
    if (E.failed()) {
      const std::string msg = E.failure();
      std::vector<Job*> ab;
      E.abort_all(EECMG_EDEVICE, ab);
      return fail(EECMG_EDEVICE, msg);
    }
  }
  he = hipMemcpy(u_out, job.u_out_dev, bytes, hipMemcpyDeviceToHost);
  E.release(&job);
  if (he != hipSuccess) return fail(EECMG_EDEVICE, std::string("hipMemcpy D2H: ") + hipGetErrorString(he));
  if (params && params->stats) fill_stats(&job, (eecmg_stats*)params->stats);
  if (job.status != EECMG_OK) return fail(job.status, "non-finite value in the smoother");
  return EECMG_OK;
}

int eecmg_restore_batch_dev(int n_images, const void* const* g_delta_dev, const int* H, const int* W,
                            const double* const* psf, const int* psf_radius, const int* n_levels,
                            const int* const* iters_per_level, const double* k, const eecmg_params* params,
                            void* const* u_out_dev, void* hip_stream) {
  g_err.clear();
  if (n_images < 0) return fail(EECMG_EINVAL, "n_images < 0");
  if (n_images == 0) return EECMG_OK;
  if (!g_delta_dev || !H || !W || !psf || !psf_radius || !n_levels || !k || !u_out_dev)
    return fail(EECMG_EINVAL, "NULL array argument");
  std::vector<std::unique_ptr<Job>> owned;
  std::vector<Job*> jobs;
  int prec = -1;
  for (int i = 0; i < n_images; ++i) {
    std::unique_ptr<Job> j(new Job());
    const eecmg_params* pi = params ? &params[i] : nullptr;
    int rc = build_plan(H[i], W[i], psf[i], psf_radius[i], n_levels[i], iters_per_level ? iters_per_level[i] : nullptr,
                        k[i], pi, false, j->plan);
    if (rc) return fail(rc, "image " + std::to_string(i) + ": " + g_err);
    if (prec < 0) prec = j->plan.f64;
    if (prec != (int)j->plan.f64) return fail(EECMG_EINVAL, "all images of a batch must share one precision");
    rc = check_dev_ptr(g_delta_dev[i], "g_delta_dev[i]");
    if (rc) return rc;
    rc = check_dev_ptr(u_out_dev[i], "u_out_dev[i]");
    if (rc) return rc;
    j->g_in_dev = g_delta_dev[i];
    j->u_out_dev = u_out_dev[i];
    jobs.push_back(j.get());
    owned.push_back(std::move(j));
  }
  int dev = 0, rc = current_device(&dev);
  if (rc) return rc;
  const int lanes = std::min(batch_lane_count(), n_images / kMinJobsPerLane);
  if (lanes >= 2) {
    rc = restore_jobs_lanes(dev, jobs, (hipStream_t)hip_stream, lanes);
  } else {
    PlainEngine* pe = plain_engine(dev, &rc);
    if (!pe) return rc;
    std::lock_guard<std::mutex> g(pe->mu);
    rc = restore_jobs_on(pe, jobs, (hipStream_t)hip_stream);
  }
  if (rc) return rc;
  int first = EECMG_OK;
  for (int i = 0; i < n_images; ++i) {
    if (params && params[i].stats) fill_stats(jobs[i], (eecmg_stats*)params[i].stats);
    if (jobs[i]->status != EECMG_OK && first == EECMG_OK) first = jobs[i]->status;
  }
  if (first != EECMG_OK) return fail(first, "an image of the batch failed");
  return EECMG_OK;
}

// ------------------------------------------------------------------ operators
static int op_taps(const double* psf, int r, bool f64, bool flip, void** d_taps, int* variant) {
  const int n = 2 * r + 1;
  LevelPlan lp;
  lp.rad = r;
  lp.psf.assign(psf, psf + (size_t)n * n);
  choose_variant(lp, f64, false);  // operator calls: by the PSF only
  *variant = lp.variant;
  const std::vector<double>& t = flip ? lp.taps_t : lp.taps;
  const size_t bytes = t.size() * (f64 ? 8 : 4);
  EECMG_HIP(hipMalloc(d_taps, bytes));
  if (f64) {
    EECMG_HIP(hipMemcpy(*d_taps, t.data(), bytes, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(t.begin(), t.end());
    EECMG_HIP(hipMemcpy(*d_taps, f.data(), bytes, hipMemcpyHostToDevice));
  }
  return EECMG_OK;
}

static int check_prec(int precision) {
  if (precision < 0 || precision > 1) return fail(EECMG_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  return EECMG_OK;
}

int eecmg_op_conv_dev(const void* x_dev, void* y_dev, int H, int W, const double* psf, int psf_radius,
                      int transpose, int precision, void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (H < 1 || W < 1 || psf_radius < 0 || psf_radius > kMaxRadius || !psf)
    return fail(EECMG_EINVAL, "bad size, radius or psf");
  if (x_dev == y_dev) return fail(EECMG_EINVAL, "x and y must not alias");
  if ((rc = check_dev_ptr(x_dev, "x_dev")) || (rc = check_dev_ptr(y_dev, "y_dev"))) return rc;
  const bool f64 = precision == EECMG_FP64;
  if ((size_t)H * (size_t)W * (f64 ? 8 : 4) >= ((size_t)1 << 32))
    return fail(EECMG_EINVAL, "image exceeds 4 GiB (32-bit offsets)");
  void* taps = nullptr;
  int variant = 0;
  rc = op_taps(psf, psf_radius, f64, transpose != 0, &taps, &variant);
  if (rc) return rc;
  hipError_t e = op_conv(x_dev, y_dev, H, W, taps, variant, psf_radius, f64, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
  (void)hipFree(taps);
  if (e != hipSuccess) return fail(EECMG_EDEVICE, hipGetErrorString(e));
  return EECMG_OK;
}

int eecmg_op_smoother_dev(const void* g_dev, void* u_dev, int H, int W, const double* psf, int psf_radius, int cap,
                          const eecmg_params* params, eecmg_stats* stats_out, void* hip_stream) {
  g_err.clear();
  int rc;
  if ((rc = check_dev_ptr(g_dev, "g_dev")) || (rc = check_dev_ptr(u_dev, "u_dev"))) return rc;
  if (cap < 0) return fail(EECMG_EINVAL, "cap must be >= 0");
  Job job;
  rc = build_plan(H, W, psf, psf_radius, 1, &cap, 10.0, params, false, job.plan);
  if (rc) return rc;
  int dev = 0;
  rc = current_device(&dev);
  if (rc) return rc;
  PlainEngine* pe = plain_engine(dev, &rc);
  if (!pe) return rc;
  std::lock_guard<std::mutex> g(pe->mu);
  job.g_in_dev = g_dev;
  job.u_init_dev = u_dev;
  job.u_out_dev = u_dev;
  std::vector<Job*> jobs{&job};
  rc = restore_jobs_on(pe, jobs, (hipStream_t)hip_stream);
  if (rc) return rc;
  EECMG_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
  if (stats_out) fill_stats(&job, stats_out);
  if (job.status != EECMG_OK) return fail(job.status, "non-finite value in the smoother");
  return EECMG_OK;
}

int eecmg_op_restrict_dev(const void* g_fine_dev, int Hf, int Wf, void* g_coarse_dev, int precision,
                          void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (Hf < 1 || Wf < 1) return fail(EECMG_EINVAL, "bad size");
  if ((rc = check_dev_ptr(g_fine_dev, "g_fine_dev")) || (rc = check_dev_ptr(g_coarse_dev, "g_coarse_dev"))) return rc;
  hipError_t e = op_restrict(g_fine_dev, Hf, Wf, g_coarse_dev, precision == EECMG_FP64, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(EECMG_EDEVICE, hipGetErrorString(e));
  return EECMG_OK;
}

int eecmg_op_coarse_psf(const double* psf, int psf_radius, int mode, double* psf_coarse) {
  g_err.clear();
  if (!psf || !psf_coarse || psf_radius < 0 || psf_radius > kMaxRadius) return fail(EECMG_EINVAL, "bad psf");
  const int n = 2 * psf_radius + 1;
  std::vector<double> in(psf, psf + (size_t)n * n), out;
  int rc = decimate_psf(in, psf_radius, mode, out);
  if (rc) return rc;
  std::memcpy(psf_coarse, out.data(), out.size() * sizeof(double));
  return EECMG_OK;
}

#define EECMG_OP_TAIL(expr)                                                     \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ == hipSuccess) e_ = hipStreamSynchronize((hipStream_t)hip_stream);   \
    if (e_ != hipSuccess) return fail(EECMG_EDEVICE, hipGetErrorString(e_));    \
    return EECMG_OK;                                                            \
  } while (0)

int eecmg_op_extrapolate_dev(const void* uA_dev, const void* uB_dev, int HB, int WB, void* ut_dev, int precision,
                             void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (HB < 5 || WB < 5) return fail(EECMG_EINVAL, "the coarser grid needs at least 3 nodes per axis");
  if ((rc = check_dev_ptr(uA_dev, "uA_dev")) || (rc = check_dev_ptr(uB_dev, "uB_dev")) ||
      (rc = check_dev_ptr(ut_dev, "ut_dev")))
    return rc;
  EECMG_OP_TAIL(op_extrapolate(uA_dev, uB_dev, HB, WB, ut_dev, precision == EECMG_FP64, (hipStream_t)hip_stream));
}

int eecmg_op_prolong_quad_dev(const void* ut_dev, int HC, int WC, void* uC_dev, int precision, void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (HC < 5 || WC < 5) return fail(EECMG_EINVAL, "the coarser grid needs at least 3 nodes per axis");
  if ((rc = check_dev_ptr(ut_dev, "ut_dev")) || (rc = check_dev_ptr(uC_dev, "uC_dev"))) return rc;
  EECMG_OP_TAIL(op_prolong_quad(ut_dev, HC, WC, uC_dev, precision == EECMG_FP64, (hipStream_t)hip_stream));
}

int eecmg_op_prolong_linear_dev(const void* uB_dev, int HC, int WC, void* uC_dev, int precision, void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (HC < 3 || WC < 3) return fail(EECMG_EINVAL, "the coarser grid needs at least 2 nodes per axis");
  if ((rc = check_dev_ptr(uB_dev, "uB_dev")) || (rc = check_dev_ptr(uC_dev, "uC_dev"))) return rc;
  EECMG_OP_TAIL(op_prolong_linear(uB_dev, HC, WC, uC_dev, precision == EECMG_FP64, (hipStream_t)hip_stream));
}

int eecmg_op_transfer_dev(const void* uB_dev, int HC, int WC, void* uC_dev, int prolongation, double smooth_h,
                          int pm_steps, double k, double tau, int precision, void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (prolongation != 0 && prolongation != 1) return fail(EECMG_EINVAL, "prolongation must be 0 (P) or 1 (linear)");
  if (HC < (prolongation == 0 ? 5 : 3) || WC < (prolongation == 0 ? 5 : 3))
    return fail(EECMG_EINVAL, "the coarser grid is too small for the prolongation");
  if (!(smooth_h > 0.0)) return fail(EECMG_EINVAL, "smooth_h must be > 0");
  if (pm_steps != 0 && pm_steps != 1) return fail(EECMG_EINVAL, "pm_steps must be 0 or 1");
  if (pm_steps == 1 && (!(k > 0.0) || !(tau > 0.0 && tau <= 0.25))) return fail(EECMG_EINVAL, "bad k or tau");
  if ((rc = check_dev_ptr(uB_dev, "uB_dev")) || (rc = check_dev_ptr(uC_dev, "uC_dev"))) return rc;
  if (uB_dev == uC_dev) return fail(EECMG_EINVAL, "the transfer is out of place: uB and uC must not alias");
  EECMG_OP_TAIL(op_fused_transfer(uB_dev, HC, WC, uC_dev, prolongation == 0, smooth_h, pm_steps == 1, k, tau,
                                  precision == EECMG_FP64, (hipStream_t)hip_stream));
}

int eecmg_op_local_smooth_dev(const void* u_dev, void* out_dev, int H, int W, double smooth_h, int precision,
                              void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (H < 1 || W < 1 || !(smooth_h > 0.0)) return fail(EECMG_EINVAL, "bad size or smooth_h");
  if ((rc = check_dev_ptr(u_dev, "u_dev")) || (rc = check_dev_ptr(out_dev, "out_dev"))) return rc;
  if (u_dev == out_dev) return fail(EECMG_EINVAL, "S is out of place: u and out must not alias");
  EECMG_OP_TAIL(op_local_smooth(u_dev, out_dev, H, W, smooth_h, precision == EECMG_FP64, (hipStream_t)hip_stream));
}

int eecmg_op_pm_step_dev(const void* u_dev, void* out_dev, int H, int W, double k, double tau, int precision,
                         void* hip_stream) {
  g_err.clear();
  int rc = check_prec(precision);
  if (rc) return rc;
  if (H < 1 || W < 1 || !(k > 0.0) || !(tau > 0.0 && tau <= 0.25)) return fail(EECMG_EINVAL, "bad size, k or tau");
  if ((rc = check_dev_ptr(u_dev, "u_dev")) || (rc = check_dev_ptr(out_dev, "out_dev"))) return rc;
  if (u_dev == out_dev) return fail(EECMG_EINVAL, "D is out of place: u and out must not alias");
  EECMG_OP_TAIL(op_pm_step(u_dev, out_dev, H, W, k, tau, precision == EECMG_FP64, (hipStream_t)hip_stream));
}


// ------------------------------------------------------------ request loop
int eecmg_ctx_config_default(eecmg_ctx_config* cfg) {
  if (!cfg) return fail(EECMG_EINVAL, "cfg is NULL");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(eecmg_ctx_config);
  cfg->device = 0;
  cfg->hbm_budget_bytes = (size_t)8 << 30;
  cfg->max_slots = 64;
  cfg->max_queue = 4096;
  return EECMG_OK;
}

}  // extern "C"

namespace eecmg {

// Pinned host buffers recycled by size class (powers of two), so the
// request loop never allocates or frees pinned memory on its hot path.
class PinnedPool {
 public:
  ~PinnedPool() {}
  void* get(size_t bytes, size_t* cls_out) {
    size_t cls = (size_t)1 << 16;
    while (cls < bytes) cls <<= 1;
    *cls_out = cls;
    std::lock_guard<std::mutex> g(mu_);
    auto& v = free_[cls];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void* p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    free_[cls].push_back(p);
  }
  void release_all() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
    free_.clear();
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
};

struct Request {
  std::unique_ptr<Job> job;
  size_t in_cls = 0, out_cls = 0;
  bool admitted = false;
  bool finished = false;
  int status = EECMG_PENDING;
};

}  // namespace eecmg

struct eecmg_ctx {
  int device = 0;
  eecmg_ctx_config cfg{};
  std::unique_ptr<eecmg::Engine> eng;
  hipStream_t stream = nullptr;       // kernels of every admitted request
  hipStream_t copy_stream = nullptr;  // their input and output copies
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::unique_ptr<eecmg::Request>> reqs;
  uint64_t next_id = 1;
  bool stopping = false;
  std::thread th;
  eecmg::PinnedPool pool;
  int active = 0;
};

namespace eecmg {

static void progress_loop(eecmg_ctx* C) {
  (void)hipSetDevice(C->device);
  Engine& E = *C->eng;
  std::vector<Job*> fin;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(C->mu);
      // admission: FIFO with a look-ahead window, by slot and device budget
      int scanned = 0;
      for (auto it = C->queue.begin(); it != C->queue.end() && scanned < 32;) {
        Request* r = C->reqs[*it].get();
        if (r->job->cancelled) {
          r->finished = true;
          r->status = EECMG_ECANCELED;
          it = C->queue.erase(it);
          C->cv_done.notify_all();
          continue;
        }
        if (C->active >= C->cfg.max_slots) break;
        if (E.admit(r->job.get()) != EECMG_OK) {
          ++it;
          ++scanned;
          continue;
        }
        Job* j = r->job.get();
        if (hipMemcpyAsync((void*)j->g_in_dev, j->host_in, (size_t)j->plan.H * j->plan.W * j->plan.esz,
                           hipMemcpyHostToDevice, C->copy_stream) != hipSuccess ||
            E.mark_input(j, C->copy_stream) != EECMG_OK)
          j->cancelled = true;
        r->admitted = true;
        ++C->active;
        it = C->queue.erase(it);
      }
      if (C->active == 0) {
        if (C->stopping && C->queue.empty()) return;
        C->cv_work.wait(lk, [&] { return C->stopping || !C->queue.empty(); });
        continue;
      }
    }
    bool launched = E.step(fin);
    if (!launched && fin.empty() && !E.failed()) E.wait_some();
    if (E.failed()) {
      // a HIP error or a stall: every admitted request fails with EDEVICE
      // (the device is drained first); queued requests stay queued
      launched = false;
      E.abort_all(EECMG_EDEVICE, fin);
    }
    if (!fin.empty()) {
      std::lock_guard<std::mutex> lk(C->mu);
      for (Job* j : fin) {
        E.release(j);
        --C->active;
        auto it = C->reqs.find(j->id);
        if (it != C->reqs.end()) {
          it->second->finished = true;
          it->second->status = j->status;
        }
      }
      C->cv_done.notify_all();
    }
  }
}

}  // namespace eecmg

extern "C" {

int eecmg_create(const eecmg_ctx_config* cfg, eecmg_ctx** out) {
  g_err.clear();
  if (!out) return fail(EECMG_EINVAL, "out is NULL");
  eecmg_ctx_config c;
  if (cfg) {
    if (cfg->struct_size != sizeof(eecmg_ctx_config)) return fail(EECMG_EINVAL, "cfg->struct_size mismatch");
    c = *cfg;
  } else {
    eecmg_ctx_config_default(&c);
  }
  if (c.max_slots < 1 || c.max_slots > EECMG_MAX_SLOTS) return fail(EECMG_EINVAL, "max_slots out of range");
  if (c.max_queue < 1) return fail(EECMG_EINVAL, "max_queue must be >= 1");
  if (c.hbm_budget_bytes < ((size_t)1 << 20)) return fail(EECMG_EINVAL, "hbm_budget_bytes too small");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || c.device >= ndev)
    return fail(EECMG_EINVAL, "invalid device");
  std::unique_ptr<eecmg_ctx> C(new eecmg_ctx());
  C->device = c.device;
  C->cfg = c;
  EECMG_HIP(hipSetDevice(c.device));
  EECMG_HIP(hipStreamCreateWithFlags(&C->stream, hipStreamNonBlocking));
  EECMG_HIP(hipStreamCreateWithFlags(&C->copy_stream, hipStreamNonBlocking));
  C->eng.reset(new Engine(c.device));
  int rc = C->eng->init(C->stream);
  if (rc) return rc;
  C->eng->set_copy_stream(C->copy_stream);
  rc = C->eng->arena().reserve(c.hbm_budget_bytes);
  if (rc) return rc;
  C->eng->read_knobs();  // the context's scheduler knobs are fixed at creation
  C->th = std::thread(progress_loop, C.get());
  *out = C.release();
  return EECMG_OK;
}

int eecmg_submit(eecmg_ctx* C, const void* g_delta, int H, int W, const double* psf, int psf_radius, int n_levels,
                 const int* iters_per_level, double k, const eecmg_params* params, uint64_t* request_id) {
  g_err.clear();
  if (!C || !g_delta || !request_id) return fail(EECMG_EINVAL, "NULL argument");
  std::unique_ptr<Request> r(new Request());
  r->job.reset(new Job());
  Job* j = r->job.get();
  int rc = build_plan(H, W, psf, psf_radius, n_levels, iters_per_level, k, params, true, j->plan);
  if (rc) return rc;
  if (j->plan.bytes > C->eng->arena().size())
    return fail(EECMG_ENOMEM, "request needs " + std::to_string(j->plan.bytes) + " bytes, more than the budget");
  const size_t bytes = (size_t)H * W * j->plan.esz;
  j->host_in = C->pool.get(bytes, &r->in_cls);
  j->host_out = C->pool.get(bytes, &r->out_cls);
  if (!j->host_in || !j->host_out) {
    C->pool.put(j->host_in, r->in_cls);
    C->pool.put(j->host_out, r->out_cls);
    return fail(EECMG_ENOMEM, "pinned host staging allocation failed");
  }
  staging_copy(j->host_in, g_delta, bytes);
  j->t_submit = now_s();
  std::lock_guard<std::mutex> lk(C->mu);
  if ((int)C->queue.size() >= C->cfg.max_queue) {
    C->pool.put(j->host_in, r->in_cls);
    C->pool.put(j->host_out, r->out_cls);
    return fail(EECMG_EAGAIN, "request queue full");
  }
  const uint64_t id = C->next_id++;
  j->id = id;
  C->reqs[id] = std::move(r);
  C->queue.push_back(id);
  *request_id = id;
  C->cv_work.notify_one();
  return EECMG_OK;
}

static int collect(eecmg_ctx* C, uint64_t id, void* u_out, eecmg_stats* stats_out, bool block) {
  // take a finished request out of the table under the lock; copy its result
  // after releasing it, so the progress thread is never held up by the copy
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(C->mu);
    auto done = [&] {
      auto f = C->reqs.find(id);
      return f == C->reqs.end() || f->second->finished;
    };
    if (C->reqs.find(id) == C->reqs.end()) return fail(EECMG_ENOTFOUND, "unknown request id");
    if (block) C->cv_done.wait(lk, done);
    auto it = C->reqs.find(id);
    if (it == C->reqs.end()) return fail(EECMG_ENOTFOUND, "unknown request id");
    if (!it->second->finished) return EECMG_PENDING;
    r = std::move(it->second);
    C->reqs.erase(it);
  }
  Job* j = r->job.get();
  const int st = r->status;
  if (st == EECMG_OK && u_out) staging_copy(u_out, j->host_out, (size_t)j->plan.H * j->plan.W * j->plan.esz);
  if (stats_out) fill_stats(j, stats_out);
  C->pool.put(j->host_in, r->in_cls);
  C->pool.put(j->host_out, r->out_cls);
  if (st != EECMG_OK) return fail(st, st == EECMG_ECANCELED ? "request cancelled" : "request failed");
  return EECMG_OK;
}

int eecmg_poll(eecmg_ctx* C, uint64_t request_id, void* u_out, eecmg_stats* stats_out) {
  g_err.clear();
  if (!C) return fail(EECMG_EINVAL, "ctx is NULL");
  return collect(C, request_id, u_out, stats_out, false);
}

int eecmg_wait(eecmg_ctx* C, uint64_t request_id, void* u_out, eecmg_stats* stats_out) {
  g_err.clear();
  if (!C) return fail(EECMG_EINVAL, "ctx is NULL");
  return collect(C, request_id, u_out, stats_out, true);
}

int eecmg_cancel(eecmg_ctx* C, uint64_t request_id) {
  g_err.clear();
  if (!C) return fail(EECMG_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(C->mu);
  auto it = C->reqs.find(request_id);
  if (it == C->reqs.end()) return fail(EECMG_ENOTFOUND, "unknown request id");
  it->second->job->cancelled = true;
  C->cv_work.notify_one();
  return EECMG_OK;
}

int eecmg_ctx_info(eecmg_ctx* C, int* queued, int* active, size_t* bytes_in_use) {
  g_err.clear();
  if (!C) return fail(EECMG_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(C->mu);
  if (queued) *queued = (int)C->queue.size();
  if (active) *active = C->active;
  if (bytes_in_use) *bytes_in_use = C->eng->arena().used();
  return EECMG_OK;
}

int eecmg_destroy(eecmg_ctx* C) {
  g_err.clear();
  if (!C) return fail(EECMG_EINVAL, "ctx is NULL");
  {
    std::lock_guard<std::mutex> lk(C->mu);
    C->stopping = true;
    for (auto& kv : C->reqs) kv.second->job->cancelled = true;
    C->cv_work.notify_all();
  }
  if (C->th.joinable()) C->th.join();
  (void)hipSetDevice(C->device);
  (void)hipStreamSynchronize(C->stream);
  (void)hipStreamSynchronize(C->copy_stream);
  for (auto& kv : C->reqs) {
    C->pool.put(kv.second->job->host_in, kv.second->in_cls);
    C->pool.put(kv.second->job->host_out, kv.second->out_cls);
  }
  C->reqs.clear();
  C->eng->arena().release();
  C->eng->shutdown();
  C->pool.release_all();
  (void)hipStreamDestroy(C->stream);
  (void)hipStreamDestroy(C->copy_stream);
  delete C;
  return EECMG_OK;
}

}  // extern "C"
