// HIP kernels (gfx950, wave64) of the EECMG cascade.
//
// Every kernel works on row-major pitched images in HBM.  Stencils stage a
// tile plus its halo in LDS; the blur operator is evaluated with a
// register-blocked sliding column (each lane owns one column and kV output
// rows, so every LDS value feeds up to kV FMAs); inner products are
// accumulated per lane in FP64, reduced across the wave with shuffles and
// across the block in a fixed order, and written as one partial per tile.
// Small finalize kernels sum the partials of a job in a fixed order and run
// the scalar part of the Krylov recurrences on the device, so results are
// deterministic and independent of how many jobs share a launch.
#include <math.h>

#include "eecmg_internal.h"

namespace eecmg {

// ---------------------------------------------------------------------------
// Launch-list helpers
// ---------------------------------------------------------------------------

// Blocks are dispatched round-robin over the 8 XCDs.  Remap so that each XCD
// receives a contiguous run of tiles: vertically adjacent tiles then share
// their halo rows through the same L2.
__device__ __forceinline__ int remap_xcd(int b, int nb) {
  if (nb < 64) return b;
  const int xcd = b & 7, j = b >> 3, q = nb >> 3, rm = nb & 7;
  return (xcd < rm) ? xcd * (q + 1) + j : rm * (q + 1) + (xcd - rm) * q + j;
}

struct Loc {
  int e;  // entry in the launch list
  int d;  // descriptor index
  int t;  // tile within the job
};

__device__ __forceinline__ Loc locate(const LaunchList& ll, int b) {
  int lo = 0, hi = ll.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ll.start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return Loc{lo, ll.job[lo], b - ll.start[lo]};
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <typename T>
__device__ __forceinline__ T to_t(double x) {
  return (T)x;
}

// Sum NV per-lane FP64 values over the 256-thread block in a fixed order and
// store them (thread 0) to out[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* __restrict__ out) {
  __shared__ double red[4][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
  }
}

// Fixed-order sum of selected components of the tile partials of one job,
// returned to every thread of the block.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int ntiles, const int (&comp)[NV],
                                             double (&out)[NV]) {
  __shared__ double red[4][NV];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 256) {
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += part[(size_t)t * kNPart + comp[i]];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = acc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// ---------------------------------------------------------------------------
// Blur operator on an LDS tile.
//
// tile holds the input on rows [y0 - R, y0 + kTH + R) and columns
// [x0 - R, x0 + kTW + R) (zero outside the image), row stride kTW + 2 RMAX.
// The lane computes, for column x0 + lane and rows y0 + wave*kV + v,
//   acc[v] = sum_{|a|,|b| <= R} taps[(a+R)(2R+1) + (b+R)] x(row - a, col - b).
// For each column offset b the lane loads its column segment once into
// registers (xc, shifted so that every register index is a compile-time
// constant) and applies all row offsets a to its kV outputs.
// ---------------------------------------------------------------------------
template <typename T, int RMAX>
__device__ __forceinline__ void conv_tile(const T* __restrict__ tile, int R, const T* __restrict__ taps, int wave,
                                          int lane, T (&acc)[kV]) {
  constexpr int LW = kTW + 2 * RMAX;
#pragma unroll
  for (int v = 0; v < kV; ++v) acc[v] = T(0);
  const int n = 2 * R + 1;
  for (int b = -R; b <= R; ++b) {
    T xc[kV + 2 * RMAX];
    const int col = lane + R - b;
#pragma unroll
    for (int t = 0; t < kV + 2 * RMAX; ++t) {
      const int lr = wave * kV + t - (RMAX - R);
      xc[t] = (t >= RMAX - R && t < RMAX + R + kV) ? tile[lr * LW + col] : T(0);
    }
#pragma unroll
    for (int a = -RMAX; a <= RMAX; ++a) {
      if (a >= -R && a <= R) {
        const T wt = taps[(a + R) * n + (b + R)];
#pragma unroll
        for (int v = 0; v < kV; ++v) acc[v] = fma(wt, xc[v + RMAX - a], acc[v]);
      }
    }
  }
}

// Tile geometry shared by the smoother kernels.
struct TileGeo {
  int R, h, w, pitch, y0, x0, wave, lane;
};

__device__ __forceinline__ TileGeo tile_geo(const JobDesc& d, int t) {
  TileGeo g;
  g.R = uni(d.rad);
  g.h = uni(d.h);
  g.w = uni(d.w);
  g.pitch = uni(d.pitch);
  const int tiles_x = uni(d.tiles_x);
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  g.y0 = ty * kTH;
  g.x0 = tx * kTW;
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  return g;
}

// Load tile + halo through a per-pixel functor f(offset, interior) -> T
// (interior: the pixel belongs to this tile's output region).  Pixels
// outside the image are zero (the operator's zero boundary condition).
template <typename T, int RMAX, typename F>
__device__ __forceinline__ void load_tile(T* __restrict__ tile, const TileGeo& g, F f) {
  constexpr int LW = kTW + 2 * RMAX;
  for (int ly = g.wave; ly < kTH + 2 * g.R; ly += 4) {
    const int gy = g.y0 - g.R + ly;
    const bool row_in = gy >= 0 && gy < g.h;
    const bool row_int = ly >= g.R && ly < g.R + kTH;
    for (int lx = g.lane; lx < kTW + 2 * g.R; lx += 64) {
      const int gx = g.x0 - g.R + lx;
      T v = T(0);
      if (row_in && gx >= 0 && gx < g.w) {
        const bool interior = row_int && lx >= g.R && lx < g.R + kTW;
        v = f((size_t)gy * g.pitch + gx, interior);
      }
      tile[ly * LW + lx] = v;
    }
  }
}

// r = g - H u0, stored in r[0]; partial <r,r> in slot 1.  (CGLS and MR)
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_init1(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo(d, L.t);
  const T* __restrict__ u = (const T*)d.u;
  const T* __restrict__ gg = (const T*)d.g;
  T* __restrict__ r = (T*)d.r[0];
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool) { return u[o]; });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, g.R, (const T*)d.taps, g.wave, g.lane, acc);
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < g.h && gx < g.w) {
      const size_t o = (size_t)gy * g.pitch + gx;
      const T rv = to_t<T>((double)gg[o] - (double)acc[v]);
      r[o] = rv;
      part[0] += (double)rv * (double)rv;
    }
  }
  block_sum_store<1>(part, d.partials + (size_t)L.t * kNPart + 1);
}

// s = H^T r, p[0] = s; partial <s,s> in slot 2.
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_cg_init2(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo(d, L.t);
  const T* __restrict__ r = (const T*)d.r[0];
  T* __restrict__ s = (T*)d.s;
  T* __restrict__ p = (T*)d.p[0];
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool) { return r[o]; });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, g.R, (const T*)d.taps_t, g.wave, g.lane, acc);
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < g.h && gx < g.w) {
      const size_t o = (size_t)gy * g.pitch + gx;
      s[o] = acc[v];
      p[o] = acc[v];
      part[0] += (double)acc[v] * (double)acc[v];
    }
  }
  block_sum_store<1>(part, d.partials + (size_t)L.t * kNPart + 2);
}

// Pass A of iteration k: p_new = s + beta p_old (on tile + halo), q = H p_new;
// partial <q,q> in slot 0.
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_cg_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo(d, L.t);
  const int par = uni(st->par);
  const double beta = st->beta;
  const T* __restrict__ s = (const T*)d.s;
  const T* __restrict__ po = (const T*)d.p[par];
  T* __restrict__ pn = (T*)d.p[par ^ 1];
  T* __restrict__ q = (T*)d.q[0];
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool interior) {
    const T v = to_t<T>((double)s[o] + beta * (double)po[o]);
    if (interior) pn[o] = v;
    return v;
  });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, g.R, (const T*)d.taps, g.wave, g.lane, acc);
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < g.h && gx < g.w) {
      const size_t o = (size_t)gy * g.pitch + gx;
      q[o] = acc[v];
      part[0] += (double)acc[v] * (double)acc[v];
    }
  }
  block_sum_store<1>(part, d.partials + (size_t)L.t * kNPart + 0);
}

// Pass B of iteration k: r_new = r - alpha q (tile + halo), s = H^T r_new,
// u += alpha p_new; partials <r,r> (slot 1) and <s,s> (slot 2).
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_cg_b(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo(d, L.t);
  const int par = uni(st->par);
  const double alpha = st->alpha;
  const T* __restrict__ ro = (const T*)d.r[par];
  T* __restrict__ rn = (T*)d.r[par ^ 1];
  const T* __restrict__ q = (const T*)d.q[0];
  const T* __restrict__ pn = (const T*)d.p[par ^ 1];
  T* __restrict__ u = (T*)d.u;
  T* __restrict__ s = (T*)d.s;
  double part[2] = {0.0, 0.0};
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool interior) {
    const T v = to_t<T>((double)ro[o] - alpha * (double)q[o]);
    if (interior) {
      rn[o] = v;
      part[0] += (double)v * (double)v;
    }
    return v;
  });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, g.R, (const T*)d.taps_t, g.wave, g.lane, acc);
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < g.h && gx < g.w) {
      const size_t o = (size_t)gy * g.pitch + gx;
      s[o] = acc[v];
      part[1] += (double)acc[v] * (double)acc[v];
      u[o] = to_t<T>((double)u[o] + alpha * (double)pn[o]);
    }
  }
  block_sum_store<2>(part, d.partials + (size_t)L.t * kNPart + 1);
}

// ---------------------------------------------------------------------------
// MR kernel (minimal-residual iteration, one operator product per step)
// ---------------------------------------------------------------------------
// If a step alpha is pending: r_new = r - alpha q and u += alpha r; then
// q_new = H r_new.  Partials <r_new,q_new> (0), <r_new,r_new> (1), <q,q> (2).
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_mr_pass(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  constexpr int LW = kTW + 2 * RMAX;
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo(d, L.t);
  const int par = uni(st->par);
  const bool pending = uni(st->pending) != 0;
  const double alpha = st->alpha;
  const T* __restrict__ ro = (const T*)d.r[par];
  const T* __restrict__ qo = (const T*)d.q[par];
  T* __restrict__ rn = (T*)d.r[par ^ 1];
  T* __restrict__ qn = (T*)d.q[par ^ 1];
  T* __restrict__ u = (T*)d.u;
  double part[3] = {0.0, 0.0, 0.0};
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool interior) {
    const T r0 = ro[o];
    const T v = pending ? to_t<T>((double)r0 - alpha * (double)qo[o]) : r0;
    if (interior) {
      rn[o] = v;
      part[1] += (double)v * (double)v;
      if (pending) u[o] = to_t<T>((double)u[o] + alpha * (double)r0);
    }
    return v;
  });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, g.R, (const T*)d.taps, g.wave, g.lane, acc);
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < g.h && gx < g.w) {
      const size_t o = (size_t)gy * g.pitch + gx;
      qn[o] = acc[v];
      const T rc = tile[(g.wave * kV + v + g.R) * LW + g.lane + g.R];
      part[0] += (double)rc * (double)acc[v];
      part[2] += (double)acc[v] * (double)acc[v];
    }
  }
  block_sum_store<3>(part, d.partials + (size_t)L.t * kNPart + 0);
}

// ---------------------------------------------------------------------------
// Finalize kernels: one block per job, scalar recurrences in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// Stopping tests of the smoother, in the order: non-finite, discrepancy
// principle ||r|| <= c delta (RMS norm), iteration cap m_l, convergence guard.
__device__ __forceinline__ void check_stop(SolverState* st, const JobDesc& d, double rr, double guard_val,
                                           double guard_ref, bool nonfinite) {
  const double rms = sqrt(rr / ((double)d.h * (double)d.w));
  int reason = kStopNone;
  if (nonfinite)
    reason = kStopNonFinite;
  else if (d.stop_rule && rms <= d.cdelta)
    reason = kStopDiscrepancy;
  else if (st->k >= d.cap)
    reason = kStopCap;
  else if (guard_val == 0.0 || guard_val <= d.eps2 * guard_ref)
    reason = kStopGuard;
  st->rr = rr;
  if (reason != kStopNone) {
    st->done = reason;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = reason;
    d.rec[d.level].rms = rms;
  }
}

__global__ __launch_bounds__(256) void k_cg_fin_init(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  double v[2];
  const int comp[2] = {1, 2};
  sum_partials<2>(d.partials, d.ntiles, comp, v);
  if (threadIdx.x != 0) return;
  SolverState* st = d.st;
  st->k = 0;
  st->par = 0;
  st->beta = 0.0;
  st->alpha = 0.0;
  st->done = kStopNone;
  st->pending = 0;
  st->level = d.level;
  st->gamma = v[1];
  st->gamma0 = v[1];
  st->rr0 = v[0];
  d.rec[d.level].iters = 0;
  d.rec[d.level].reason = kStopNone;
  d.rec[d.level].rms = sqrt(v[0] / ((double)d.h * (double)d.w));
  check_stop(st, d, v[0], v[1], v[1], !finite_d(v[0]) || !finite_d(v[1]));
}

__global__ __launch_bounds__(256) void k_cg_fin_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  SolverState* st = d.st;
  if (st->done) return;
  double v[1];
  const int comp[1] = {0};
  sum_partials<1>(d.partials, d.ntiles, comp, v);
  if (threadIdx.x != 0) return;
  const double eta = v[0];
  st->eta = eta;
  if (!finite_d(eta) || eta == 0.0) {
    const int reason = finite_d(eta) ? kStopGuard : kStopNonFinite;
    st->done = reason;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = reason;
    d.rec[d.level].rms = sqrt(st->rr / ((double)d.h * (double)d.w));
    return;
  }
  st->alpha = st->gamma / eta;
}

__global__ __launch_bounds__(256) void k_cg_fin_b(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  SolverState* st = d.st;
  if (st->done) return;
  double v[2];
  const int comp[2] = {1, 2};
  sum_partials<2>(d.partials, d.ntiles, comp, v);
  if (threadIdx.x != 0) return;
  const double gnew = v[1];
  st->beta = gnew / st->gamma;
  st->gamma = gnew;
  st->k += 1;
  st->par ^= 1;
  st->seq += 1;
  check_stop(st, d, v[0], gnew, st->gamma0, !finite_d(v[0]) || !finite_d(gnew));
}

__global__ __launch_bounds__(256) void k_mr_fin_init(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  double v[1];
  const int comp[1] = {1};
  sum_partials<1>(d.partials, d.ntiles, comp, v);
  if (threadIdx.x != 0) return;
  SolverState* st = d.st;
  st->k = 0;
  st->par = 0;
  st->alpha = 0.0;
  st->beta = 0.0;
  st->done = kStopNone;
  st->pending = 0;
  st->level = d.level;
  st->rr0 = v[0];
  d.rec[d.level].iters = 0;
  d.rec[d.level].reason = kStopNone;
  d.rec[d.level].rms = sqrt(v[0] / ((double)d.h * (double)d.w));
  check_stop(st, d, v[0], v[0], v[0], !finite_d(v[0]));
}

__global__ __launch_bounds__(256) void k_mr_fin(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  SolverState* st = d.st;
  if (st->done) return;
  double v[3];
  const int comp[3] = {0, 1, 2};
  sum_partials<3>(d.partials, d.ntiles, comp, v);
  if (threadIdx.x != 0) return;
  if (st->pending) st->k += 1;
  st->pending = 0;
  st->par ^= 1;
  st->seq += 1;
  const double rq = v[0], rr = v[1], qq = v[2];
  check_stop(st, d, rr, rr, st->rr0, !finite_d(rr) || !finite_d(rq) || !finite_d(qq));
  if (st->done) return;
  st->eta = qq;
  if (qq == 0.0) {
    st->done = kStopGuard;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = kStopGuard;
    d.rec[d.level].rms = sqrt(rr / ((double)d.h * (double)d.w));
    return;
  }
  st->rq = rq;
  st->alpha = rq / qq;
  st->pending = 1;
}

// ---------------------------------------------------------------------------
// Level transfer operators (Sections 3 and 4), pixel-parallel in FP64.
// ---------------------------------------------------------------------------
struct XArgs {
  const void* s0;  // first source
  const void* s1;  // second source (Pi: level l)
  void* dst;
  int h0, w0, p0;  // first source grid
  int h1, w1, p1;  // second source grid
  int hd, wd, pd;  // destination grid
  double a0, a1;   // operator parameters
};

// Quadratic extrapolation of a virtual node from the three nodes before it
// (exact for quadratics).
__device__ __forceinline__ double qx3(double v1, double v2, double v3) { return 3.0 * v1 - 3.0 * v2 + v3; }

// Pi correction d(a,b) = uB(2a,2b) - uA(a,b) on the level-(l-1) grid, with one
// virtual node per axis (along j first, then along i).
template <typename T>
struct PiD {
  const T* uA;
  const T* uB;
  int hA, wA, pA, pB;
  __device__ __forceinline__ double real(int a, int b) const {
    return (double)uB[(size_t)(2 * a) * pB + 2 * b] - (double)uA[(size_t)a * pA + b];
  }
  __device__ __forceinline__ double rowext(int a, int b) const {
    if (b < wA) return real(a, b);
    return qx3(real(a, wA - 1), real(a, wA - 2), real(a, wA - 3));
  }
  __device__ __forceinline__ double operator()(int a, int b) const {
    if (a < hA) return rowext(a, b);
    return qx3(rowext(hA - 1, b), rowext(hA - 2, b), rowext(hA - 3, b));
  }
};

// New extrapolation Pi (Section 3.2): output on grid B.
template <typename T>
__device__ __forceinline__ void pi_point(const XArgs& x, int p, int q) {
  const T* uA = (const T*)x.s0;
  const T* uB = (const T*)x.s1;
  const PiD<T> D{uA, uB, x.h0, x.w0, x.p0, x.p1};
  const int a = p >> 1, b = q >> 1;
  double corr;
  if (!(p & 1) && !(q & 1))
    corr = D(a, b) * 0.25;
  else if (!(p & 1))
    corr = (D(a, b) + D(a, b + 1)) * 0.125;
  else if (!(q & 1))
    corr = (D(a, b) + D(a + 1, b)) * 0.125;
  else
    corr = (D(a, b) + D(a + 1, b) + D(a, b + 1) + D(a + 1, b + 1)) * 0.0625;
  ((T*)x.dst)[(size_t)p * x.pd + q] = to_t<T>((double)uB[(size_t)p * x.p1 + q] + corr);
}

// Source of the quadratic interpolation extended by two virtual nodes per
// axis (along j for the real rows first, then along i).
template <typename T>
struct QExt {
  const T* u;
  int h, w, p;
  __device__ __forceinline__ double at(int i, int j) const { return (double)u[(size_t)i * p + j]; }
  __device__ __forceinline__ double rowext(int i, int j) const {
    if (j < w) return at(i, j);
    const double e0 = qx3(at(i, w - 1), at(i, w - 2), at(i, w - 3));
    if (j == w) return e0;
    return qx3(e0, at(i, w - 1), at(i, w - 2));
  }
  __device__ __forceinline__ double operator()(int i, int j) const {
    if (i < h) return rowext(i, j);
    const double e0 = qx3(rowext(h - 1, j), rowext(h - 2, j), rowext(h - 3, j));
    if (i == h) return e0;
    return qx3(e0, rowext(h - 1, j), rowext(h - 2, j));
  }
};

// One axis of the quadratic interpolation: fine index I, coarse panel
// (2a, 2a+1, 2a+2) with Lagrange weights (3/8, 3/4, -1/8) and (-1/8, 3/4, 3/8)
// at the quarter points.
template <typename F>
__device__ __forceinline__ double quad1(int I, F f) {
  const int p = I >> 1;
  if (!(I & 1)) return f(p);
  if (!(p & 1)) return 0.375 * f(p) + 0.75 * f(p + 1) - 0.125 * f(p + 2);
  return -0.125 * f(p - 1) + 0.75 * f(p) + 0.375 * f(p + 1);
}

template <typename T>
__device__ __forceinline__ void quad_point(const XArgs& x, int I, int J) {
  const QExt<T> E{(const T*)x.s0, x.h0, x.w0, x.p0};
  // along i first (T(I, q) for the needed columns q), then along j
  const double v = quad1(J, [&](int q) { return quad1(I, [&](int p) { return E(p, q); }); });
  ((T*)x.dst)[(size_t)I * x.pd + J] = to_t<T>(v);
}

// Linear prolongation of eq. (15) with one linearly extrapolated virtual
// node per axis (along j first, then along i).
template <typename T>
__device__ __forceinline__ void linear_point(const XArgs& x, int I, int J) {
  const T* u = (const T*)x.s0;
  const int h = x.h0, w = x.w0, p = x.p0;
  auto at = [&](int i, int j) { return (double)u[(size_t)i * p + j]; };
  auto rowext = [&](int i, int j) { return j < w ? at(i, j) : 2.0 * at(i, w - 1) - at(i, w - 2); };
  auto E = [&](int i, int j) { return i < h ? rowext(i, j) : 2.0 * rowext(h - 1, j) - rowext(h - 2, j); };
  const int a = I >> 1, b = J >> 1;
  double v;
  if (!(I & 1) && !(J & 1))
    v = E(a, b);
  else if (!(I & 1))
    v = 0.5 * (E(a, b) + E(a, b + 1));
  else if (!(J & 1))
    v = 0.5 * (E(a, b) + E(a + 1, b));
  else
    v = 0.5 * (E(a, b) + E(a + 1, b + 1));
  ((T*)x.dst)[(size_t)I * x.pd + J] = to_t<T>(v);
}

// Local smoothing S (Section 3.3, eq. 18-19): weighted LS fit of
// a0 + a1 s + a2 t on the 3x3 window with w = exp(-((u_c - u_n)/h)^2)
// (exactly 0 beyond (./h)^2 > 30, out-of-image neighbours dropped), output
// a0.  The fit is centred on the pixel value and on the weighted centroid,
// and the 2x2 system for (a1, a2) is solved by a plane rotation that
// diagonalises it, dropping eigenvalues below 1e-12 of the largest; the fitted
// centre value stays accurate for near-collinear weight patterns.
template <typename T>
__device__ __forceinline__ void smooth_point(const XArgs& x, int i, int j) {
  const T* u = (const T*)x.s0;
  const int H = x.h0, W = x.w0, P = x.p0;
  const double inv_h = 1.0 / x.a0;
  const double uc = (double)u[(size_t)i * P + j];
  double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0, b0 = 0, b1 = 0, b2 = 0;
#pragma unroll
  for (int s = -1; s <= 1; ++s) {
#pragma unroll
    for (int t = -1; t <= 1; ++t) {
      const int ii = i + s, jj = j + t;
      if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
      const double v = (double)u[(size_t)ii * P + jj] - uc;
      const double z = v * inv_h;
      const double e = z * z;
      double wt;
      if (sizeof(T) == 4)
        wt = e > 30.0 ? 0.0 : (double)expf(-(float)e);
      else
        wt = e > 30.0 ? 0.0 : exp(-e);
      m00 += wt;
      m01 += wt * s;
      m02 += wt * t;
      m11 += wt * (s * s);
      m12 += wt * (s * t);
      m22 += wt * (t * t);
      b0 += wt * v;
      b1 += wt * s * v;
      b2 += wt * t * v;
    }
  }
  const double sb = m01 / m00, tb = m02 / m00, vb = b0 / m00;
  const double S11 = m11 - m01 * sb, S12 = m12 - m01 * tb, S22 = m22 - m02 * tb;
  const double c1 = b1 - m01 * vb, c2 = b2 - m02 * vb;
  const double th = 0.5 * atan2(2.0 * S12, S11 - S22);
  double sn, cs;
  sincos(th, &sn, &cs);
  const double l1 = S11 * cs * cs + 2.0 * S12 * cs * sn + S22 * sn * sn;
  const double l2 = S11 * sn * sn - 2.0 * S12 * cs * sn + S22 * cs * cs;
  const double lmax = fmax(fabs(l1), fabs(l2));
  double corr = 0.0;
  if (l1 > 1e-12 * lmax && l1 > 0.0) corr += (sb * cs + tb * sn) * (c1 * cs + c2 * sn) / l1;
  if (l2 > 1e-12 * lmax && l2 > 0.0) corr += (tb * cs - sb * sn) * (c2 * cs - c1 * sn) / l2;
  ((T*)x.dst)[(size_t)i * x.pd + j] = to_t<T>(uc + (vb - corr));
}

// One explicit Perona-Malik step (Section 4, eq. 21, 23-25):
// out = u + tau sum_{in-image nb} (c_nb + c)/2 (u_nb - u), c = 1/(1+|grad u|^2/k^2)
// with |grad u| from central differences on a replicated border.
template <typename T>
__device__ __forceinline__ double pm_c(const T* u, int H, int W, int P, int i, int j, double ik2) {
  const int ip = i + 1 < H ? i + 1 : H - 1, im = i > 0 ? i - 1 : 0;
  const int jp = j + 1 < W ? j + 1 : W - 1, jm = j > 0 ? j - 1 : 0;
  const double ux = 0.5 * ((double)u[(size_t)ip * P + j] - (double)u[(size_t)im * P + j]);
  const double uy = 0.5 * ((double)u[(size_t)i * P + jp] - (double)u[(size_t)i * P + jm]);
  return 1.0 / (1.0 + (ux * ux + uy * uy) * ik2);
}

template <typename T>
__device__ __forceinline__ void pm_point(const XArgs& x, int i, int j) {
  const T* u = (const T*)x.s0;
  const int H = x.h0, W = x.w0, P = x.p0;
  const double ik2 = 1.0 / (x.a0 * x.a0), tau = x.a1;
  const double uc = (double)u[(size_t)i * P + j];
  const double cc = pm_c(u, H, W, P, i, j, ik2);
  double acc = 0.0;
  if (i + 1 < H) acc += 0.5 * (pm_c(u, H, W, P, i + 1, j, ik2) + cc) * ((double)u[(size_t)(i + 1) * P + j] - uc);
  if (i > 0) acc += 0.5 * (pm_c(u, H, W, P, i - 1, j, ik2) + cc) * ((double)u[(size_t)(i - 1) * P + j] - uc);
  if (j + 1 < W) acc += 0.5 * (pm_c(u, H, W, P, i, j + 1, ik2) + cc) * ((double)u[(size_t)i * P + j + 1] - uc);
  if (j > 0) acc += 0.5 * (pm_c(u, H, W, P, i, j - 1, ik2) + cc) * ((double)u[(size_t)i * P + j - 1] - uc);
  ((T*)x.dst)[(size_t)i * x.pd + j] = to_t<T>(uc + tau * acc);
}

// Pixel loop of one 64 x 16 tile of the destination grid.
template <typename T, int OP>
__device__ __forceinline__ void xfer_tile(const XArgs& x, int t) {
  const int tiles_x = (x.wd + kXW - 1) / kXW;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int j = tx * kXW + (threadIdx.x & 63);
  if (j >= x.wd) return;
  for (int k = 0; k < kXH / 4; ++k) {
    const int i = ty * kXH + (threadIdx.x >> 6) * (kXH / 4) + k;
    if (i >= x.hd) break;
    if (OP == kXfExtrap)
      pi_point<T>(x, i, j);
    else if (OP == kXfQuad)
      quad_point<T>(x, i, j);
    else if (OP == kXfLinear)
      linear_point<T>(x, i, j);
    else if (OP == kXfSmooth)
      smooth_point<T>(x, i, j);
    else
      pm_point<T>(x, i, j);
  }
}

__device__ __forceinline__ void* xbuf(const JobDesc& d, int sel) {
  switch (sel) {
    case kBufT1: return d.t1;
    case kBufT2: return d.t2;
    case kBufUB: return const_cast<void*>(d.uB);
    default: return d.u;
  }
}

// Engine form: the job's descriptor supplies the grids and buffers.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_xfer(LaunchList ll, const JobDesc* __restrict__ descs, int src, int dst) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  XArgs x;
  if (OP == kXfExtrap) {
    x.s0 = d.uA;
    x.h0 = d.hA; x.w0 = d.wA; x.p0 = d.pA;
    x.s1 = d.uB;
    x.h1 = d.hB; x.w1 = d.wB; x.p1 = d.pB;
    x.dst = xbuf(d, dst);
    x.hd = d.hB; x.wd = d.wB; x.pd = d.pB;
  } else {
    if (OP == kXfQuad || OP == kXfLinear) {
      x.s0 = xbuf(d, src);
      x.h0 = d.hB; x.w0 = d.wB; x.p0 = d.pB;
    } else {
      x.s0 = xbuf(d, src);
      x.h0 = d.h; x.w0 = d.w; x.p0 = d.pitch;
    }
    x.s1 = nullptr;
    x.h1 = x.w1 = x.p1 = 0;
    x.dst = xbuf(d, dst);
    x.hd = d.h; x.wd = d.w; x.pd = d.pitch;
  }
  x.a0 = (OP == kXfSmooth) ? d.smooth_h : d.pm_k;
  x.a1 = d.tau;
  xfer_tile<T, OP>(x, L.t);
}

// Operator form on one dense image.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_xfer_op(XArgs x) {
  xfer_tile<T, OP>(x, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Restriction (eq. 12-13) and output copy
// ---------------------------------------------------------------------------
// One pass over the dense finest-level input writes every level's
// right-hand side g_l(i, j) = g(2^(L-l) i, 2^(L-l) j) and initialises the
// solution pyramid (zero, or the given initial guess on the finest level).
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const int H = d.H, W = d.W, NL = d.L;
  const int tiles_x = (W + kXW - 1) / kXW;
  const int ty = L.t / tiles_x, tx = L.t - ty * tiles_x;
  const int x = tx * kXW + (threadIdx.x & 63);
  if (x >= W) return;
  const T* gin = (const T*)d.g_in;
  const T* uin = (const T*)d.u_in;
  for (int k = 0; k < kXH / 4; ++k) {
    const int y = ty * kXH + (threadIdx.x >> 6) * (kXH / 4) + k;
    if (y >= H) break;
    const T v = gin[(size_t)y * W + x];
    for (int l = NL - 1; l >= 0; --l) {
      const int sh = NL - 1 - l, m = (1 << sh) - 1;
      if ((y & m) || (x & m)) break;
      const size_t o = (size_t)(y >> sh) * d.lp[l] + (x >> sh);
      ((T*)d.g_lv[l])[o] = v;
      ((T*)d.u_lv[l])[o] = (l == NL - 1 && uin) ? uin[(size_t)y * W + x] : T(0);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_out_copy(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const int H = d.H, W = d.W;
  const int tiles_x = (W + kXW - 1) / kXW;
  const int ty = L.t / tiles_x, tx = L.t - ty * tiles_x;
  const int x = tx * kXW + (threadIdx.x & 63);
  if (x >= W) return;
  const T* u = (const T*)d.u_lv[d.L - 1];
  T* out = (T*)d.u_out;
  for (int k = 0; k < kXH / 4; ++k) {
    const int y = ty * kXH + (threadIdx.x >> 6) * (kXH / 4) + k;
    if (y >= H) break;
    out[(size_t)y * W + x] = u[(size_t)y * d.fine_pitch + x];
  }
}

// ---------------------------------------------------------------------------
// Operator-form convolution on one dense image (y = H x with given taps).
// ---------------------------------------------------------------------------
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void k_op_conv(const T* __restrict__ x, T* __restrict__ y, int H, int W,
                                                 const T* __restrict__ taps, int R) {
  __shared__ T tile[(kTH + 2 * RMAX) * (kTW + 2 * RMAX)];
  const int tiles_x = (W + kTW - 1) / kTW;
  TileGeo g;
  g.R = R;
  g.h = H;
  g.w = W;
  g.pitch = W;
  g.y0 = (blockIdx.x / tiles_x) * kTH;
  g.x0 = (blockIdx.x % tiles_x) * kTW;
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  load_tile<T, RMAX>(tile, g, [&](size_t o, bool) { return x[o]; });
  __syncthreads();
  T acc[kV];
  conv_tile<T, RMAX>(tile, R, taps, g.wave, g.lane, acc);
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int gy = g.y0 + g.wave * kV + v;
    if (gy < H && gx < W) y[(size_t)gy * W + gx] = acc[v];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_op_restrict(const T* __restrict__ gf, int Hf, int Wf, T* __restrict__ gc,
                                                     int Hc, int Wc) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= Hc * Wc) return;
  const int i = idx / Wc, j = idx - i * Wc;
  gc[idx] = gf[(size_t)(2 * i) * Wf + 2 * j];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int rmax_class_for(int r) { return r <= 3 ? 3 : (r <= 6 ? 6 : 12); }

static int tiles2(int h, int w, int th, int tw) { return ((h + th - 1) / th) * ((w + tw - 1) / tw); }

int blocks_for_stage(Stage st, const JobDesc& d) {
  switch (st) {
    case kRestrict:
    case kOutCopy: return tiles2(d.H, d.W, kXH, kXW);
    case kCgInit1:
    case kCgInit2:
    case kCgA:
    case kCgB:
    case kMrInit:
    case kMrPass: return d.ntiles;
    case kCgFinInit:
    case kCgFinA:
    case kCgFinB:
    case kMrFinInit:
    case kMrFin: return 1;
    case kXfExtrap: return tiles2(d.hB, d.wB, kXH, kXW);
    default: return tiles2(d.h, d.w, kXH, kXW);
  }
}

template <typename T, int RMAX>
static hipError_t launch_smoother(Stage st, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  const dim3 grid(ll.total), block(256);
  switch (st) {
    case kCgInit1:
    case kMrInit: hipLaunchKernelGGL((k_init1<T, RMAX>), grid, block, 0, s, ll, descs); break;
    case kCgInit2: hipLaunchKernelGGL((k_cg_init2<T, RMAX>), grid, block, 0, s, ll, descs); break;
    case kCgA: hipLaunchKernelGGL((k_cg_a<T, RMAX>), grid, block, 0, s, ll, descs); break;
    case kCgB: hipLaunchKernelGGL((k_cg_b<T, RMAX>), grid, block, 0, s, ll, descs); break;
    case kMrPass: hipLaunchKernelGGL((k_mr_pass<T, RMAX>), grid, block, 0, s, ll, descs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_typed(Stage st, int rmax_class, const LaunchList& ll, const JobDesc* descs, int src,
                               int dst, hipStream_t s) {
  const dim3 grid(ll.total), block(256);
  switch (st) {
    case kRestrict: hipLaunchKernelGGL(k_restrict<T>, grid, block, 0, s, ll, descs); return hipGetLastError();
    case kOutCopy: hipLaunchKernelGGL(k_out_copy<T>, grid, block, 0, s, ll, descs); return hipGetLastError();
    case kXfExtrap:
      hipLaunchKernelGGL((k_xfer<T, kXfExtrap>), grid, block, 0, s, ll, descs, src, dst);
      return hipGetLastError();
    case kXfQuad:
      hipLaunchKernelGGL((k_xfer<T, kXfQuad>), grid, block, 0, s, ll, descs, src, dst);
      return hipGetLastError();
    case kXfLinear:
      hipLaunchKernelGGL((k_xfer<T, kXfLinear>), grid, block, 0, s, ll, descs, src, dst);
      return hipGetLastError();
    case kXfSmooth:
      hipLaunchKernelGGL((k_xfer<T, kXfSmooth>), grid, block, 0, s, ll, descs, src, dst);
      return hipGetLastError();
    case kXfPm:
      hipLaunchKernelGGL((k_xfer<T, kXfPm>), grid, block, 0, s, ll, descs, src, dst);
      return hipGetLastError();
    default: break;
  }
  if (rmax_class <= 3) return launch_smoother<T, 3>(st, ll, descs, s);
  if (rmax_class <= 6) return launch_smoother<T, 6>(st, ll, descs, s);
  return launch_smoother<T, 12>(st, ll, descs, s);
}

hipError_t launch_stage(Stage st, bool f64, int rmax_class, const LaunchList& ll, const JobDesc* descs, int src,
                        int dst, hipStream_t s) {
  if (ll.n <= 0) return hipSuccess;
  const dim3 block(256);
  switch (st) {
    case kCgFinInit: hipLaunchKernelGGL(k_cg_fin_init, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kCgFinA: hipLaunchKernelGGL(k_cg_fin_a, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kCgFinB: hipLaunchKernelGGL(k_cg_fin_b, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kMrFinInit: hipLaunchKernelGGL(k_mr_fin_init, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kMrFin: hipLaunchKernelGGL(k_mr_fin, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    default: break;
  }
  return f64 ? launch_typed<double>(st, rmax_class, ll, descs, src, dst, s)
             : launch_typed<float>(st, rmax_class, ll, descs, src, dst, s);
}

template <typename T>
static hipError_t op_conv_t(const void* x, void* y, int H, int W, const void* taps, int r, hipStream_t s) {
  const int blocks = tiles2(H, W, kTH, kTW);
  const int rc = rmax_class_for(r);
  if (rc <= 3)
    hipLaunchKernelGGL((k_op_conv<T, 3>), dim3(blocks), dim3(256), 0, s, (const T*)x, (T*)y, H, W, (const T*)taps, r);
  else if (rc <= 6)
    hipLaunchKernelGGL((k_op_conv<T, 6>), dim3(blocks), dim3(256), 0, s, (const T*)x, (T*)y, H, W, (const T*)taps, r);
  else
    hipLaunchKernelGGL((k_op_conv<T, 12>), dim3(blocks), dim3(256), 0, s, (const T*)x, (T*)y, H, W, (const T*)taps,
                       r);
  return hipGetLastError();
}

hipError_t op_conv(const void* x, void* y, int H, int W, const void* taps, int r, bool f64, hipStream_t s) {
  return f64 ? op_conv_t<double>(x, y, H, W, taps, r, s) : op_conv_t<float>(x, y, H, W, taps, r, s);
}

hipError_t op_restrict(const void* gf, int Hf, int Wf, void* gc, bool f64, hipStream_t s) {
  const int Hc = (Hf + 1) / 2, Wc = (Wf + 1) / 2;
  const int blocks = (Hc * Wc + 255) / 256;
  if (f64)
    hipLaunchKernelGGL(k_op_restrict<double>, dim3(blocks), dim3(256), 0, s, (const double*)gf, Hf, Wf, (double*)gc,
                       Hc, Wc);
  else
    hipLaunchKernelGGL(k_op_restrict<float>, dim3(blocks), dim3(256), 0, s, (const float*)gf, Hf, Wf, (float*)gc, Hc,
                       Wc);
  return hipGetLastError();
}

template <int OP>
static hipError_t op_xfer(const XArgs& x, bool f64, hipStream_t s) {
  const int blocks = tiles2(x.hd, x.wd, kXH, kXW);
  if (f64)
    hipLaunchKernelGGL((k_xfer_op<double, OP>), dim3(blocks), dim3(256), 0, s, x);
  else
    hipLaunchKernelGGL((k_xfer_op<float, OP>), dim3(blocks), dim3(256), 0, s, x);
  return hipGetLastError();
}

hipError_t op_extrapolate(const void* uA, const void* uB, int HB, int WB, void* ut, bool f64, hipStream_t s) {
  XArgs x{};
  x.s0 = uA;
  x.h0 = (HB + 1) / 2;
  x.w0 = (WB + 1) / 2;
  x.p0 = x.w0;
  x.s1 = uB;
  x.h1 = HB;
  x.w1 = WB;
  x.p1 = WB;
  x.dst = ut;
  x.hd = HB;
  x.wd = WB;
  x.pd = WB;
  return op_xfer<kXfExtrap>(x, f64, s);
}

hipError_t op_prolong_quad(const void* ut, int HC, int WC, void* uC, bool f64, hipStream_t s) {
  XArgs x{};
  x.s0 = ut;
  x.h0 = (HC + 1) / 2;
  x.w0 = (WC + 1) / 2;
  x.p0 = x.w0;
  x.dst = uC;
  x.hd = HC;
  x.wd = WC;
  x.pd = WC;
  return op_xfer<kXfQuad>(x, f64, s);
}

hipError_t op_prolong_linear(const void* uB, int HC, int WC, void* uC, bool f64, hipStream_t s) {
  XArgs x{};
  x.s0 = uB;
  x.h0 = (HC + 1) / 2;
  x.w0 = (WC + 1) / 2;
  x.p0 = x.w0;
  x.dst = uC;
  x.hd = HC;
  x.wd = WC;
  x.pd = WC;
  return op_xfer<kXfLinear>(x, f64, s);
}

hipError_t op_local_smooth(const void* u, void* out, int H, int W, double h, bool f64, hipStream_t s) {
  XArgs x{};
  x.s0 = u;
  x.h0 = H;
  x.w0 = W;
  x.p0 = W;
  x.dst = out;
  x.hd = H;
  x.wd = W;
  x.pd = W;
  x.a0 = h;
  return op_xfer<kXfSmooth>(x, f64, s);
}

hipError_t op_pm_step(const void* u, void* out, int H, int W, double k, double tau, bool f64, hipStream_t s) {
  XArgs x{};
  x.s0 = u;
  x.h0 = H;
  x.w0 = W;
  x.p0 = W;
  x.dst = out;
  x.hd = H;
  x.wd = W;
  x.pd = W;
  x.a0 = k;
  x.a1 = tau;
  return op_xfer<kXfPm>(x, f64, s);
}

}  // namespace eecmg
