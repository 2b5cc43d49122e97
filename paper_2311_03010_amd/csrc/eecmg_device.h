// Device-side building blocks of the EECMG kernels (gfx950, wave64):
// launch-list lookup, fixed-order FP64 reductions, LDS tile staging, the
// blur-operator policies and the smoother pass kernels templated on them.
#pragma once

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

// Pointers taken from a job descriptor are generic; casting them to the global
// address space lets the compiler emit global (not flat) loads and stores
// with a scalar base and a 32-bit offset.
#define EECMG_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ EECMG_G T* gp(void* p) {
  return (EECMG_G T*)p;
}
template <typename T>
__device__ __forceinline__ const EECMG_G T* gpc(const void* p) {
  return (const EECMG_G T*)p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum NV per-lane FP64 values over an NT-thread block in a fixed order and
// store them (thread 0) to out[i * stride], i < NV.
template <int NT, int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* __restrict__ out, int stride) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if constexpr (NT == 64) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) out[i * stride] = v[i];
    }
  } else {
    constexpr int NW = NT / 64;
    __shared__ double red[NW][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double s = red[0][i];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += red[w][i];
        out[i * stride] = s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Blur-operator policies.  Each policy evaluates, for the lane's column
// x0 + lane of a TH x TW output tile, (H x)(i, j) = sum_{a,b} psf(a,b) x(i-a, j-b)
// from an LDS tile holding rows [y0 - R, y0 + TH + R) and columns
// [x0 - R, x0 + TW + R) (zero outside the image), and calls
// emit(row, value) for each output row of the lane as soon as it is
// complete.  H^T is the same operator with the flipped PSF (the host passes
// flipped taps).
// ---------------------------------------------------------------------------

// General PSF: all (2R+1)^2 taps, R known at run time (R <= RMAX).  Four waves
// share a 64 x 32 tile, kV = 8 output rows each; for each column offset b a
// lane loads its column segment once into registers (shifted so that every
// register index is a compile-time constant) and applies every row offset.
template <typename T, int RMAX>
struct ConvGeneral {
  static constexpr int NT = 256, TW = kTW, TH = kTH, LW = kTW + 2 * RMAX, LH = kTH + 2 * RMAX, RC = RMAX;
  static constexpr bool kRuntimeR = true;
  template <typename Emit>
  __device__ static __forceinline__ void conv(const T* __restrict__ tile, const T* __restrict__ taps, int R, int wave,
                                              int lane, Emit emit) {
    T acc[kV];
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
#pragma unroll
    for (int v = 0; v < kV; ++v) emit(wave * kV + v, acc[v]);
  }
};

// Sliding-column scheme shared by the separable and symmetric policies.  The
// lane walks down its column one LDS row t at a time; row t feeds the outputs
// v = t - R + a (a = R .. -R), so output v receives its first contribution at
// t = v and is complete after t = v + 2R.  Exactly NW = 2R + 1 outputs are
// pending at any time, so they live in a circular register buffer indexed by
// v mod NW.  The row loop runs in groups of NW rows with the group body
// unrolled: every register index is then a compile-time constant (no dynamic
// VGPR indexing) whatever the tile height.  Rows past the tile only feed
// outputs v >= TH, which are never emitted; the LDS tile is padded to whole
// groups so those reads stay inside it.
template <int R>
struct Slide {
  static constexpr int NW = 2 * R + 1;
  static constexpr int LH = kTH + 2 * R;
  static constexpr int NG = (LH + NW - 1) / NW;
  static constexpr int LH_PAD = NG * NW;
  static constexpr int slot(int k, int a) { return ((k - R + a) % NW + NW) % NW; }
};

// Rank-one PSF psf(a,b) = col(a) row(b) (the Gaussian of Section 5 and its
// coarse levels).  For each LDS row the lane forms the horizontal filter
// h = sum_b row(b) x(., j-b) once and adds col(a) h to the pending outputs.
// Taps: row(-R..R) followed by col(-R..R).
template <typename T, int R>
struct ConvSep {
  using S = Slide<R>;
  static constexpr int NT = 64, TW = kTW, TH = kTH, LW = kTW + 2 * R, LH = S::LH_PAD, RC = R;
  static constexpr bool kRuntimeR = false;
  template <typename Emit>
  __device__ static __forceinline__ void conv(const T* __restrict__ tile, const T* __restrict__ taps, int, int,
                                              int lane, Emit emit) {
    constexpr int NW = S::NW;
    T rw[NW], cl[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      rw[k] = taps[k];
      cl[k] = taps[NW + k];
    }
    T acc[NW];
#pragma unroll 1
    for (int gi = 0; gi < S::NG; ++gi) {
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int t = gi * NW + k;
        const T* __restrict__ row = tile + t * LW + lane + R;
        T h = rw[0] * row[R];
#pragma unroll
        for (int b = -R + 1; b <= R; ++b) h = fma(rw[b + R], row[-b], h);
#pragma unroll
        for (int a = R; a >= -R; --a) {
          if (a == R)
            acc[S::slot(k, a)] = cl[a + R] * h;
          else
            acc[S::slot(k, a)] = fma(cl[a + R], h, acc[S::slot(k, a)]);
        }
        const int vd = t - 2 * R;
        if (vd >= 0 && vd < TH) emit(vd, acc[S::slot(k, -R)]);
      }
    }
  }
};

// Largest b with a^2 + b^2 <= R^2 (disk support), or R (square support).
constexpr int sym_span(int R, bool disk, int a) {
  if (!disk) return R;
  int b = 0;
  while ((b + 1) * (b + 1) + a * a <= R * R) ++b;
  return b;
}
constexpr int sym_offset(int R, bool disk, int a) {
  int o = 0;
  for (int k = 0; k < a; ++k) o += sym_span(R, disk, k) + 1;
  return o;
}
constexpr int sym_ntaps(int R, bool disk) { return sym_offset(R, disk, R + 1); }

// PSF symmetric under both axis reflections, psf(a,b) = psf(-a,b) = psf(a,-b),
// with square or disk support (the out-of-focus disk of the 4096^2
// workload).  Rows a and -a share one horizontal "row filter"
//   h_a = psf(a,0) x(j) + sum_{b>=1} psf(a,b) (x(j-b) + x(j+b)),
// computed once per LDS row from the pair sums and added to the outputs a
// rows below and above: about (R+1)(R+2)/2 + 2R ops per row and pixel
// instead of (2R+1)^2 FMAs.  Taps: the quadrant a, b >= 0, row by row
// (b = 0..span(a)).
template <typename T, int R, bool DISK>
struct ConvSym {
  using S = Slide<R>;
  static constexpr int NT = 64, TW = kTW, TH = kTH, LW = kTW + 2 * R, LH = S::LH_PAD, RC = R;
  static constexpr bool kRuntimeR = false;
  static constexpr int NTAPS = sym_ntaps(R, DISK);
  template <typename Emit>
  __device__ static __forceinline__ void conv(const T* __restrict__ tile, const T* __restrict__ taps, int, int,
                                              int lane, Emit emit) {
    constexpr int NW = S::NW;
    T wt[NTAPS];
#pragma unroll
    for (int k = 0; k < NTAPS; ++k) wt[k] = taps[k];
    T acc[NW];
#pragma unroll 1
    for (int gi = 0; gi < S::NG; ++gi) {
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int t = gi * NW + k;
        const T* __restrict__ row = tile + t * LW + lane + R;
        const T x0 = row[0];
        T pr[R + 1];
#pragma unroll
        for (int b = 1; b <= R; ++b) pr[b] = row[b] + row[-b];
        T h[R + 1];
#pragma unroll
        for (int a = 0; a <= R; ++a) {
          const int o = sym_offset(R, DISK, a);
          T v = wt[o] * x0;
#pragma unroll
          for (int b = 1; b <= R; ++b)
            if (b <= sym_span(R, DISK, a)) v = fma(wt[o + b], pr[b], v);
          h[a] = v;
        }
#pragma unroll
        for (int a = R; a >= -R; --a) {
          const T hv = h[a >= 0 ? a : -a];
          if (a == R)
            acc[S::slot(k, a)] = hv;
          else
            acc[S::slot(k, a)] = acc[S::slot(k, a)] + hv;
        }
        const int vd = t - 2 * R;
        if (vd >= 0 && vd < TH) emit(vd, acc[S::slot(k, -R)]);
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Tile staging
// ---------------------------------------------------------------------------
struct TileGeo {
  int R, h, w, pitch, y0, x0, wave, lane;
};

template <typename P>
__device__ __forceinline__ TileGeo tile_geo(const JobDesc& d, int t) {
  TileGeo g;
  g.R = uni(d.rad);
  g.h = uni(d.h);
  g.w = uni(d.w);
  g.pitch = uni(d.pitch);
  const int tiles_x = uni(d.tiles_x);
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  g.y0 = ty * P::TH;
  g.x0 = tx * P::TW;
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  return g;
}

// Load tile + halo: every tile element in the image gets combine(load(o)),
// elements outside the image are zero (the operator's zero boundary
// condition); o is the element's 32-bit offset in the level's pitched array.
// For compile-time radii the loop is fully unrolled in two phases: every
// global load is issued first, from an address clamped into the image (always
// valid), then the values are combined (branch-free) and written to LDS, so a
// wave keeps dozens of loads in flight instead of waiting row by row.
template <typename T, typename P, typename LoadF, typename CombF>
__device__ __forceinline__ void load_tile(T* __restrict__ tile, const TileGeo& g, LoadF load, CombF combine) {
  if constexpr (P::kRuntimeR) {
    const int R = g.R;
    constexpr int NWV = P::NT / 64;
    for (int ly = g.wave; ly < P::TH + 2 * R; ly += NWV) {
      const int gy = g.y0 - R + ly;
      const bool row_in = gy >= 0 && gy < g.h;
      for (int lx = g.lane; lx < P::TW + 2 * R; lx += 64) {
        const int gx = g.x0 - R + lx;
        T v = T(0);
        if (row_in && gx >= 0 && gx < g.w) v = combine(load((unsigned)(gy * g.pitch + gx)));
        tile[ly * P::LW + lx] = v;
      }
    }
  } else {
    constexpr int R = P::RC, LWr = P::TW + 2 * R, N = LWr * (P::TH + 2 * R);
    constexpr int IT = (N + P::NT - 1) / P::NT;
    using V = decltype(load(0u));
    V vals[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = (int)threadIdx.x + k * P::NT;
      const int ly = idx / LWr, lx = idx - ly * LWr;
      const int gy = min(max(g.y0 - R + ly, 0), g.h - 1);
      const int gx = min(max(g.x0 - R + lx, 0), g.w - 1);
      vals[k] = load((unsigned)(gy * g.pitch + gx));
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = (int)threadIdx.x + k * P::NT;
      if (k < IT - 1 || idx < N) {
        const int ly = idx / LWr, lx = idx - ly * LWr;
        const int gy = g.y0 - R + ly, gx = g.x0 - R + lx;
        const bool ok = gy >= 0 && gy < g.h && gx >= 0 && gx < g.w;
        const T v = combine(vals[k]);
        tile[ly * P::LW + lx] = ok ? v : T(0);
      }
    }
  }
}

// The tile's own output pixels (no halo), one column per lane, rows split
// between the waves: f(load(o), o, row) for every in-image pixel, with all
// loads issued as one burst (from clamped, always valid addresses).
template <typename P, typename LoadF, typename UseF>
__device__ __forceinline__ void for_interior(const TileGeo& g, LoadF load, UseF use) {
  constexpr int NWV = P::NT / 64, ROWS = P::TH / NWV;
  const int gx = g.x0 + g.lane;
  const int gxc = min(gx, g.w - 1);
  using V = decltype(load(0u));
  V vals[ROWS];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int gy = min(g.y0 + g.wave * ROWS + i, g.h - 1);
    vals[i] = load((unsigned)(gy * g.pitch + gxc));
  }
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int gy = g.y0 + g.wave * ROWS + i;
    if (gy < g.h && gx < g.w) use(vals[i], (unsigned)(gy * g.pitch + gx), g.wave * ROWS + i);
  }
}

// Interior pixels read back from the LDS tile (after the barrier that follows
// load_tile): use(v, o, in_image) for the lane's rows; the caller predicates
// its stores on in_image.
template <typename T, typename P, typename UseF>
__device__ __forceinline__ void tile_interior(const T* __restrict__ tile, const TileGeo& g, int R, UseF use) {
  constexpr int NWV = P::NT / 64, ROWS = P::TH / NWV;
  const int gx = g.x0 + g.lane;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    const int row = g.wave * ROWS + i;
    const int gy = g.y0 + row;
    use(tile[(row + R) * P::LW + g.lane + R], (unsigned)(gy * g.pitch + gx), gy < g.h && gx < g.w);
  }
}

template <typename P>
__device__ __forceinline__ int pol_R(const TileGeo& g) {
  return P::kRuntimeR ? g.R : (P::LW - P::TW) / 2;
}

// ---------------------------------------------------------------------------
// Smoother pass kernels, templated on the element type and blur policy.
// ---------------------------------------------------------------------------

template <typename T>
struct Two {
  T a, b;
};

// r = g - H u0, stored in r[0]; partial <r,r> in slot 1.  (CGLS and MR)
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_init1(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[P::LH * P::LW];
  __shared__ T gsh[P::TH * P::TW];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo<P>(d, L.t);
  const auto* __restrict__ u = gpc<T>(d.u);
  const auto* __restrict__ gg = gpc<T>(d.g);
  auto* __restrict__ r = gp<T>(d.r[0]);
  load_tile<T, P>(tile, g, [&](unsigned o) { return u[o]; }, [](T v) { return v; });
  for_interior<P>(g, [&](unsigned o) { return gg[o]; }, [&](T v, unsigned, int row) { gsh[row * P::TW + g.lane] = v; });
  __syncthreads();
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
  P::conv(tile, (const T*)d.taps, g.R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    const T rv = gsh[v * P::TW + g.lane] - acc;
    if (gy < g.h && gx < g.w) {
      r[(unsigned)(gy * g.pitch + gx)] = rv;
      part[0] += (double)rv * (double)rv;
    }
  });
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)1 * d.pstride + L.t, d.pstride);
}

// s = H^T r, p[0] = s; partial <s,s> in slot 2.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_cg_init2(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[P::LH * P::LW];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo<P>(d, L.t);
  const auto* __restrict__ r = gpc<T>(d.r[0]);
  auto* __restrict__ s = gp<T>(d.s);
  auto* __restrict__ p = gp<T>(d.p[0]);
  load_tile<T, P>(tile, g, [&](unsigned o) { return r[o]; }, [](T v) { return v; });
  __syncthreads();
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
  P::conv(tile, (const T*)d.taps_t, g.R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    if (gy < g.h && gx < g.w) {
      const unsigned o = (unsigned)(gy * g.pitch + gx);
      s[o] = acc;
      p[o] = acc;
      part[0] += (double)acc * (double)acc;
    }
  });
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)2 * d.pstride + L.t, d.pstride);
}

// Pass A of iteration k: p_new = s + beta p_old (on tile + halo), q = H p_new;
// partial <q,q> in slot 0.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_cg_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[P::LH * P::LW];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int par = uni(st->par);
  const T beta = (T)st->beta;
  const auto* __restrict__ s = gpc<T>(d.s);
  const auto* __restrict__ po = gpc<T>(d.p[par]);
  auto* __restrict__ pn = gp<T>(d.p[par ^ 1]);
  auto* __restrict__ q = gp<T>(d.q[0]);
  load_tile<T, P>(
      tile, g, [&](unsigned o) { return Two<T>{s[o], po[o]}; }, [&](Two<T> x) { return fma(beta, x.b, x.a); });
  __syncthreads();
  tile_interior<T, P>(tile, g, pol_R<P>(g), [&](T v, unsigned o, bool in) {
    if (in) pn[o] = v;
  });
  double part[1] = {0.0};
  const int gx = g.x0 + g.lane;
  P::conv(tile, (const T*)d.taps, g.R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    if (gy < g.h && gx < g.w) {
      q[(unsigned)(gy * g.pitch + gx)] = acc;
      part[0] += (double)acc * (double)acc;
    }
  });
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)0 * d.pstride + L.t, d.pstride);
}

// Pass B of iteration k: r_new = r - alpha q (tile + halo), u += alpha p_new,
// s = H^T r_new; partials <r,r> (slot 1) and <s,s> (slot 2).
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_cg_b(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[P::LH * P::LW];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int par = uni(st->par);
  const T alpha = (T)st->alpha;
  const auto* __restrict__ ro = gpc<T>(d.r[par]);
  auto* __restrict__ rn = gp<T>(d.r[par ^ 1]);
  const auto* __restrict__ q = gpc<T>(d.q[0]);
  const auto* __restrict__ pn = gpc<T>(d.p[par ^ 1]);
  auto* __restrict__ u = gp<T>(d.u);
  auto* __restrict__ s = gp<T>(d.s);
  double part[2] = {0.0, 0.0};
  load_tile<T, P>(
      tile, g, [&](unsigned o) { return Two<T>{ro[o], q[o]}; }, [&](Two<T> x) { return fma(-alpha, x.b, x.a); });
  for_interior<P>(
      g, [&](unsigned o) { return Two<T>{u[o], pn[o]}; },
      [&](Two<T> x, unsigned o, int) { u[o] = fma(alpha, x.b, x.a); });
  __syncthreads();
  tile_interior<T, P>(tile, g, pol_R<P>(g), [&](T v, unsigned o, bool in) {
    if (in) rn[o] = v;
    part[0] += in ? (double)v * (double)v : 0.0;
  });
  const int gx = g.x0 + g.lane;
  P::conv(tile, (const T*)d.taps_t, g.R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    if (gy < g.h && gx < g.w) {
      s[(unsigned)(gy * g.pitch + gx)] = acc;
      part[1] += (double)acc * (double)acc;
    }
  });
  block_sum_store<P::NT, 2>(part, d.partials + (size_t)1 * d.pstride + L.t, d.pstride);
}

// MR pass: if a step alpha is pending, r_new = r - alpha q and u += alpha r;
// then q_new = H r_new.  Partials <r_new,q_new> (0), <r_new,r_new> (1), <q,q> (2).
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_mr_pass(LaunchList ll, const JobDesc* __restrict__ descs) {
  __shared__ T tile[P::LH * P::LW];
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int R = pol_R<P>(g);
  const int par = uni(st->par);
  const bool pending = uni(st->pending) != 0;
  const T alpha = pending ? (T)st->alpha : T(0);
  const auto* __restrict__ ro = gpc<T>(d.r[par]);
  const auto* __restrict__ qo = gpc<T>(d.q[par]);
  auto* __restrict__ rn = gp<T>(d.r[par ^ 1]);
  auto* __restrict__ qn = gp<T>(d.q[par ^ 1]);
  auto* __restrict__ u = gp<T>(d.u);
  double part[3] = {0.0, 0.0, 0.0};
  if (pending) {
    load_tile<T, P>(
        tile, g, [&](unsigned o) { return Two<T>{ro[o], qo[o]}; }, [&](Two<T> x) { return fma(-alpha, x.b, x.a); });
    for_interior<P>(
        g, [&](unsigned o) { return Two<T>{u[o], ro[o]}; },
        [&](Two<T> x, unsigned o, int) { u[o] = fma(alpha, x.b, x.a); });
  } else {
    load_tile<T, P>(tile, g, [&](unsigned o) { return ro[o]; }, [](T v) { return v; });
  }
  __syncthreads();
  tile_interior<T, P>(tile, g, R, [&](T v, unsigned o, bool in) {
    if (in) rn[o] = v;
    part[1] += in ? (double)v * (double)v : 0.0;
  });
  const int gx = g.x0 + g.lane;
  P::conv(tile, (const T*)d.taps, g.R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    if (gy < g.h && gx < g.w) {
      qn[(unsigned)(gy * g.pitch + gx)] = acc;
      const T rc = tile[(v + R) * P::LW + g.lane + R];
      part[0] += (double)rc * (double)acc;
      part[2] += (double)acc * (double)acc;
    }
  });
  block_sum_store<P::NT, 3>(part, d.partials + (size_t)0 * d.pstride + L.t, d.pstride);
}

// Operator form: y = H x on one dense image with the given taps layout.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_op_conv(const T* __restrict__ x, T* __restrict__ y, int H, int W,
                                                   const T* __restrict__ taps, int R) {
  __shared__ T tile[P::LH * P::LW];
  const int tiles_x = (W + P::TW - 1) / P::TW;
  TileGeo g;
  g.R = R;
  g.h = H;
  g.w = W;
  g.pitch = W;
  g.y0 = (blockIdx.x / tiles_x) * P::TH;
  g.x0 = (blockIdx.x % tiles_x) * P::TW;
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  load_tile<T, P>(tile, g, [&](unsigned o) { return x[o]; }, [](T v) { return v; });
  __syncthreads();
  const int gx = g.x0 + g.lane;
  P::conv(tile, taps, R, g.wave, g.lane, [&](int v, T acc) {
    const int gy = g.y0 + v;
    if (gy < H && gx < W) y[(unsigned)(gy * W + gx)] = acc;
  });
}

// Dispatch of one smoother stage for one policy.
template <typename T, typename P>
hipError_t launch_policy(Stage st, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  const dim3 grid(ll.total), block(P::NT);
  switch (st) {
    case kCgInit1:
    case kMrInit: hipLaunchKernelGGL((k_init1<T, P>), grid, block, 0, s, ll, descs); break;
    case kCgInit2: hipLaunchKernelGGL((k_cg_init2<T, P>), grid, block, 0, s, ll, descs); break;
    case kCgA: hipLaunchKernelGGL((k_cg_a<T, P>), grid, block, 0, s, ll, descs); break;
    case kCgB: hipLaunchKernelGGL((k_cg_b<T, P>), grid, block, 0, s, ll, descs); break;
    case kMrPass: hipLaunchKernelGGL((k_mr_pass<T, P>), grid, block, 0, s, ll, descs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_op_conv(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  const int blocks = ((H + P::TH - 1) / P::TH) * ((W + P::TW - 1) / P::TW);
  hipLaunchKernelGGL((k_op_conv<T, P>), dim3(blocks), dim3(P::NT), 0, s, (const T*)x, (T*)y, H, W, (const T*)taps,
                     R);
  return hipGetLastError();
}

}  // namespace eecmg
