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

// Pointers taken from a job descriptor are generic; GPtr casts them to the
// global address space and indexes with a 32-bit byte offset, so the compiler
// emits global (not flat) loads and stores with a scalar base and one VGPR
// offset.  Every level array is below 4 GiB (checked when a job is planned).
#define EECMG_G __attribute__((address_space(1)))
template <typename T>
struct GPtr {
  EECMG_G T* p;
  __device__ __forceinline__ EECMG_G T& operator[](unsigned o) const {
    return *(EECMG_G T*)((EECMG_G char*)p + o * (unsigned)sizeof(T));
  }
};
template <typename T>
struct GPtrC {
  const EECMG_G T* p;
  __device__ __forceinline__ const EECMG_G T& operator[](unsigned o) const {
    return *(const EECMG_G T*)((const EECMG_G char*)p + o * (unsigned)sizeof(T));
  }
};
// Buffer view of one array for the streaming kernels: raw buffer loads and
// stores whose range the hardware checks against the array size, so an
// access at element offset >= n reads 0 and a store there is dropped.  The
// kernels pass offset `n` (the view's `none`) for pixels outside the image
// and need neither clamping nor branches around memory operations.
template <typename T>
struct BufView {
  __amdgpu_buffer_rsrc_t rs;
  __device__ __forceinline__ T ld(unsigned o) const {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, o * 4u, 0, 0));
    } else {
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, o * 8u, 0, 0));
    }
  }
  __device__ __forceinline__ void st(unsigned o, T v) const {
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, o * 4u, 0, 0);
    } else {
      using V2 = unsigned __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), rs, o * 8u, 0, 0);
    }
  }
};
// n: elements in the array (the level's h x pitch); below 2^32 bytes.
template <typename T>
__device__ __forceinline__ BufView<T> bview(const void* p, unsigned n) {
  return BufView<T>{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(n * (unsigned)sizeof(T)),
                                                      0x00020000)};
}

template <typename T>
__device__ __forceinline__ GPtr<T> gp(void* p) {
  return GPtr<T>{(EECMG_G T*)p};
}
template <typename T>
__device__ __forceinline__ GPtrC<T> gpc(const void* p) {
  return GPtrC<T>{(const EECMG_G T*)p};
}

// Order a wave's LDS stores before its following LDS loads (of other lanes'
// values).  The LDS unit performs one wave's operations in issue order, so
// only the compiler has to be kept from moving them across each other; the
// waves of a block run independently.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// share a 64 x TH_ tile (TH_ = 32, or short tiles on small levels), KV = TH_/4
// output rows each; for each column offset b a lane loads its column segment
// once into registers (shifted so that every register index is a
// compile-time constant) and applies every row offset.
template <typename T, int RMAX, int TH_ = kTH>
struct ConvGeneral {
  static_assert(TH_ % 4 == 0, "four waves share the tile rows");
  static constexpr int KV = TH_ / 4;
  static constexpr int NT = 256, TW = kTW, TH = TH_, LW = kTW + 2 * RMAX, LH = TH_ + 2 * RMAX, RC = RMAX;
  static constexpr bool kRuntimeR = true, kStream = false, kVSym = false;
  static constexpr int kWavesPerEU = 1;
  template <typename Emit>
  __device__ static __forceinline__ void conv(const T* __restrict__ tile, const T* __restrict__ taps, int R, int wave,
                                              int lane, Emit emit) {
    T acc[KV];
#pragma unroll
    for (int v = 0; v < KV; ++v) acc[v] = T(0);
    const int n = 2 * R + 1;
    for (int b = -R; b <= R; ++b) {
      T xc[KV + 2 * RMAX];
      const int col = lane + R - b;
#pragma unroll
      for (int t = 0; t < KV + 2 * RMAX; ++t) {
        const int lr = wave * KV + t - (RMAX - R);
        xc[t] = (t >= RMAX - R && t < RMAX + R + KV) ? tile[lr * LW + col] : T(0);
      }
#pragma unroll
      for (int a = -RMAX; a <= RMAX; ++a) {
        if (a >= -R && a <= R) {
          const T wt = taps[(a + R) * n + (b + R)];
#pragma unroll
          for (int v = 0; v < KV; ++v) acc[v] = fma(wt, xc[v + RMAX - a], acc[v]);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < KV; ++v) emit(wave * KV + v, acc[v]);
  }
};

// Sliding-column scheme shared by the separable, symmetric and uniform-disk
// policies.  The lane walks down its column one input row t at a time; row t
// feeds the outputs v = t - R + a (a = R .. -R), so output v receives its
// first contribution at t = v and is complete after t = v + 2R.  Exactly
// NW = 2R + 1 outputs are pending at any time, so they live in a circular
// register buffer indexed by v mod NW.  The row loop runs in groups of NW rows
// with the group body unrolled: every register index is then a compile-time
// constant (no dynamic VGPR indexing) whatever the strip height.
//
// A policy provides St (its taps and the pending outputs), init(St&, taps)
// and step(St&, row, k): consume the input row whose centre element for the
// lane is row[0] (row[b] is column offset b), with k = t mod NW, and return
// output t - 2R (meaningful once t >= 2R).
template <int R>
struct Slide {
  static constexpr int NW = 2 * R + 1;
  static constexpr int slot(int k, int a) { return ((k - R + a) % NW + NW) % NW; }
  // Materialise the pending outputs at the end of each row: keeps the
  // compiler from deferring the additions (and every row filter feeding
  // them) to the end of the unrolled group, which multiplies register use.
  template <typename T>
  __device__ static __forceinline__ void pin(T (&acc)[NW]) {
#pragma unroll
    for (int i = 0; i < NW; ++i) asm volatile("" : "+v"(acc[i]));
  }
};

// Minimum waves per SIMD requested for a streaming kernel holding `regs`
// values of per-lane state besides its pending outputs (FP32 only: the FP64
// state is twice as large and left to the allocator).
template <typename T>
constexpr int stream_waves(int R, int regs) {
  return sizeof(T) != 4 ? 1 : (2 * R + 1 + regs <= 22 ? 6 : (2 * R + 1 + regs <= 40 ? 4 : 1));
}

// Rank-one PSF psf(a,b) = col(a) row(b) (the Gaussian of Section 5 and its
// coarse levels).  For each input row the lane forms the horizontal filter
// h = sum_b row(b) x(., j-b) once and adds col(a) h to the pending outputs.
// Taps: row(-R..R) followed by col(-R..R).  SM: strip mode (strip_th).
template <typename T, int R, int SM = 0>
struct ConvSep {
  using S = Slide<R>;
  static constexpr int NT = 64 * kStripsPerBlock, TW = kTW, TH = strip_th(R, SM), LW = kTW + 2 * R, RC = R;
  static constexpr bool kRuntimeR = false, kStream = true;
  static constexpr bool kVSym = false;  // the column filter need not be symmetric
  // streaming kernels hide memory latency with waves: ask the register
  // allocator for at least this many per SIMD where the state fits (it
  // otherwise trades occupancy for instruction-level parallelism)
  static constexpr int kWavesPerEU = stream_waves<T>(R, 2 * (2 * R + 1));
  struct St {
    T rw[S::NW], cl[S::NW], acc[S::NW];
  };
  __device__ static __forceinline__ void init(St& s, const T* __restrict__ taps) {
#pragma unroll
    for (int k = 0; k < S::NW; ++k) {
      s.rw[k] = taps[k];
      s.cl[k] = taps[S::NW + k];
    }
  }
  __device__ static __forceinline__ T step(St& s, const T* __restrict__ row, int k) {
    T h = s.rw[0] * row[R];
#pragma unroll
    for (int b = -R + 1; b <= R; ++b) h = fma(s.rw[b + R], row[-b], h);
#pragma unroll
    for (int a = R; a >= -R; --a) {
      if (a == R)
        s.acc[S::slot(k, a)] = s.cl[a + R] * h;
      else
        s.acc[S::slot(k, a)] = fma(s.cl[a + R], h, s.acc[S::slot(k, a)]);
    }
    S::pin(s.acc);
    return s.acc[S::slot(k, -R)];
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
// with square or disk support.  Rows a and -a share one horizontal "row
// filter"
//   h_a = psf(a,0) x(j) + sum_{b>=1} psf(a,b) (x(j-b) + x(j+b)),
// computed once per input row from the pair sums and added to the outputs a
// rows below and above: about (R+1)(R+2)/2 + 2R ops per row and pixel
// instead of (2R+1)^2 FMAs.  Taps: the quadrant a, b >= 0, row by row
// (b = 0..span(a)).
template <typename T, int R, bool DISK, int SM = 0>
struct ConvSym {
  using S = Slide<R>;
  static constexpr int NT = 64 * kStripsPerBlock, TW = kTW, TH = strip_th(R, SM), LW = kTW + 2 * R, RC = R;
  static constexpr bool kRuntimeR = false, kStream = true;
  static constexpr bool kVSym = true;  // symmetric in the vertical direction: strips may walk up
  // streaming kernels hide memory latency with waves: ask the register
  // allocator for at least this many per SIMD where the state fits (it
  // otherwise trades occupancy for instruction-level parallelism)
  static constexpr int NTAPS = sym_ntaps(R, DISK);
  static constexpr int kWavesPerEU = stream_waves<T>(R, NTAPS);
  struct St {
    T wt[NTAPS], acc[S::NW];
  };
  __device__ static __forceinline__ void init(St& s, const T* __restrict__ taps) {
#pragma unroll
    for (int k = 0; k < NTAPS; ++k) s.wt[k] = taps[k];
  }
  __device__ static __forceinline__ T step(St& s, const T* __restrict__ row, int k) {
    const T x0 = row[0];
    T pr[R + 1];
#pragma unroll
    for (int b = 1; b <= R; ++b) pr[b] = row[b] + row[-b];
    T h[R + 1];
#pragma unroll
    for (int a = 0; a <= R; ++a) {
      const int o = sym_offset(R, DISK, a);
      T v = s.wt[o] * x0;
#pragma unroll
      for (int b = 1; b <= R; ++b)
        if (b <= sym_span(R, DISK, a)) v = fma(s.wt[o + b], pr[b], v);
      h[a] = v;
    }
#pragma unroll
    for (int a = R; a >= -R; --a) {
      const T hv = h[a >= 0 ? a : -a];
      if (a == R)
        s.acc[S::slot(k, a)] = hv;
      else
        s.acc[S::slot(k, a)] = s.acc[S::slot(k, a)] + hv;
    }
    S::pin(s.acc);
    return s.acc[S::slot(k, -R)];
  }
};

// Uniform disk, psf(a,b) = w for a^2 + b^2 <= R^2 (the out-of-focus blur of
// the experiments): the row filter of offset a is a plain sum over the span
// |b| <= span(a).  The spans are nested, so one running sum of the pair sums
// gives every row filter: 2R adds per input row instead of one FMA per tap,
// and the weight is applied once per output.  Taps: {w}.
template <typename T, int R, int SM = 0>
struct ConvBox {
  using S = Slide<R>;
  static constexpr int NT = 64 * kStripsPerBlock, TW = kTW, TH = strip_th(R, SM), LW = kTW + 2 * R, RC = R;
  static constexpr bool kRuntimeR = false, kStream = true;
  static constexpr bool kVSym = true;  // symmetric in the vertical direction: strips may walk up
  // streaming kernels hide memory latency with waves: ask the register
  // allocator for at least this many per SIMD where the state fits (it
  // otherwise trades occupancy for instruction-level parallelism)
  static constexpr int kWavesPerEU = stream_waves<T>(R, R + 1);
  struct St {
    T w, acc[S::NW];
  };
  __device__ static __forceinline__ void init(St& s, const T* __restrict__ taps) { s.w = taps[0]; }
  __device__ static __forceinline__ T step(St& s, const T* __restrict__ row, int k) {
    T cum[R + 1];
    cum[0] = row[0];
#pragma unroll
    for (int b = 1; b <= R; ++b) cum[b] = cum[b - 1] + (row[b] + row[-b]);
#pragma unroll
    for (int a = R; a >= -R; --a) {
      const T hv = cum[sym_span(R, true, a >= 0 ? a : -a)];
      if (a == R)
        s.acc[S::slot(k, a)] = hv;
      else
        s.acc[S::slot(k, a)] = s.acc[S::slot(k, a)] + hv;
    }
    S::pin(s.acc);
    return s.w * s.acc[S::slot(k, -R)];
  }
};

// ---------------------------------------------------------------------------
// Tile staging
// ---------------------------------------------------------------------------
struct TileGeo {
  int R, h, w, pitch, y0, x0, wave, lane;
};

// Block t of a smoother pass: the tile t (general policy, four waves share
// it), or the strips kStripsPerBlock t + wave (streaming policies, one per
// wave; a strip index past the level's last strip lies below the image, and
// stream_strip returns at once for it).
template <typename P>
__device__ __forceinline__ TileGeo tile_geo(const JobDesc& d, int t) {
  TileGeo g;
  g.R = uni(d.rad);
  g.h = uni(d.h);
  g.w = uni(d.w);
  g.pitch = uni(d.pitch);
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  const int tiles_x = uni(d.tiles_x);
  const int s = P::kStream ? t * kStripsPerBlock + g.wave : t;
  const int ty = s / tiles_x, tx = s - ty * tiles_x;
  g.y0 = ty * P::TH;
  g.x0 = tx * P::TW;
  return g;
}

// Load tile + halo (general policy): every tile element in the image gets
// combine(load(o)), elements outside the image are zero (the operator's zero
// boundary condition); o is the element's 32-bit offset in the level's
// pitched array.
// The loads of up to 16 elements per thread are issued together (from
// clamped, always valid addresses) before any is used, so a small level's
// pass waits for one round of memory latency instead of one per tile row.
template <typename T, typename P, typename LoadF, typename CombF>
__device__ __forceinline__ void load_tile(T* __restrict__ tile, const TileGeo& g, LoadF load, CombF combine) {
  const int R = g.R;
  constexpr int NWV = P::NT / 64;
  constexpr int NR = (P::LH + NWV - 1) / NWV, NC = (P::LW + 63) / 64;  // per thread, at the largest radius
  constexpr int CR = NR * NC <= 16 ? NR : (16 / NC > 0 ? 16 / NC : 1);  // rows per burst
  const int rows = P::TH + 2 * R, cols = P::TW + 2 * R;
  using V = decltype(load(0u));
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += CR) {
    V v[CR][NC];
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      const int gy = min(max(g.y0 - R + g.wave + (r0 + i) * NWV, 0), g.h - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int gx = min(max(g.x0 - R + g.lane + 64 * c, 0), g.w - 1);
        v[i][c] = load((unsigned)(gy * g.pitch + gx));
      }
    }
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      const int ly = g.wave + (r0 + i) * NWV;
      const int gy = g.y0 - R + ly;
      const bool row_in = r0 + i < NR && ly < rows && gy >= 0 && gy < g.h;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int lx = g.lane + 64 * c;
        const int gx = g.x0 - R + lx;
        if (r0 + i < NR && ly < rows && lx < cols)
          tile[ly * P::LW + lx] = (row_in && gx >= 0 && gx < g.w) ? combine(v[i][c]) : T(0);
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

// Strips of odd tile rows walk bottom-up when the policy allows it (see
// stream_strip).
template <typename P>
__device__ __forceinline__ bool strip_up(const TileGeo& g) {
  if constexpr (P::kStream && P::kVSym)
    return ((g.y0 / P::TH) & 1) != 0;
  else
    return false;
}

template <typename P>
__device__ __forceinline__ int pol_R(const TileGeo& g) {
  return P::kRuntimeR ? g.R : (P::LW - P::TW) / 2;
}

// ---------------------------------------------------------------------------
// Streaming strips (sliding-column policies).  A wave owns the 64-column x
// TH-row output strip of its tile and walks once down the input rows
// y0 - R .. y0 + TH + R - 1.  Lane l holds input column x0 - R + l and, for
// l < 2R, also x0 + 64 - R + l.  Each row's global loads are issued kPrefetch
// rows ahead into a register ring; the combined row is written to a two-row
// LDS buffer (64 + 2R columns) from which every lane reads its 2R + 1 window
// columns, so LDS holds one row per wave and occupancy is set by registers.
// Callbacks:
//   load_in(o) -> VI      raw input at offset o (clamped, always valid)
//   combine(VI) -> T      conv input value (zero outside the image is applied
//                         by the driver)
//   load_int(o) -> VN     extra data at the interior pixel of the lane
//   interior(o, v, in, n) input row inside the strip: v is the combined value
//                         at the lane's interior column (the column whose value
//                         the lane holds: x0 - R + l for l >= R, else
//                         x0 + 64 - R + l), o its offset, in = inside image
//   load_em(o) -> VE      extra data at the lane's output pixel
//   emit(o, acc, in, c, e) output row done at column x0 + l: acc = (H x), c =
//                         the combined input at that same pixel
// ---------------------------------------------------------------------------
struct NoLoad {};
struct NoLoadF {
  __device__ NoLoad operator()(unsigned) const { return NoLoad{}; }
};
struct NoInterior {
  template <typename T>
  __device__ void operator()(unsigned, T, bool, NoLoad) const {}
};

constexpr int kPrefetch = 2;

// Element offset of row y (uniform), hidden from the optimizer by an empty
// asm statement (no instruction): otherwise it folds the per-step row
// offsets of an unrolled row group into per-lane offsets that it keeps in
// vector registers across the strip loop, and the streaming kernels spill.
__device__ __forceinline__ unsigned row_offset(int y, int pitch) {
  unsigned o = (unsigned)(y * pitch);
  asm volatile("" : "+s"(o));
  return o;
}

// none: the out-of-range element offset of the level's arrays (h x pitch).
// Loads at none return 0 (combine(0) must be 0, the zero boundary), and
// interior/emit receive none as the offset of pixels outside the image, so
// their stores are dropped; `in` tells the callbacks which pixels count.
// up: walk the strip bottom-up (policies symmetric in the vertical
// direction only).  Strips of odd tile rows do, so two vertically adjacent
// strips reach the rows their halos share at the same time and the second
// read of those rows finds them in L2.
// A strip whose rows, halo included, all lie inside the image skips the
// per-row tests in the row groups between its first and its last: they are
// a few scalar compares and selects per stream and row, about a quarter of
// the instructions a wave issues per row.  Every access and result is the
// same either way.
template <bool Tests>
struct StripMode {
  static constexpr bool kRows = Tests;   // test that rows lie in the image
  static constexpr bool kSteps = Tests;  // test the step against the strip's phases
};
using StripAll = StripMode<true>;
using StripInner = StripMode<false>;
template <typename T, typename P, typename InF, typename CombF, typename IntLoadF, typename IntF, typename EmLoadF,
          typename EmF>
__device__ __forceinline__ void stream_strip(const TileGeo& g, bool up, unsigned none, typename P::St& st, InF load_in,
                                             CombF combine, IntLoadF load_int, IntF interior, EmLoadF load_em,
                                             EmF emit) {
  constexpr int R = P::RC, NW = 2 * R + 1, GS = strip_group(R), TH = P::TH, LH = TH + 2 * R, NG = LH / GS;
  constexpr int LW = kTW + 2 * R;
  static_assert(NG * GS == LH && GS % NW == 0, "strip height must fill whole row groups");
  constexpr int D = GS < kPrefetch ? GS : kPrefetch;
  constexpr int RW = 2 * kTW;  // row buffer width: every lane writes both of its values
  static_assert(LW <= RW, "row buffer too narrow");
  __shared__ T rowbufs[kStripsPerBlock][2 * RW];  // one row buffer per wave
  if (g.y0 >= g.h) return;  // a strip index past the level's last strip
  T* const rowbuf = rowbufs[g.wave];
  using VI = decltype(load_in(0u));
  using VN = decltype(load_int(0u));
  using VE = decltype(load_em(0u));
  const int lane = g.lane;
  const bool has2 = lane < 2 * R;
  const int c1 = g.x0 - R + lane, c2 = g.x0 + kTW - R + lane;
  const bool in1 = c1 >= 0 && c1 < g.w, in2 = has2 && c2 < g.w;
  const int ic = lane >= R ? c1 : c2;  // >= x0
  const bool inic = ic < g.w;
  const int ec = g.x0 + lane;
  const bool inec = ec < g.w;
  VI pa[GS], pb[GS];
  VN pn[GS];
  VE pe[GS];
  T cen[NW];
  // image row of step t, and of the output completed at step t (R steps
  // behind); rows are uniform, and a row outside the image (or past the
  // strip) maps every lane to none
  const int ybase = up ? g.y0 + TH + R - 1 : g.y0 - R, ystep = up ? -1 : 1;
  auto row_at = [&](int t) { return ybase + ystep * t; };
  auto out_at = [&](int t) { return ybase + ystep * (t - R); };
  // the tests a mode keeps (see StripMode); those it drops hold for its rows
  auto issue = [&](int t, VI& a, VI& b, VN& n, VE& e, auto mode) {
    using Md = decltype(mode);
    const int y = row_at(t);
    const bool row_ok = (!Md::kSteps || t < LH) && (!Md::kRows || (y >= 0 && y < g.h));
    const unsigned base = row_offset(y, g.pitch);
    a = load_in((row_ok && in1) ? base + (unsigned)c1 : none);
    b = load_in((row_ok && in2) ? base + (unsigned)c2 : none);
    n = load_int((row_ok && (!Md::kSteps || (t >= R && t < R + TH)) && inic) ? base + (unsigned)ic : none);
    const int yo = out_at(t);
    const unsigned obase = row_offset(yo, g.pitch);
    const bool emit_ok = (!Md::kSteps || (t >= 2 * R && t < LH)) && (!Md::kRows || yo < g.h);
    e = load_em((emit_ok && inec) ? obase + (unsigned)ec : none);
  };
  auto group = [&](int gi, auto mode) __attribute__((always_inline)) {
    using Md = decltype(mode);
#pragma unroll
    for (int kg = 0; kg < GS; ++kg) {
      const int t = gi * GS + kg, k = kg % NW;  // k = t mod NW
      const VI a = pa[kg], b = pb[kg];
      const VN n = pn[kg];
      const VE e = pe[kg];
      issue(t + D, pa[(kg + D) % GS], pb[(kg + D) % GS], pn[(kg + D) % GS], pe[(kg + D) % GS], mode);
      const int y = row_at(t);
      const T v1 = combine(a);
      const T v2 = combine(b);
      T* rb = rowbuf + (t & 1) * RW;
      rb[lane] = v1;
      rb[kTW + lane] = v2;
      // interior and emit run on every step (outside their rows with in =
      // false and offset none), so no memory operation sits in a branch
      {
        const unsigned base = row_offset(y, g.pitch);
        const bool in = (!Md::kSteps || (t >= R && t < R + TH)) && (!Md::kRows || y < g.h) && inic;
        interior(in ? base + (unsigned)ic : none, lane >= R ? v1 : v2, in, n);
      }
      wave_lds_sync();
      const T* row = rb + lane + R;
      cen[k] = row[0];
      const T out = P::step(st, row, k);
      {
        const int yo = out_at(t);
        const unsigned obase = row_offset(yo, g.pitch);
        const bool in = (!Md::kSteps || t >= 2 * R) && (!Md::kRows || yo < g.h) && inec;
        emit(in ? obase + (unsigned)ec : none, out, in, cen[((k - R) % NW + NW) % NW], e);
      }
    }
  };
  // Between the first and the last group every step lies past the strip's
  // first 2R rows (GS > 2R), and its prefetch (D <= GS - R rows ahead) stays
  // inside the interior rows, so no step test can fail there.
  static_assert(GS > 2 * R && D + R <= GS, "strip phases must fit in one row group");
  const bool inside = g.y0 - R >= 0 && g.y0 + TH + R <= g.h;
  // groups [0, lo) and [hi, NG) with the tests, [lo, hi) without
  const int lo = inside ? 1 : NG, hi = inside ? NG - 1 : NG;
#pragma unroll
  for (int t = 0; t < D; ++t) issue(t, pa[t], pb[t], pn[t], pe[t], StripAll{});
  int gi = 0;
#pragma unroll 1
  for (; gi < lo; ++gi) group(gi, StripAll{});
#pragma unroll 1
  for (; gi < hi; ++gi) group(gi, StripInner{});
#pragma unroll 1
  for (; gi < NG; ++gi) group(gi, StripAll{});
}

// ---------------------------------------------------------------------------
// Finalize: the scalar Krylov recurrences in FP64, run on the device by one
// 256-thread block per job after each pass.  Partials are summed in a fixed
// order that depends only on the job's tile count, so results are
// deterministic and independent of how many jobs share a launch.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// Fixed-order sum of selected components of the tile partials of one job,
// returned to every thread of the NT-thread block.  The order is that of 256
// threads whatever NT is (a 64-thread block plays four of them per thread),
// so a finalize gives the same bits in every kernel that runs it: virtual
// thread i adds tiles i, i + 256, i + 512, ... in that order to +0; each group
// of 64 virtual threads is reduced by wave_sum and the four group sums are
// added in order.  Eight loads per thread are in flight at a time.  (Partials
// are sums that start at +0, so none is -0 and the +0 that pads a batch adds
// nothing: the batching does not change a bit.)
template <int NV, int NT>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int ntiles, int stride,
                                             const int (&comp)[NV], double (&out)[NV]) {
  constexpr int NTO = 256, V = NTO / NT, NWO = NTO / 64, B = 8 / V;
  static_assert(NT % 64 == 0 && NTO % NT == 0 && 8 % V == 0, "block size must divide the canonical 256");
  double acc[NV][V];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double* __restrict__ c = part + (size_t)comp[i] * stride;
    double a[V];
#pragma unroll
    for (int j = 0; j < V; ++j) a[j] = 0.0;
    for (int t0 = (int)threadIdx.x; t0 < ntiles; t0 += B * NTO) {
      double v[V][B];
#pragma unroll
      for (int j = 0; j < V; ++j)
#pragma unroll
        for (int m = 0; m < B; ++m) {
          const int t = t0 + j * NT + m * NTO;
          v[j][m] = t < ntiles ? c[t] : 0.0;
        }
#pragma unroll
      for (int j = 0; j < V; ++j)
#pragma unroll
        for (int m = 0; m < B; ++m) a[j] += v[j][m];
    }
#pragma unroll
    for (int j = 0; j < V; ++j) acc[i][j] = wave_sum(a[j]);
  }
  // virtual thread threadIdx.x + j NT lies in group (threadIdx.x >> 6) + j NT / 64
  __shared__ double red[NWO][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < V; ++j) red[wave + j * (NT / 64)][i] = acc[i][j];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double v = red[0][i];
#pragma unroll
    for (int w = 1; w < NWO; ++w) v += red[w][i];
    out[i] = v;
  }
}

// Publish the job's progress (level tag, iterations, stop reason) to pinned
// host memory as one 64-bit system-scope store; the host only uses it to
// decide how many more iterations to enqueue.
__device__ __forceinline__ void publish(const JobDesc& d, const SolverState* st) {
  __hip_atomic_store(d.mirror, mirror_word(d.tag, st->k, st->done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Stopping tests of the smoother, in the order: non-finite, discrepancy
// principle ||r|| <= c delta (RMS norm), iteration cap m_l, convergence guard.
__device__ __forceinline__ int stop_reason(const JobDesc& d, int k, double rr, double guard_val, double guard_ref,
                                           bool nonfinite) {
  const double rms = sqrt(rr / ((double)d.h * (double)d.w));
  if (nonfinite) return kStopNonFinite;
  if (d.stop_rule && rms <= d.cdelta) return kStopDiscrepancy;
  if (k >= d.cap) return kStopCap;
  if (guard_val == 0.0 || guard_val <= d.eps2 * guard_ref) return kStopGuard;
  return kStopNone;
}

__device__ __forceinline__ void check_stop(SolverState* st, const JobDesc& d, double rr, double guard_val,
                                           double guard_ref, bool nonfinite) {
  const double rms = sqrt(rr / ((double)d.h * (double)d.w));
  const int reason = stop_reason(d, st->k, rr, guard_val, guard_ref, nonfinite);
  st->rr = rr;
  if (reason != kStopNone) {
    st->done = reason;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = reason;
    d.rec[d.level].rms = rms;
  }
}

// The scalar updates run in one thread with the summed partials v, on the
// job's solver state st (pub: publish the progress word to the host).
// CGLS start: partials <r,r> (1) and <s,s> (2) of r = g - H u0, s = H^T r.
constexpr int kCompCgInit[2] = {1, 2};
__device__ inline void fin_cg_init(const JobDesc& d, SolverState* st, const double (&v)[2], bool pub = true) {
  st->k = 0;
  st->par = 0;
  st->beta = 0.0;
  st->alpha = 0.0;
  for (int i = 0; i < kPRing; ++i) st->alph[i] = 0.0;
  st->na = 0;
  st->gam[1] = 0.0;
  st->done = kStopNone;
  st->pending = 0;
  st->level = d.level;
  st->gamma = v[1];
  st->gam[0] = v[1];
  st->gamma0 = v[1];
  st->rr0 = v[0];
  d.rec[d.level].iters = 0;
  d.rec[d.level].reason = kStopNone;
  d.rec[d.level].rms = sqrt(v[0] / ((double)d.h * (double)d.w));
  check_stop(st, d, v[0], v[1], v[1], !finite_d(v[0]) || !finite_d(v[1]));
  if (pub) publish(d, st);
}

// After pass A: eta = <q,q> (0), alpha = gamma / eta.
constexpr int kCompCgA[1] = {0};
__device__ inline void fin_cg_a(const JobDesc& d, SolverState* st, const double (&v)[1], bool pub = true) {
  const double eta = v[0];
  st->eta = eta;
  if (!finite_d(eta) || eta == 0.0) {
    const int reason = finite_d(eta) ? kStopGuard : kStopNonFinite;
    st->done = reason;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = reason;
    d.rec[d.level].rms = sqrt(st->rr / ((double)d.h * (double)d.w));
    if (pub) publish(d, st);
    return;
  }
  st->alpha = st->gamma / eta;
  st->alph[st->k % kPRing] = st->alpha;
  st->na = st->k + 1;
}

// After pass B: <r,r> (1), gamma_new = <s,s> (2), beta = gamma_new / gamma.
constexpr int kCompCgB[2] = {1, 2};
__device__ inline void fin_cg_b(const JobDesc& d, SolverState* st, const double (&v)[2], bool pub = true) {
  const double gnew = v[1];
  st->beta = gnew / st->gamma;
  st->gamma = gnew;
  st->k += 1;
  st->gam[st->k & 1] = gnew;
  st->par ^= 1;
  st->seq += 1;
  check_stop(st, d, v[0], gnew, st->gamma0, !finite_d(v[0]) || !finite_d(gnew));
  if (pub) publish(d, st);
}

// MR start: <r,r> (1) of r = g - H u0.
constexpr int kCompMrInit[1] = {1};
__device__ inline void fin_mr_init(const JobDesc& d, SolverState* st, const double (&v)[1], bool pub = true) {
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
  if (pub) publish(d, st);
}

// After an MR pass: <r,q> (0), <r,r> (1), <q,q> (2); the pending step of the
// pass counts as an iteration, the next step is alpha = <r,q> / <q,q>.
constexpr int kCompMr[3] = {0, 1, 2};
__device__ inline void fin_mr(const JobDesc& d, SolverState* st, const double (&v)[3], bool pub = true) {
  if (st->pending) st->k += 1;
  st->pending = 0;
  st->par ^= 1;
  st->seq += 1;
  const double rq = v[0], rr = v[1], qq = v[2];
  check_stop(st, d, rr, rr, st->rr0, !finite_d(rr) || !finite_d(rq) || !finite_d(qq));
  if (!st->done) {
    st->eta = qq;
    if (qq == 0.0) {
      st->done = kStopGuard;
      d.rec[d.level].iters = st->k;
      d.rec[d.level].reason = kStopGuard;
      d.rec[d.level].rms = sqrt(rr / ((double)d.h * (double)d.w));
    } else {
      st->rq = rq;
      st->alpha = rq / qq;
      st->pending = 1;
    }
  }
  if (pub) publish(d, st);
}

// Body of a finalize kernel: sum the partials, then the scalar update.  With
// skip_if_done the stop flag is read together with the partials (one memory
// round trip instead of two) and a level that has already stopped discards
// the sums.
template <int NV, typename F>
__device__ __forceinline__ void finalize_block(const JobDesc& d, const int (&comp)[NV], bool skip_if_done, int ntiles,
                                               F fin) {
  const int done = skip_if_done ? d.st->done : 0;
  double v[NV];
  sum_partials<NV, 256>(d.partials, ntiles, d.pstride, comp, v);
  if (threadIdx.x == 0 && !done) fin(d, v);
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
__global__ __launch_bounds__(P::NT) __attribute__((amdgpu_waves_per_eu(P::kWavesPerEU))) void k_init1(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo<P>(d, L.t);
  const auto u = gpc<T>(d.u);
  const auto gg = gpc<T>(d.g);
  auto r = gp<T>(d.r[0]);
  double part[1] = {0.0};
  if constexpr (P::kStream) {
    typename P::St st;
    P::init(st, (const T*)d.taps);
    const unsigned n = (unsigned)(g.h * g.pitch);
    const auto U = bview<T>(d.u, n), G = bview<T>(d.g, n), Rn = bview<T>(d.r[0], n);
    stream_strip<T, P>(
        g, strip_up<P>(g), n, st, [&](unsigned o) { return U.ld(o); }, [](T v) { return v; }, NoLoadF{}, NoInterior{},
        [&](unsigned o) { return G.ld(o); },
        [&](unsigned o, T acc, bool in, T, T gv) {
          const T rv = gv - acc;
          Rn.st(o, rv);
          part[0] += in ? (double)rv * (double)rv : 0.0;
        });
  } else {
    __shared__ T tile[P::LH * P::LW];
    __shared__ T gsh[P::TH * P::TW];
    load_tile<T, P>(tile, g, [&](unsigned o) { return u[o]; }, [](T v) { return v; });
    for_interior<P>(g, [&](unsigned o) { return gg[o]; },
                    [&](T v, unsigned, int row) { gsh[row * P::TW + g.lane] = v; });
    __syncthreads();
    const int gx = g.x0 + g.lane;
    constexpr int KV = P::TH / 4;  // output rows per thread: wave * KV + 0 .. KV - 1
    T rk[KV];
    P::conv(tile, (const T*)d.taps, g.R, g.wave, g.lane, [&](int v, T acc) {
      const int gy = g.y0 + v;
      const T rv = gsh[v * P::TW + g.lane] - acc;
      const bool in = gy < g.h && gx < g.w;
      if (in) {
        r[(unsigned)(gy * g.pitch + gx)] = rv;
        part[0] += (double)rv * (double)rv;
      }
      rk[v - g.wave * KV] = in ? rv : T(0);
    });
    if ((ll.flags & kLaunchInitS) && g.R == 0) {
      // one-tap blur: s = H^T r from the tile of r just formed, laid out and
      // zero outside the image as k_cg_init2 would load it, by the same
      // product in the same order (so the same bits as that kernel)
      __syncthreads();
#pragma unroll
      for (int v = 0; v < KV; ++v) tile[(g.wave * KV + v) * P::LW + g.lane] = rk[v];
      __syncthreads();
      auto s = gp<T>(d.s);
      double both[2] = {part[0], 0.0};  // partials <r,r> (slot 1) and <s,s> (slot 2)
      P::conv(tile, (const T*)d.taps_t, 0, g.wave, g.lane, [&](int v, T acc) {
        const int gy = g.y0 + v;
        if (gy < g.h && gx < g.w) {
          s[(unsigned)(gy * g.pitch + gx)] = acc;
          both[1] += (double)acc * (double)acc;
        }
      });
      block_sum_store<P::NT, 2>(both, d.partials + (size_t)1 * d.pstride + L.t, d.pstride);
      return;
    }
  }
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)1 * d.pstride + L.t, d.pstride);
}

// s = H^T r; partial <s,s> in slot 2.  The first direction p_0 = s is formed
// by the first pass A, which reads no previous direction.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) __attribute__((amdgpu_waves_per_eu(P::kWavesPerEU))) void k_cg_init2(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const TileGeo g = tile_geo<P>(d, L.t);
  const auto r = gpc<T>(d.r[0]);
  auto s = gp<T>(d.s);
  double part[1] = {0.0};
  auto put = [&](unsigned o, T acc) {
    s[o] = acc;
    part[0] += (double)acc * (double)acc;
  };
  if constexpr (P::kStream) {
    typename P::St st;
    P::init(st, (const T*)d.taps_t);
    const unsigned n = (unsigned)(g.h * g.pitch);
    const auto Rr = bview<T>(d.r[0], n), S = bview<T>(d.s, n);
    stream_strip<T, P>(
        g, strip_up<P>(g), n, st, [&](unsigned o) { return Rr.ld(o); }, [](T v) { return v; }, NoLoadF{}, NoInterior{}, NoLoadF{},
        [&](unsigned o, T acc, bool in, T, NoLoad) {
          S.st(o, acc);
          part[0] += in ? (double)acc * (double)acc : 0.0;
        });
  } else {
    __shared__ T tile[P::LH * P::LW];
    load_tile<T, P>(tile, g, [&](unsigned o) { return r[o]; }, [](T v) { return v; });
    __syncthreads();
    const int gx = g.x0 + g.lane;
    P::conv(tile, (const T*)d.taps_t, g.R, g.wave, g.lane, [&](int v, T acc) {
      const int gy = g.y0 + v;
      if (gy < g.h && gx < g.w) put((unsigned)(gy * g.pitch + gx), acc);
    });
  }
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)2 * d.pstride + L.t, d.pstride);
}

// Direction buffer slot i, the slots evenly spaced from p[0] (p[1] is slot
// 1): kPRing of them on lazy_u levels, two elsewhere.
__device__ __forceinline__ int dir_slots(const JobDesc& d) { return uni(d.lazy_u) ? kPRing : 2; }
__device__ __forceinline__ void* dir_slot(const JobDesc& d, int i) {
  return (char*)d.p[0] + (size_t)i * (size_t)((char*)d.p[1] - (char*)d.p[0]);
}

// Pass A of iteration k: p_new = s + beta p_old (on tile + halo), q = H p_new;
// partial <q,q> in slot 0.  Iteration 0 has beta = 0 and no previous
// direction: p_old reads as zero (an empty buffer range), so p_0 = s.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) __attribute__((amdgpu_waves_per_eu(P::kWavesPerEU))) void k_cg_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  // with kLaunchFoldB every block of an entry that owes a finalize (kf >= 0)
  // evaluates it from its job's partials, in the finalize kernel's order: the
  // previous pass B's, or at iteration 0 the initialisation's.  The stop
  // decision and beta are then identical everywhere; logical tile 0 records
  // them.  The iteration index comes from the launch list.
  const int kf = (uni(d.fold_a) && (ll.flags & kLaunchFoldB)) ? uni(ll.kf[L.e]) : -1;
  const bool foldb = kf >= 0;
  // iteration 0 with the initialisation's finalize starts the level here: the
  // solver state still holds the previous level's stop, so it is not consulted
  const bool finit = kf == 0;
  if (!finit && __builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int k = foldb ? kf : uni(st->k);
  T beta;
  if (finit) {
    double v[2];
    sum_partials<2, P::NT>(d.partials, uni(d.ntiles), d.pstride, kCompCgInit, v);
    const int reason = stop_reason(d, 0, v[0], v[1], v[1], !finite_d(v[0]) || !finite_d(v[1]));
    if (L.t == 0 && threadIdx.x == 0) fin_cg_init(d, d.st, v);
    if (reason != kStopNone) return;
    beta = T(0);
  } else if (foldb && k > 0) {
    double v[2];
    sum_partials<2, P::NT>(d.partials, uni(d.ntiles), d.pstride, kCompCgB, v);
    const int reason = stop_reason(d, k, v[0], v[1], st->gamma0, !finite_d(v[0]) || !finite_d(v[1]));
    if (L.t == 0 && threadIdx.x == 0) fin_cg_b(d, d.st, v);
    if (reason != kStopNone) return;
    beta = (T)(v[1] / st->gam[(k - 1) & 1]);
  } else {
    beta = (T)st->beta;
  }
  // p_{k-1} in slot k, p_k into slot k + 1 (modulo the level's slot count)
  const int ns = dir_slots(d);
  void* const pold = dir_slot(d, k % ns);
  void* const pnew = dir_slot(d, (k + 1) % ns);
  const bool first = k == 0;
  const auto s = gpc<T>(d.s);
  const auto po = gpc<T>(pold);
  auto pn = gp<T>(pnew);
  auto q = gp<T>(d.q[0]);
  double part[1] = {0.0};
  auto load = [&](unsigned o) { return Two<T>{s[o], first ? T(0) : po[o]}; };
  auto comb = [&](Two<T> x) { return fma(beta, x.b, x.a); };
  if constexpr (P::kStream) {
    typename P::St ps;
    P::init(ps, (const T*)d.taps);
    const unsigned n = (unsigned)(g.h * g.pitch);
    const auto S = bview<T>(d.s, n), Po = bview<T>(pold, first ? 0u : n), Pn = bview<T>(pnew, n);
    const auto Q = bview<T>(d.q[0], n);
    stream_strip<T, P>(
        g, strip_up<P>(g), n, ps, [&](unsigned o) { return Two<T>{S.ld(o), Po.ld(o)}; }, comb, NoLoadF{},
        [&](unsigned o, T v, bool, NoLoad) { Pn.st(o, v); }, NoLoadF{},
        [&](unsigned o, T acc, bool in, T, NoLoad) {
          Q.st(o, acc);
          part[0] += in ? (double)acc * (double)acc : 0.0;
        });
  } else {
    __shared__ T tile[P::LH * P::LW];
    load_tile<T, P>(tile, g, load, comb);
    __syncthreads();
    tile_interior<T, P>(tile, g, pol_R<P>(g), [&](T v, unsigned o, bool in) {
      if (in) pn[o] = v;
    });
    const int gx = g.x0 + g.lane;
    P::conv(tile, (const T*)d.taps, g.R, g.wave, g.lane, [&](int v, T acc) {
      const int gy = g.y0 + v;
      if (gy < g.h && gx < g.w) {
        q[(unsigned)(gy * g.pitch + gx)] = acc;
        part[0] += (double)acc * (double)acc;
      }
    });
  }
  block_sum_store<P::NT, 1>(part, d.partials + (size_t)0 * d.pstride + L.t, d.pstride);
}

// Pass B of iteration k: r_new = r - alpha q (tile + halo), s = H^T r_new,
// and the solution update; partials <r,r> (slot 1) and <s,s> (slot 2).
// The solution update u += alpha_k p_k is applied per iteration (kUOne), or,
// on levels the host marks lazy_u, deferred (kUDefer: no u or p traffic
// here): pass A keeps the directions in a ring of kPRing slots and k_flush_u
// applies up to kPRing - 1 terms at once, u = (..(u + alpha_j p_j) + ..) +
// alpha_k p_k, rounded to T after each term exactly as single updates.
enum : int { kUOne = 0, kUDefer = 1 };

template <typename T, typename P, int UM>
__device__ __forceinline__ void cg_b_body(const JobDesc& d, const TileGeo& g, int par, T alpha,
                                          double (&part)[2]) {
  const auto ro = gpc<T>(d.r[par]);
  auto rn = gp<T>(d.r[par ^ 1]);
  const auto q = gpc<T>(d.q[0]);
  const auto pn = gpc<T>(d.p[par ^ 1]);
  auto u = gp<T>(d.u);
  auto s = gp<T>(d.s);
  auto load = [&](unsigned o) { return Two<T>{ro[o], q[o]}; };
  auto comb = [&](Two<T> x) { return fma(-alpha, x.b, x.a); };
  if constexpr (P::kStream) {
    typename P::St ps;
    P::init(ps, (const T*)d.taps_t);
    const unsigned n = (unsigned)(g.h * g.pitch);
    const auto Ro = bview<T>(d.r[par], n), Rn = bview<T>(d.r[par ^ 1], n), Q = bview<T>(d.q[0], n);
    const auto Pn = bview<T>(d.p[par ^ 1], n), U = bview<T>(d.u, n);
    const auto S = bview<T>(d.s, n);
    auto emit = [&](unsigned o, T acc, bool in, T, NoLoad) {
      S.st(o, acc);
      part[1] += in ? (double)acc * (double)acc : 0.0;
    };
    auto ld_in = [&](unsigned o) { return Two<T>{Ro.ld(o), Q.ld(o)}; };
    if constexpr (UM == kUDefer) {
      stream_strip<T, P>(
          g, strip_up<P>(g), n, ps, ld_in, comb, NoLoadF{},
          [&](unsigned o, T v, bool in, NoLoad) {
            Rn.st(o, v);
            part[0] += in ? (double)v * (double)v : 0.0;
          },
          NoLoadF{}, emit);
    } else {
      stream_strip<T, P>(
          g, strip_up<P>(g), n, ps, ld_in, comb, [&](unsigned o) { return Two<T>{U.ld(o), Pn.ld(o)}; },
          [&](unsigned o, T v, bool in, Two<T> x) {
            Rn.st(o, v);
            U.st(o, fma(alpha, x.b, x.a));
            part[0] += in ? (double)v * (double)v : 0.0;
          },
          NoLoadF{}, emit);
    }
  } else {
    __shared__ T tile[P::LH * P::LW];
    load_tile<T, P>(tile, g, load, comb);
    if constexpr (UM == kUOne) {
      for_interior<P>(
          g, [&](unsigned o) { return Two<T>{u[o], pn[o]}; },
          [&](Two<T> x, unsigned o, int) { u[o] = fma(alpha, x.b, x.a); });
    }
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
  }
}

template <typename T, typename P>
__global__ __launch_bounds__(P::NT) __attribute__((amdgpu_waves_per_eu(P::kWavesPerEU))) void k_cg_b(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int par = uni(st->par);
  const int k = uni(st->k);
  T alpha;
  if (uni(d.fold_a) && (ll.flags & kLaunchFoldA)) {
    // the finalize of pass A, evaluated by every block from the same partials
    // in the same order (identical alpha everywhere); logical tile 0 records
    // it, or the stop when <q,q> is 0 or not finite
    double v[1];
    sum_partials<1, P::NT>(d.partials, d.ntiles, d.pstride, kCompCgA, v);
    const bool lead = L.t == 0 && threadIdx.x == 0;
    if (!finite_d(v[0]) || v[0] == 0.0) {
      if (lead) fin_cg_a(d, d.st, v);
      return;
    }
    if (lead) fin_cg_a(d, d.st, v);
    alpha = (T)(st->gamma / v[0]);
  } else {
    alpha = (T)st->alph[k % kPRing];
  }
  double part[2] = {0.0, 0.0};
  if (uni(d.lazy_u))
    cg_b_body<T, P, kUDefer>(d, g, par, alpha, part);
  else
    cg_b_body<T, P, kUOne>(d, g, par, alpha, part);
  block_sum_store<P::NT, 2>(part, d.partials + (size_t)1 * d.pstride + L.t, d.pstride);
}

// MR pass: if a step alpha is pending, r_new = r - alpha q and u += alpha r;
// then q_new = H r_new.  Partials <r_new,q_new> (0), <r_new,r_new> (1), <q,q> (2).
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) void k_mr_pass(LaunchList ll, const JobDesc* __restrict__ descs) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (__builtin_amdgcn_readfirstlane(st->done)) return;
  const TileGeo g = tile_geo<P>(d, L.t);
  const int par = uni(st->par);
  const bool pending = uni(st->pending) != 0;
  const T alpha = pending ? (T)st->alpha : T(0);
  const auto ro = gpc<T>(d.r[par]);
  const auto qo = gpc<T>(d.q[par]);
  auto rn = gp<T>(d.r[par ^ 1]);
  auto qn = gp<T>(d.q[par ^ 1]);
  auto u = gp<T>(d.u);
  double part[3] = {0.0, 0.0, 0.0};
  if constexpr (P::kStream) {
    typename P::St ps;
    P::init(ps, (const T*)d.taps);
    const unsigned n = (unsigned)(g.h * g.pitch);
    const auto Ro = bview<T>(d.r[par], n), Qo = bview<T>(d.q[par], n), Rn = bview<T>(d.r[par ^ 1], n);
    const auto Qn = bview<T>(d.q[par ^ 1], n), U = bview<T>(d.u, n);
    auto emit = [&](unsigned o, T acc, bool in, T rc, NoLoad) {
      Qn.st(o, acc);
      part[0] += in ? (double)rc * (double)acc : 0.0;
      part[2] += in ? (double)acc * (double)acc : 0.0;
    };
    if (pending) {
      stream_strip<T, P>(
          g, strip_up<P>(g), n, ps, [&](unsigned o) { return Two<T>{Ro.ld(o), Qo.ld(o)}; },
          [&](Two<T> x) { return fma(-alpha, x.b, x.a); }, [&](unsigned o) { return Two<T>{U.ld(o), Ro.ld(o)}; },
          [&](unsigned o, T v, bool in, Two<T> x) {
            Rn.st(o, v);
            U.st(o, fma(alpha, x.b, x.a));
            part[1] += in ? (double)v * (double)v : 0.0;
          },
          NoLoadF{}, emit);
    } else {
      stream_strip<T, P>(
          g, strip_up<P>(g), n, ps, [&](unsigned o) { return Ro.ld(o); }, [](T v) { return v; }, NoLoadF{},
          [&](unsigned o, T v, bool in, NoLoad) {
            Rn.st(o, v);
            part[1] += in ? (double)v * (double)v : 0.0;
          },
          NoLoadF{}, emit);
    }
  } else {
    __shared__ T tile[P::LH * P::LW];
    const int R = pol_R<P>(g);
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
  }
  block_sum_store<P::NT, 3>(part, d.partials + (size_t)0 * d.pstride + L.t, d.pstride);
}

// Operator form: y = H x on one dense image with the given taps layout.
template <typename T, typename P>
__global__ __launch_bounds__(P::NT) __attribute__((amdgpu_waves_per_eu(P::kWavesPerEU))) void k_op_conv(const T* __restrict__ x, T* __restrict__ y, int H, int W,
                                                   const T* __restrict__ taps, int R) {
  const int tiles_x = (W + P::TW - 1) / P::TW;
  TileGeo g;
  g.R = R;
  g.h = H;
  g.w = W;
  g.pitch = W;
  g.wave = uni(threadIdx.x >> 6);
  g.lane = threadIdx.x & 63;
  const int t = P::kStream ? (int)blockIdx.x * kStripsPerBlock + g.wave : (int)blockIdx.x;
  g.y0 = (t / tiles_x) * P::TH;
  g.x0 = (t % tiles_x) * P::TW;
  const auto xg = gpc<T>(x);
  auto yg = gp<T>(y);
  if constexpr (P::kStream) {
    typename P::St st;
    P::init(st, taps);
    const unsigned n = (unsigned)(H * W);
    const auto X = bview<T>(x, n), Y = bview<T>(y, n);
    stream_strip<T, P>(
        g, strip_up<P>(g), n, st, [&](unsigned o) { return X.ld(o); }, [](T v) { return v; }, NoLoadF{}, NoInterior{}, NoLoadF{},
        [&](unsigned o, T acc, bool, T, NoLoad) { Y.st(o, acc); });
  } else {
    __shared__ T tile[P::LH * P::LW];
    load_tile<T, P>(tile, g, [&](unsigned o) { return xg[o]; }, [](T v) { return v; });
    __syncthreads();
    const int gx = g.x0 + g.lane;
    P::conv(tile, taps, R, g.wave, g.lane, [&](int v, T acc) {
      const int gy = g.y0 + v;
      if (gy < H && gx < W) yg[(unsigned)(gy * W + gx)] = acc;
    });
  }
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
  const int tiles = ((H + P::TH - 1) / P::TH) * ((W + P::TW - 1) / P::TW);
  const int blocks = P::kStream ? (tiles + kStripsPerBlock - 1) / kStripsPerBlock : tiles;
  hipLaunchKernelGGL((k_op_conv<T, P>), dim3(blocks), dim3(P::NT), 0, s, (const T*)x, (T*)y, H, W, (const T*)taps,
                     R);
  return hipGetLastError();
}

}  // namespace eecmg
