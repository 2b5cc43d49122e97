// HIP kernels (gfx950, wave64) of the EECMG cascade, other than the smoother
// passes: the finalize kernels that run the scalar Krylov recurrences on the
// device, the level-transfer operators, restriction, output copy, and the
// top-level launch dispatch.
//
// Finalize kernels sum the per-tile FP64 partials of one job in a fixed
// order, so every result is deterministic and independent of how many jobs
// share a launch.
#include <math.h>

#include "eecmg_device.h"

namespace eecmg {

// ---------------------------------------------------------------------------
// Finalize kernels: one block per job, scalar recurrences in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// Fixed-order sum of selected components of the tile partials of one job,
// returned to every thread of the 256-thread block.  Thread i sums the
// contiguous chunk [i*ch, (i+1)*ch) of each component in index order, then the
// 256 chunk sums are combined by a fixed tree: the result depends only on the
// job's own partials.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int ntiles, int stride,
                                             const int (&comp)[NV], double (&out)[NV]) {
  __shared__ double red[4][NV];
  const int ch = (ntiles + 255) / 256;
  const int t0 = min((int)threadIdx.x * ch, ntiles), t1 = min(t0 + ch, ntiles);
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double* __restrict__ c = part + (size_t)comp[i] * stride;
    double a = 0.0;
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
      const double v0 = c[t], v1 = c[t + 1], v2 = c[t + 2], v3 = c[t + 3];
      a = (((a + v0) + v1) + v2) + v3;
    }
    for (; t < t1; ++t) a += c[t];
    acc[i] = a;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = wave_sum(acc[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = acc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// Publish the job's progress (level tag, iterations, stop reason) to pinned
// host memory as one 64-bit system-scope store; the host only uses it to
// decide how many more iterations to enqueue.
__device__ __forceinline__ void publish(const JobDesc& d, const SolverState* st) {
  __hip_atomic_store(d.mirror, mirror_word(d.tag, st->k, st->done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

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
  sum_partials<2>(d.partials, d.ntiles, d.pstride, comp, v);
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
  publish(d, st);
}

__global__ __launch_bounds__(256) void k_cg_fin_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  SolverState* st = d.st;
  if (st->done) return;
  double v[1];
  const int comp[1] = {0};
  sum_partials<1>(d.partials, d.ntiles, d.pstride, comp, v);
  if (threadIdx.x != 0) return;
  const double eta = v[0];
  st->eta = eta;
  if (!finite_d(eta) || eta == 0.0) {
    const int reason = finite_d(eta) ? kStopGuard : kStopNonFinite;
    st->done = reason;
    d.rec[d.level].iters = st->k;
    d.rec[d.level].reason = reason;
    d.rec[d.level].rms = sqrt(st->rr / ((double)d.h * (double)d.w));
    publish(d, st);
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
  sum_partials<2>(d.partials, d.ntiles, d.pstride, comp, v);
  if (threadIdx.x != 0) return;
  const double gnew = v[1];
  st->beta = gnew / st->gamma;
  st->gamma = gnew;
  st->k += 1;
  st->par ^= 1;
  st->seq += 1;
  check_stop(st, d, v[0], gnew, st->gamma0, !finite_d(v[0]) || !finite_d(gnew));
  publish(d, st);
}

__global__ __launch_bounds__(256) void k_mr_fin_init(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  double v[1];
  const int comp[1] = {1};
  sum_partials<1>(d.partials, d.ntiles, d.pstride, comp, v);
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
  publish(d, st);
}

__global__ __launch_bounds__(256) void k_mr_fin(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  SolverState* st = d.st;
  if (st->done) return;
  double v[3];
  const int comp[3] = {0, 1, 2};
  sum_partials<3>(d.partials, d.ntiles, d.pstride, comp, v);
  if (threadIdx.x != 0) return;
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
  publish(d, st);
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
// and the 2x2 system for (a1, a2) is solved through its eigen-decomposition
// (one Jacobi rotation, no trigonometric calls), dropping eigenvalues below
// 1e-12 of the largest; the fitted centre value stays accurate for
// near-collinear weight patterns.
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
  // symmetric 2x2 Schur decomposition by one Jacobi rotation (t = tan of the
  // rotation angle from tau = (S22 - S11) / (2 S12), the smaller root)
  double cs = 1.0, sn = 0.0, l1 = S11, l2 = S22;
  if (S12 != 0.0) {
    const double tau = (S22 - S11) / (2.0 * S12);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    cs = 1.0 / sqrt(1.0 + t * t);
    sn = t * cs;
    l1 = S11 - t * S12;
    l2 = S22 + t * S12;
  }
  // eigenvectors (cs, -sn) for l1 and (sn, cs) for l2
  const double lmax = fmax(fabs(l1), fabs(l2));
  double corr = 0.0;
  if (l1 > 1e-12 * lmax && l1 > 0.0) corr += (sb * cs - tb * sn) * (c1 * cs - c2 * sn) / l1;
  if (l2 > 1e-12 * lmax && l2 > 0.0) corr += (sb * sn + tb * cs) * (c1 * sn + c2 * cs) / l2;
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
hipError_t sm_f32_sep(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_f32_sym(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_f64_sep(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_f64_sym(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_gen(Stage st, bool f64, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t opc_f32_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f32_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f64_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f64_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_gen(bool f64, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);

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

static hipError_t launch_smoother(Stage st, bool f64, int variant, const LaunchList& ll, const JobDesc* descs,
                                  hipStream_t s) {
  const int kind = variant / 100, R = variant % 100;
  switch (kind) {
    case kConvGeneral: return sm_gen(st, f64, R, ll, descs, s);
    case kConvSep: return f64 ? sm_f64_sep(st, R, ll, descs, s) : sm_f32_sep(st, R, ll, descs, s);
    case kConvSymSquare:
      return f64 ? sm_f64_sym(st, false, R, ll, descs, s) : sm_f32_sym(st, false, R, ll, descs, s);
    case kConvSymDisk: return f64 ? sm_f64_sym(st, true, R, ll, descs, s) : sm_f32_sym(st, true, R, ll, descs, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_typed(Stage st, int variant, const LaunchList& ll, const JobDesc* descs, int src, int dst,
                               hipStream_t s) {
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
  return launch_smoother(st, sizeof(T) == 8, variant, ll, descs, s);
}

hipError_t launch_stage(Stage st, bool f64, int variant, const LaunchList& ll, const JobDesc* descs, int src,
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
  return f64 ? launch_typed<double>(st, variant, ll, descs, src, dst, s)
             : launch_typed<float>(st, variant, ll, descs, src, dst, s);
}

hipError_t op_conv(const void* x, void* y, int H, int W, const void* taps, int variant, int radius, bool f64,
                   hipStream_t s) {
  const int kind = variant / 100, R = variant % 100;
  switch (kind) {
    case kConvGeneral: return opc_gen(f64, x, y, H, W, taps, radius, s);  // template class from the radius
    case kConvSep: return f64 ? opc_f64_sep(x, y, H, W, taps, R, s) : opc_f32_sep(x, y, H, W, taps, R, s);
    case kConvSymSquare:
      return f64 ? opc_f64_sym(false, x, y, H, W, taps, R, s) : opc_f32_sym(false, x, y, H, W, taps, R, s);
    case kConvSymDisk:
      return f64 ? opc_f64_sym(true, x, y, H, W, taps, R, s) : opc_f32_sym(true, x, y, H, W, taps, R, s);
    default: return hipErrorInvalidValue;
  }
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
