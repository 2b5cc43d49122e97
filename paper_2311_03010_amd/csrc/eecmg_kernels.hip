// HIP kernels (gfx950, wave64) of the EECMG cascade, other than the smoother
// passes: the level-transfer operators, restriction, output copy, and the
// top-level launch dispatch.
#include <math.h>

#include <algorithm>

#include "eecmg_device.h"

namespace eecmg {

// ---------------------------------------------------------------------------
// Finalize kernels: one 256-thread block per job, scalar recurrences in FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fin_cg_init(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  finalize_block(d, kCompCgInit, false, d.ntiles,
                 [](const JobDesc& dd, const double(&v)[2]) { fin_cg_init(dd, dd.st, v); });
}

__global__ __launch_bounds__(256) void k_fin_cg_a(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  finalize_block(d, kCompCgA, true, d.ntiles, [](const JobDesc& dd, const double(&v)[1]) { fin_cg_a(dd, dd.st, v); });
}

__global__ __launch_bounds__(256) void k_fin_cg_b(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  // pass B's partials come from its own strips when it recomputes q
  finalize_block(d, kCompCgB, true, d.ntiles,
                 [](const JobDesc& dd, const double(&v)[2]) { fin_cg_b(dd, dd.st, v); });
}

__global__ __launch_bounds__(256) void k_fin_mr_init(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  finalize_block(d, kCompMrInit, false, d.ntiles,
                 [](const JobDesc& dd, const double(&v)[1]) { fin_mr_init(dd, dd.st, v); });
}

__global__ __launch_bounds__(256) void k_fin_mr(LaunchList ll, const JobDesc* __restrict__ descs) {
  const JobDesc& d = descs[ll.job[blockIdx.x]];
  finalize_block(d, kCompMr, true, d.ntiles, [](const JobDesc& dd, const double(&v)[3]) { fin_mr(dd, dd.st, v); });
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
// (exact for quadratics), 3 v1 - 3 v2 + v3 as two explicit FMAs: left to
// itself the compiler may contract either product, differently from one
// inlined call to the next, so the same node could round differently in the
// coarse cascade and in the engine's transfer kernels.
__device__ __forceinline__ double qx3(double v1, double v2, double v3) { return fma(3.0, v1, fma(-3.0, v2, v3)); }

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
__device__ __forceinline__ double pi_value(const XArgs& x, int p, int q) {
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
  return (double)uB[(size_t)p * x.p1 + q] + corr;
}

template <typename T>
__device__ __forceinline__ void pi_point(const XArgs& x, int p, int q) {
  ((T*)x.dst)[(size_t)p * x.pd + q] = to_t<T>(pi_value<T>(x, p, q));
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
// Branch-free: the three nodes base..base+2 (base = p, or p - 1 for odd p;
// inside the extended grid for every fine I) are always read and the result
// selected; an even I takes node p itself.
template <typename F>
__device__ __forceinline__ double quad1(int I, F f) {
  const int p = I >> 1;
  const bool podd = (p & 1) != 0;
  const int base = podd ? p - 1 : p;
  const double f0 = f(base), f1 = f(base + 1), f2 = f(base + 2);
  const double w0 = podd ? -0.125 : 0.375, w2 = podd ? 0.375 : -0.125;
  const double odd = fma(w2, f2, fma(0.75, f1, w0 * f0));
  return (I & 1) ? odd : (podd ? f1 : f0);
}

// Quadratic interpolation value at fine (I, J) from the extended coarse
// values E(p, q): along i first (for the needed columns q), then along j.
template <typename F>
__device__ __forceinline__ double quad_value(int I, int J, F E) {
  return quad1(J, [&](int q) { return quad1(I, [&](int p) { return E(p, q); }); });
}

template <typename T>
__device__ __forceinline__ double quad_at(const XArgs& x, int I, int J) {
  const QExt<T> E{(const T*)x.s0, x.h0, x.w0, x.p0};
  return quad_value(I, J, E);
}
template <typename T>
__device__ __forceinline__ void quad_point(const XArgs& x, int I, int J) {
  ((T*)x.dst)[(size_t)I * x.pd + J] = to_t<T>(quad_at<T>(x, I, J));
}

// Source of the linear prolongation extended by one linearly extrapolated
// virtual node per axis (along j for the real rows first, then along i).
template <typename T>
struct LExt {
  const T* u;
  int h, w, p;
  __device__ __forceinline__ double at(int i, int j) const { return (double)u[(size_t)i * p + j]; }
  __device__ __forceinline__ double rowext(int i, int j) const {
    return j < w ? at(i, j) : 2.0 * at(i, w - 1) - at(i, w - 2);
  }
  __device__ __forceinline__ double operator()(int i, int j) const {
    return i < h ? rowext(i, j) : 2.0 * rowext(h - 1, j) - rowext(h - 2, j);
  }
};

// Linear prolongation of eq. (15): nodes copy, edge midpoints average their
// ends, cell centres average along the (a,b)-(a+1,b+1) diagonal.
template <typename F>
__device__ __forceinline__ double linear_value(int I, int J, F E) {
  const int a = I >> 1, b = J >> 1;
  if (!(I & 1) && !(J & 1)) return E(a, b);
  if (!(I & 1)) return 0.5 * (E(a, b) + E(a, b + 1));
  if (!(J & 1)) return 0.5 * (E(a, b) + E(a + 1, b));
  return 0.5 * (E(a, b) + E(a + 1, b + 1));
}

template <typename T>
__device__ __forceinline__ double linear_at(const XArgs& x, int I, int J) {
  const LExt<T> E{(const T*)x.s0, x.h0, x.w0, x.p0};
  return linear_value(I, J, E);
}
template <typename T>
__device__ __forceinline__ void linear_point(const XArgs& x, int I, int J) {
  ((T*)x.dst)[(size_t)I * x.pd + J] = to_t<T>(linear_at<T>(x, I, J));
}

// Arithmetic of S and D in a compute type C: FP64 with IEEE division and
// exp(), or FP32 (the FP32 storage mode) with the hardware reciprocal,
// square root, reciprocal square root and base-2 exponential.
template <typename C>
struct Ar;
template <>
struct Ar<double> {
  __device__ static double div(double a, double b) { return a / b; }
  __device__ static double rsqrt(double x) { return 1.0 / sqrt(x); }
  __device__ static double sqrt_(double x) { return sqrt(x); }
  // eigenvalues below this fraction of the largest are rounding noise
  static constexpr double kEig = 1e-12;
};
template <>
struct Ar<float> {
  __device__ static float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  __device__ static float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  __device__ static float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static constexpr float kEig = 1e-5f;
};

// Weight w = exp(-(v/h)^2) of a neighbour at difference v, exactly 0 beyond
// (v/h)^2 > 30 or outside the image.
template <typename C>
struct SWeight;
template <>
struct SWeight<double> {
  double inv_h;
  __device__ explicit SWeight(double h) : inv_h(1.0 / h) {}
  __device__ double operator()(double v, bool in) const {
    const double z = v * inv_h;
    const double e = z * z;
    const double x = exp(-e);
    return (in && !(e > 30.0)) ? x : 0.0;
  }
};
template <>
struct SWeight<float> {
  float nl, cut;  // -log2(e) / h^2 and 30 h^2: w = 2^(v^2 nl)
  __device__ explicit SWeight(double h)
      : nl((float)(-1.4426950408889634 / (h * h))), cut((float)(30.0 * h * h)) {}
  __device__ float operator()(float v, bool in) const {
    const float d2 = v * v;
    const float x = __builtin_amdgcn_exp2f(d2 * nl);
    return (in && !(d2 > cut)) ? x : 0.0f;
  }
};

// Local smoothing S (Section 3.3, eq. 18-19): weighted LS fit of
// a0 + a1 s + a2 t on the 3x3 window with w = exp(-((u_c - u_n)/h)^2)
// (exactly 0 beyond (./h)^2 > 30, out-of-image neighbours dropped), output
// a0.  nb[3 (s+1) + (t+1)] holds the window and w the neighbours' weights
// (w[4] unused: the centre weighs 1).  The fit is centred on the pixel value
// and on the weighted centroid, which leaves a 2x2 system S a = c for the
// slopes and a0 = u_c + vb - (sb, tb) . a.  A well conditioned S
// (det > 1e-3 tr^2, so both eigenvalues exceed 1e-3 of the larger) is solved
// by its adjugate; otherwise through its eigen-decomposition (one Jacobi
// rotation, no trigonometric calls) with eigenvalues below the compute type's
// noise level (Ar<C>::kEig of the largest) dropped, so near-collinear weight
// patterns stay accurate.  The window moments are formed from row and column
// sums (the offsets are -1, 0, 1).
template <typename C>
__device__ __forceinline__ C smooth_solve(const C (&nb)[9], const C (&w)[9]) {
  // no implicit multiply-add contraction: which of two products a sum such
  // as x y + z t absorbs would otherwise depend on the code around each
  // inlined copy, and the fused transfer must round as the stage kernels do
#pragma clang fp contract(off)
  const C uc = nb[4];
  C wv[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) wv[k] = k == 4 ? C(0) : w[k] * (nb[k] - uc);
  const C rA = (w[0] + w[1]) + w[2], rB = (w[6] + w[7]) + w[8];
  const C cL = (w[0] + w[3]) + w[6], cR = (w[2] + w[5]) + w[8];
  const C m00 = ((C(1) + rA) + rB) + (w[3] + w[5]);
  const C m01 = rB - rA, m11 = rA + rB, m02 = cR - cL, m22 = cL + cR;
  const C m12 = (w[8] + w[0]) - (w[6] + w[2]);
  const C RA = (wv[0] + wv[1]) + wv[2], RB = (wv[6] + wv[7]) + wv[8];
  const C CL = (wv[0] + wv[3]) + wv[6], CR = (wv[2] + wv[5]) + wv[8];
  const C b0 = (RA + RB) + (wv[3] + wv[5]), b1 = RB - RA, b2 = CR - CL;

  const C inv0 = Ar<C>::div(C(1), m00);
  const C sb = m01 * inv0, tb = m02 * inv0, vb = b0 * inv0;
  const C S11 = fma(-m01, sb, m11), S12 = fma(-m01, tb, m12), S22 = fma(-m02, tb, m22);
  const C c1 = fma(-m01, vb, b1), c2 = fma(-m02, vb, b2);
  const C det = fma(S11, S22, -S12 * S12), tr = S11 + S22;
  C corr;
  if (det > C(1e-3) * tr * tr) {
    corr = Ar<C>::div(sb * fma(S22, c1, -S12 * c2) + tb * fma(S11, c2, -S12 * c1), det);
  } else {
    // symmetric 2x2 Schur decomposition by one Jacobi rotation (t = tan of
    // the rotation angle from tau = (S22 - S11) / (2 S12), the smaller root)
    C cs = C(1), sn = C(0), l1 = S11, l2 = S22;
    if (S12 != C(0)) {
      const C tau = Ar<C>::div(S22 - S11, C(2) * S12);
      const C t = Ar<C>::div(tau >= C(0) ? C(1) : C(-1), fabs(tau) + Ar<C>::sqrt_(C(1) + tau * tau));
      cs = Ar<C>::rsqrt(C(1) + t * t);
      sn = t * cs;
      l1 = S11 - t * S12;
      l2 = S22 + t * S12;
    }
    // eigenvectors (cs, -sn) for l1 and (sn, cs) for l2
    const C lmax = fmax(fabs(l1), fabs(l2));
    corr = C(0);
    if (l1 > Ar<C>::kEig * lmax && l1 > C(0)) corr += Ar<C>::div((sb * cs - tb * sn) * (c1 * cs - c2 * sn), l1);
    if (l2 > Ar<C>::kEig * lmax && l2 > C(0)) corr += Ar<C>::div((sb * sn + tb * cs) * (c1 * sn + c2 * cs), l2);
  }
  return uc + (vb - corr);
}

// S of the window nb: the weight of each neighbour from its difference to the
// centre (up/down/left/right tell whether rows s = -1 / +1 and columns
// t = -1 / +1 are inside the image; outside ones weigh 0).
template <typename C>
__device__ __forceinline__ C smooth_core(const C (&nb)[9], bool up, bool down, bool left, bool right,
                                         const SWeight<C>& W) {
  const C uc = nb[4];
  C w[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) {
      w[k] = C(0);
      continue;
    }
    const int si = k / 3 - 1, ti = k % 3 - 1;
    const bool in = (si < 0 ? up : (si > 0 ? down : true)) && (ti < 0 ? left : (ti > 0 ? right : true));
    w[k] = W(nb[k] - uc, in);
  }
  return smooth_solve<C>(nb, w);
}

// S at (i, j) of an H x W image read through U(ii, jj) (in-image positions
// only: outside neighbours are read at the clamped position and dropped).
template <typename C, typename F>
__device__ __forceinline__ C smooth_value(int i, int j, int H, int W, const SWeight<C>& Wt, F U) {
  const int im = max(i - 1, 0), ip = min(i + 1, H - 1), jm = max(j - 1, 0), jp = min(j + 1, W - 1);
  const C nb[9] = {U(im, jm), U(im, j), U(im, jp), U(i, jm), U(i, j), U(i, jp), U(ip, jm), U(ip, j), U(ip, jp)};
  return smooth_core<C>(nb, i > 0, i + 1 < H, j > 0, j + 1 < W, Wt);
}

// S and D compute in the storage type: FP64 in FP64 mode, FP32 in FP32 mode.
template <typename T>
__device__ __forceinline__ T smooth_at(const XArgs& x, int i, int j) {
  const T* u = (const T*)x.s0;
  const int P = x.p0;
  return smooth_value<T>(i, j, x.h0, x.w0, SWeight<T>(x.a0), [&](int ii, int jj) { return u[(size_t)ii * P + jj]; });
}
template <typename T>
__device__ __forceinline__ void smooth_point(const XArgs& x, int i, int j) {
  ((T*)x.dst)[(size_t)i * x.pd + j] = smooth_at<T>(x, i, j);
}

// One explicit Perona-Malik step (Section 4, eq. 21, 23-25):
// out = u + tau sum_{in-image nb} (c_nb + c)/2 (u_nb - u), c = 1/(1+|grad u|^2/k^2)
// with |grad u| from central differences on a replicated border.
// The diffusivity from the values below (un), above (us), right (ue) and
// left (uw) of a pixel, each already replaced by the pixel's own value where
// that neighbour lies outside the image.
template <typename C>
__device__ __forceinline__ C pm_c_of(C un, C us, C ue, C uw, C ik2) {
  const C ux = C(0.5) * (un - us);
  const C uy = C(0.5) * (ue - uw);
  return Ar<C>::div(C(1), fma(fma(ux, ux, uy * uy), ik2, C(1)));
}

template <typename C, typename F>
__device__ __forceinline__ C pm_c(int i, int j, int H, int W, C ik2, F U) {
  const int ip = i + 1 < H ? i + 1 : H - 1, im = i > 0 ? i - 1 : 0;
  const int jp = j + 1 < W ? j + 1 : W - 1, jm = j > 0 ? j - 1 : 0;
  return pm_c_of<C>(U(ip, j), U(im, j), U(i, jp), U(i, jm), ik2);
}

// The step at a pixel (value uc, diffusivity cc) from its four neighbours'
// values and diffusivities; hn/hs/he/hw tell which neighbours lie inside the
// image (the others, whatever their values, contribute nothing).
template <typename C>
__device__ __forceinline__ C pm_step_of(C uc, C cc, C cn, C cs, C ce, C cw, C un, C us, C ue, C uw, bool hn,
                                        bool hs, bool he, bool hw, C tau) {
  C acc = C(0);
  acc = hn ? fma(C(0.5) * (cn + cc), un - uc, acc) : acc;
  acc = hs ? fma(C(0.5) * (cs + cc), us - uc, acc) : acc;
  acc = he ? fma(C(0.5) * (ce + cc), ue - uc, acc) : acc;
  acc = hw ? fma(C(0.5) * (cw + cc), uw - uc, acc) : acc;
  return fma(tau, acc, uc);
}

// C(i, j) supplies the diffusivity (pm_c) at in-image pixels.
// Out-of-image neighbours contribute nothing: they are read at the clamped
// (in-image) position and dropped through a select.
template <typename C, typename F, typename G>
__device__ __forceinline__ C pm_value(int i, int j, int H, int W, C tau, F U, G Cf) {
  const C uc = U(i, j);
  const C cc = Cf(i, j);
  const int ip = min(i + 1, H - 1), im = max(i - 1, 0), jp = min(j + 1, W - 1), jm = max(j - 1, 0);
  const C cn = Cf(ip, j), cs = Cf(im, j), ce = Cf(i, jp), cw = Cf(i, jm);
  const C un = U(ip, j), us = U(im, j), ue = U(i, jp), uw = U(i, jm);
  return pm_step_of<C>(uc, cc, cn, cs, ce, cw, un, us, ue, uw, i + 1 < H, i > 0, j + 1 < W, j > 0, tau);
}

template <typename T>
__device__ __forceinline__ T pm_at(const XArgs& x, int i, int j) {
  const T* u = (const T*)x.s0;
  const int P = x.p0, H = x.h0, W = x.w0;
  const T ik2 = (T)(1.0 / (x.a0 * x.a0));
  auto U = [&](int ii, int jj) { return u[(size_t)ii * P + jj]; };
  return pm_value<T>(i, j, H, W, (T)x.a1, U, [&](int ii, int jj) { return pm_c<T>(ii, jj, H, W, ik2, U); });
}
template <typename T>
__device__ __forceinline__ void pm_point(const XArgs& x, int i, int j) {
  ((T*)x.dst)[(size_t)i * x.pd + j] = pm_at<T>(x, i, j);
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

// Grids and buffers of one transfer stage from the job's descriptor.
template <int OP>
__device__ __forceinline__ XArgs make_xargs(const JobDesc& d, int src, int dst) {
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
  return x;
}

// Pi on the engine's levels, one 2 x 2 block of grid B per thread: the four
// outputs (2a + i, 2b + j) share the corrections d(a..a+1, b..b+1), so each
// is computed once instead of up to four times; every output is the same
// expression as pi_value (bit-identical).  A block covers kPiTH x kXW nodes
// of grid A, one per thread: a single chain of loads per thread keeps the
// kernel short on the small levels, where its latency is all it costs.
template <typename T>
__device__ __forceinline__ void pi_tile2(const XArgs& x, int t) {
  const int HA = (x.hd + 1) / 2, WA = (x.wd + 1) / 2;
  const int tiles_x = (WA + kXW - 1) / kXW;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int b = tx * kXW + (threadIdx.x & 63);
  const int a = ty * kPiTH + (threadIdx.x >> 6);
  if (b >= WA || a >= HA) return;
  const T* uA = (const T*)x.s0;
  const T* uB = (const T*)x.s1;
  T* out = (T*)x.dst;
  const PiD<T> D{uA, uB, x.h0, x.w0, x.p0, x.p1};
  const int q = 2 * b;
  const bool q1 = q + 1 < x.wd;
  {
    const int p = 2 * a;
    const bool p1 = p + 1 < x.hd;
    // d beyond the virtual nodes is never needed: those outputs do not exist
    const double d00 = D(a, b), d01 = q1 ? D(a, b + 1) : 0.0;
    const double d10 = p1 ? D(a + 1, b) : 0.0, d11 = (p1 && q1) ? D(a + 1, b + 1) : 0.0;
    const T* ub = uB + (size_t)p * x.p1 + q;
    T* o = out + (size_t)p * x.pd + q;
    o[0] = to_t<T>((double)ub[0] + d00 * 0.25);
    if (q1) o[1] = to_t<T>((double)ub[1] + (d00 + d01) * 0.125);
    if (p1) {
      o[x.pd] = to_t<T>((double)ub[x.p1] + (d00 + d10) * 0.125);
      if (q1) o[x.pd + 1] = to_t<T>((double)ub[x.p1 + 1] + (d00 + d10 + d01 + d11) * 0.0625);
    }
  }
}

__global__ __launch_bounds__(256) void k_pi2_f32(LaunchList ll, const JobDesc* __restrict__ descs, int dst) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  pi_tile2<float>(make_xargs<kXfExtrap>(descs[L.d], -1, dst), L.t);
}
__global__ __launch_bounds__(256) void k_pi2_f64(LaunchList ll, const JobDesc* __restrict__ descs, int dst) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  pi_tile2<double>(make_xargs<kXfExtrap>(descs[L.d], -1, dst), L.t);
}

// Engine form: the job's descriptor supplies the grids and buffers.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_xfer(LaunchList ll, const JobDesc* __restrict__ descs, int src, int dst) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  xfer_tile<T, OP>(make_xargs<OP>(descs[L.d], src, dst), L.t);
}

// Operator form on one dense image.
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_xfer_op(XArgs x) {
  xfer_tile<T, OP>(x, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Fused prolongation -> S -> D of one level transfer (Sections 3.2-4)
// ---------------------------------------------------------------------------
// One TY x kFX tile of the destination level per 256-thread block (TY = 32,
// or 8 on small levels, where fewer and shorter per-thread chains matter more
// than the halo overhead).  The
// prolongation (quadratic P, or the linear one of IECMG-L) is evaluated on the
// tile plus the halo that S and D need, S on the tile plus D's halo and D's
// diffusivities on the tile plus one pixel; every intermediate stays in LDS.
// Each value comes from the same point functions as the separate stage
// kernels and is rounded to T between stages exactly where they store it, so
// the fused pipeline reproduces the stages run one after another.  The
// quadratic P is evaluated separably (along i into an FP64 LDS panel, then
// along j), which is the evaluation order quad_value defines.
constexpr int kFX = 64, kFY = 32, kFYSmall = 8;
// rows per tile of the FP32 fused transfer on large levels
constexpr int kFY32 = 32;

struct FArgs {
  const void* src;  // level l-1 input of the prolongation (grid B)
  int hB, wB, pB;
  void* dst;        // level l output
  int h, w, pitch;
  double smooth_h, pm_k, tau;
};

template <bool QUAD, bool DO_D, int TY>
struct FusedGeo {
  static constexpr int HS = DO_D ? 2 : 0;  // S halo
  static constexpr int HP = HS + 1;        // P halo
  static constexpr int PH = TY + 2 * HP, PW = kFX + 2 * HP;
  static constexpr int SH = TY + 2 * HS, SW = kFX + 2 * HS;
  static constexpr int CH = TY + 2, CW = kFX + 2;
  static constexpr int BH = PH / 2 + 5, BW = PW / 2 + 5;  // coarse panel bound
  static constexpr int NQ = QUAD ? BH * BW + PH * BW : 0;
  static constexpr int NC = DO_D ? CH * CW : 0;
  static constexpr int XN = (NQ > NC ? NQ : NC) > 0 ? (NQ > NC ? NQ : NC) : 1;
};

template <typename T, bool QUAD, bool DO_D, int TY>
__device__ __forceinline__ void fused_tile(const FArgs& a, int t) {
  using G = FusedGeo<QUAD, DO_D, TY>;
  __shared__ double xs[G::XN];  // coarse panels (P), then diffusivities (D)
  __shared__ T pt[G::PH * G::PW];
  __shared__ T stl[DO_D ? G::SH * G::SW : 1];
  const int h = a.h, w = a.w;
  const int tiles_x = (w + kFX - 1) / kFX;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int I0 = ty * TY, J0 = tx * kFX;
  const int pi0 = I0 - G::HP, pj0 = J0 - G::HP;  // origin of the P tile
  const int Ia = max(pi0, 0), Ib = min(pi0 + G::PH, h) - 1;
  const int Ja = max(pj0, 0), Jb = min(pj0 + G::PW, w) - 1;
  const T* src = (const T*)a.src;

  if constexpr (QUAD) {
    const QExt<T> E{src, a.hB, a.wB, a.pB};
    const int pa = max((Ia >> 1) - 1, 0), pb = min((Ib >> 1) + 2, a.hB + 1);
    const int qa = max((Ja >> 1) - 1, 0), qb = min((Jb >> 1) + 2, a.wB + 1);
    double* bt = xs;                  // E(p, q)
    double* rt = xs + G::BH * G::BW;  // R(I, q) = quad1 along i
    for (int k = threadIdx.x; k < G::BH * G::BW; k += 256) {
      const int r = k / G::BW, c = k - r * G::BW;
      if (pa + r <= pb && qa + c <= qb) bt[k] = E(pa + r, qa + c);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < G::PH * G::BW; k += 256) {
      const int r = k / G::BW, c = k - r * G::BW;
      const int I = pi0 + r;
      if (I >= Ia && I <= Ib && qa + c <= qb)
        rt[k] = quad1(I, [&](int p) { return bt[(p - pa) * G::BW + c]; });
    }
    __syncthreads();
    for (int k = threadIdx.x; k < G::PH * G::PW; k += 256) {
      const int r = k / G::PW, c = k - r * G::PW;
      const int I = pi0 + r, J = pj0 + c;
      T v = T(0);  // outside the image: a finite filler S never weighs
      if (I >= Ia && I <= Ib && J >= Ja && J <= Jb)
        v = to_t<T>(quad1(J, [&](int q) { return rt[r * G::BW + (q - qa)]; }));
      pt[k] = v;
    }
  } else {
    const LExt<T> E{src, a.hB, a.wB, a.pB};
    for (int k = threadIdx.x; k < G::PH * G::PW; k += 256) {
      const int r = k / G::PW, c = k - r * G::PW;
      const int I = pi0 + r, J = pj0 + c;
      pt[k] = (I >= Ia && I <= Ib && J >= Ja && J <= Jb) ? to_t<T>(linear_value(I, J, E)) : T(0);
    }
  }
  __syncthreads();

  const SWeight<T> Wt(a.smooth_h);
  // S at (I, J) from the P tile: the whole window lies inside the tile
  // (out-of-image entries hold the filler), so no clamping is needed.
  auto S_at = [&](int I, int J) {
    const T* c = pt + (I - pi0) * G::PW + (J - pj0);
    const T nb[9] = {c[-G::PW - 1], c[-G::PW], c[-G::PW + 1], c[-1],          c[0],
                     c[1],          c[G::PW - 1], c[G::PW],   c[G::PW + 1]};
    return smooth_core<T>(nb, I > 0, I + 1 < h, J > 0, J + 1 < w, Wt);
  };
  T* out = (T*)a.dst;
  if constexpr (!DO_D) {
    for (int k = threadIdx.x; k < TY * kFX; k += 256) {
      const int I = I0 + k / kFX, J = J0 + k % kFX;
      if (I < h && J < w) out[(size_t)I * a.pitch + J] = S_at(I, J);
    }
  } else {
    const int si0 = I0 - G::HS, sj0 = J0 - G::HS;
    for (int k = threadIdx.x; k < G::SH * G::SW; k += 256) {
      const int r = k / G::SW, c = k - r * G::SW;
      const int I = si0 + r, J = sj0 + c;
      if (I >= 0 && I < h && J >= 0 && J < w) stl[k] = S_at(I, J);
    }
    __syncthreads();
    const T ik2 = (T)(1.0 / (a.pm_k * a.pm_k));
    auto Us = [&](int ii, int jj) { return stl[(ii - si0) * G::SW + (jj - sj0)]; };
    T* ct = reinterpret_cast<T*>(xs);  // the P panels are no longer needed
    for (int k = threadIdx.x; k < G::CH * G::CW; k += 256) {
      const int r = k / G::CW, c = k - r * G::CW;
      const int I = I0 - 1 + r, J = J0 - 1 + c;
      if (I >= 0 && I < h && J >= 0 && J < w) ct[k] = pm_c<T>(I, J, h, w, ik2, Us);
    }
    __syncthreads();
    auto Cc = [&](int ii, int jj) { return ct[(ii - (I0 - 1)) * G::CW + (jj - (J0 - 1))]; };
    for (int k = threadIdx.x; k < TY * kFX; k += 256) {
      const int I = I0 + k / kFX, J = J0 + k % kFX;
      if (I < h && J < w) out[(size_t)I * a.pitch + J] = pm_value<T>(I, J, h, w, (T)a.tau, Us, Cc);
    }
  }
}

// FP32 form of the fused transfer with fewer instructions per pixel.  A
// tile is 64 columns of the prolongation wide (one lane per column) and
// TY + 2 HP rows tall; it writes OW = 64 - 2 HP columns of TY output rows.
// After P (as above: FP64 coarse panels, one LDS row per tile row), each wave
// walks a quarter of the S rows down its 64 columns keeping three rows of
// values in registers; an edge's weight exp(-(difference/h)^2) is the same
// seen from both of its pixels (the difference only changes sign), so every
// weight is evaluated once: a pixel computes its east, south, south-east and
// south-west edges, takes its west and north-west ones from the lane to its
// left, its north-east one from the lane to its right (cross-lane shuffles)
// and its north ones from the previous row.  D walks the output rows the same
// way, its diffusivities computed once per pixel and shared with the
// neighbours through registers and shuffles.  The weights, the fit and D are
// the same expressions in the same order as the separate stage kernels, so
// the output is bit for bit theirs.
template <bool QUAD, bool DO_D, int TY>
struct SGeo {
  static constexpr int HS = DO_D ? 2 : 0;  // S halo
  static constexpr int HP = HS + 1;        // P halo
  static constexpr int OW = kTW - 2 * HP;  // output columns per tile
  static constexpr int PH = TY + 2 * HP;   // tile rows (P rows; S runs on rows 1 .. PH - 2)
  static constexpr int LW = kTW + 2;       // LDS row: columns -1 .. 64
  static constexpr int BH = PH / 2 + 5, BW = kTW / 2 + 5;  // coarse panel bound
  static constexpr int NQ = QUAD ? BH * BW + PH * BW : 0;  // doubles
  static constexpr int NS = DO_D ? (PH * LW + 1) / 2 : 0;  // smoothed rows (floats, in doubles)
  static constexpr int XN = (NQ > NS ? NQ : NS) > 0 ? (NQ > NS ? NQ : NS) : 1;
};

__host__ __device__ constexpr int sgeo_ow(bool do_d) { return kTW - 2 * ((do_d ? 2 : 0) + 1); }

template <bool QUAD, bool DO_D, int TY>
__device__ __forceinline__ void fused_tile_f32(const FArgs& a, int t) {
  using G = SGeo<QUAD, DO_D, TY>;
  constexpr int LW = G::LW;
  __shared__ double xs[G::XN];  // coarse panels (P), then the smoothed rows (S -> D)
  __shared__ float pt[G::PH * LW];
  float* const stl = reinterpret_cast<float*>(xs);  // the panels are dead once P is done
  const int h = a.h, w = a.w;
  const int tiles_x = (w + G::OW - 1) / G::OW;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int I0 = ty * TY, J0 = tx * G::OW;
  const int pi0 = I0 - G::HP, pj0 = J0 - G::HP;  // image position of tile row 0, column 0
  const int Ia = max(pi0, 0), Ib = min(pi0 + G::PH, h) - 1;
  const int Ja = max(pj0, 0), Jb = min(pj0 + kTW, w) - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* src = (const float*)a.src;
  const int J = pj0 + lane;  // this lane's column
  const bool jin = J >= Ja && J <= Jb;

  if constexpr (QUAD) {
    const QExt<float> E{src, a.hB, a.wB, a.pB};
    const int pa = max((Ia >> 1) - 1, 0), pb = min((Ib >> 1) + 2, a.hB + 1);
    const int qa = max((Ja >> 1) - 1, 0), qb = min((Jb >> 1) + 2, a.wB + 1);
    double* bt = xs;                  // E(p, q)
    double* rt = xs + G::BH * G::BW;  // R(I, q) = quad1 along i
    if (pb < a.hB && qb < a.wB) {
      // no virtual node: plain loads, one panel row per wave and step
      for (int r = wave; r <= pb - pa; r += 4)
        if (lane <= qb - qa) bt[r * G::BW + lane] = (double)src[(size_t)(pa + r) * a.pB + qa + lane];
    } else {
      for (int k = threadIdx.x; k < G::BH * G::BW; k += 256) {
        const int r = k / G::BW, c = k - r * G::BW;
        if (pa + r <= pb && qa + c <= qb) bt[k] = E(pa + r, qa + c);
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < G::PH * G::BW; k += 256) {
      const int r = k / G::BW, c = k - r * G::BW;
      const int I = pi0 + r;
      if (I >= Ia && I <= Ib && qa + c <= qb) rt[k] = quad1(I, [&](int p) { return bt[(p - pa) * G::BW + c]; });
    }
    __syncthreads();
    for (int r = wave; r < G::PH; r += 4) {
      const int I = pi0 + r;
      float v = 0.0f;  // outside the image: a finite filler S never weighs
      if (I >= Ia && I <= Ib && jin) v = to_t<float>(quad1(J, [&](int q) { return rt[r * G::BW + (q - qa)]; }));
      pt[r * LW + lane + 1] = v;
      if (lane < 2) pt[r * LW + lane * (LW - 1)] = 0.0f;  // the columns -1 and 64
    }
  } else {
    const LExt<float> E{src, a.hB, a.wB, a.pB};
    for (int r = wave; r < G::PH; r += 4) {
      const int I = pi0 + r;
      pt[r * LW + lane + 1] = (I >= Ia && I <= Ib && jin) ? to_t<float>(linear_value(I, J, E)) : 0.0f;
      if (lane < 2) pt[r * LW + lane * (LW - 1)] = 0.0f;
    }
  }
  __syncthreads();

  // S on tile rows 1 .. PH - 2, a contiguous quarter of them per wave
  {
    const SWeight<float> W(a.smooth_h);
    constexpr int NSR = G::PH - 2, CH = NSR / 4;
    static_assert(NSR % 4 == 0, "every wave smooths the same number of rows");
    const int rs0 = 1 + wave * CH;
    const bool c0 = J - 1 >= 0 && J - 1 < w, c1 = J >= 0 && J < w, c2 = J + 1 >= 0 && J + 1 < w;
    auto rin = [&](int r) { const int I = pi0 + r; return I >= 0 && I < h; };
    float* out = (float*)a.dst;
    {
      const float* pr = pt + (rs0 - 1) * LW + lane;  // pr[0..2]: columns lane - 1 .. lane + 1
      float z0 = pr[0], z1 = pr[1], z2 = pr[2];
      float y0 = pr[LW], y1 = pr[LW + 1], y2 = pr[LW + 2];
      bool rz = rin(rs0 - 1), ry = rin(rs0);
      // the edges from row rs0 - 1 down to row rs0
      float pS = W(y1 - z1, rz && ry && c1);
      float pSE = W(y2 - z1, rz && ry && c1 && c2);
      float pSW = W(y0 - z1, rz && ry && c1 && c0);
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int r = rs0 + k;
        const float* xr = pt + (r + 1) * LW + lane;
        const float x0 = xr[0], x1 = xr[1], x2 = xr[2];
        const bool rx = rin(r + 1);
        const float wE = W(y2 - y1, ry && c1 && c2);
        const float wS = W(x1 - y1, ry && rx && c1);
        const float wSE = W(x2 - y1, ry && rx && c1 && c2);
        const float wSW = W(x0 - y1, ry && rx && c1 && c0);
        const float wW = __shfl_up(wE, 1, 64);
        const float wNW = __shfl_up(pSE, 1, 64);
        const float wNE = __shfl_down(pSW, 1, 64);
        const float nb[9] = {z0, z1, z2, y0, y1, y2, x0, x1, x2};
        const float wt[9] = {wNW, pS, wNE, wW, 0.0f, wE, wSW, wS, wSE};
        const float v = smooth_solve<float>(nb, wt);
        if constexpr (DO_D) {
          stl[r * LW + lane + 1] = v;
        } else {
          const int I = pi0 + r;
          if (lane >= G::HP && lane < kTW - G::HP && ry && c1) out[(size_t)I * a.pitch + J] = v;
        }
        z0 = y0; z1 = y1; z2 = y2;
        y0 = x0; y1 = x1; y2 = x2;
        rz = ry; ry = rx;
        pS = wS; pSE = wSE; pSW = wSW;
      }
    }
  }
  if constexpr (DO_D) {
    // D on the output rows, a contiguous quarter of them per wave, walking
    // down its columns with three rows of smoothed values and of
    // diffusivities in registers (left and right neighbours from the adjacent
    // lanes); out-of-image neighbours are replaced or dropped exactly as the
    // separate step kernel's clamped reads do, so the output is bit for bit its.
    __syncthreads();
    const float ik2 = (float)(1.0 / (a.pm_k * a.pm_k));
    const float tau = (float)a.tau;
    constexpr int DCH = TY / 4;  // output rows per wave
    static_assert(TY % 4 == 0, "every wave steps the same number of rows");
    const int r0 = G::HP + wave * DCH;
    const bool he = J + 1 < w, hw = J > 0;
    const bool ol = lane >= G::HP && lane < kTW - G::HP && J < w;
    float* out = (float*)a.dst;
    auto urow = [&](int r) { return stl[r * LW + lane + 1]; };
    // diffusivity of tile row r from its values (u, ue, uw) and the rows above (um) and below (up)
    auto cof = [&](int r, float um, float u, float up, float ue, float uw) {
      const int I = pi0 + r;
      return pm_c_of<float>(I + 1 < h ? up : u, I > 0 ? um : u, he ? ue : u, hw ? uw : u, ik2);
    };
    float u0 = urow(r0 - 1), u1 = urow(r0), u2 = urow(r0 + 1);
    float c0, c1;
    {
      const float um = urow(r0 - 2);
      c0 = cof(r0 - 1, um, u0, u1, __shfl_down(u0, 1, 64), __shfl_up(u0, 1, 64));
    }
    float ue1 = __shfl_down(u1, 1, 64), uw1 = __shfl_up(u1, 1, 64);
    c1 = cof(r0, u0, u1, u2, ue1, uw1);
#pragma unroll
    for (int k = 0; k < DCH; ++k) {
      const int r = r0 + k, I = pi0 + r;
      const float u3 = urow(r + 2);
      const float ue2 = __shfl_down(u2, 1, 64), uw2 = __shfl_up(u2, 1, 64);
      const float c2 = cof(r + 1, u1, u2, u3, ue2, uw2);
      const float ce = __shfl_down(c1, 1, 64), cw = __shfl_up(c1, 1, 64);
      const float v = pm_step_of<float>(u1, c1, c2, c0, ce, cw, u2, u0, ue1, uw1, I + 1 < h, I > 0, he, hw, tau);
      if (ol && I < h) out[(size_t)I * a.pitch + J] = v;
      u0 = u1; u1 = u2; u2 = u3;
      ue1 = ue2; uw1 = uw2;
      c0 = c1; c1 = c2;
    }
  }
}

// Engine form: grids and buffers from the job's descriptor.
template <typename T, bool QUAD, bool DO_D, int TY>
__global__ __launch_bounds__(256) void k_xfer_fused(LaunchList ll, const JobDesc* __restrict__ descs, int src,
                                                    int dst) {
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  FArgs a;
  a.src = xbuf(d, src);
  a.hB = d.hB;
  a.wB = d.wB;
  a.pB = d.pB;
  a.dst = xbuf(d, dst);
  a.h = d.h;
  a.w = d.w;
  a.pitch = d.pitch;
  a.smooth_h = d.smooth_h;
  a.pm_k = d.pm_k;
  a.tau = d.tau;
  if constexpr (sizeof(T) == 4)
    fused_tile_f32<QUAD, DO_D, TY>(a, L.t);
  else
    fused_tile<T, QUAD, DO_D, TY>(a, L.t);
}

// Operator form on one dense image.
template <typename T, bool QUAD, bool DO_D>
__global__ __launch_bounds__(256) void k_xfer_fused_op(FArgs a) {
  if constexpr (sizeof(T) == 4)
    fused_tile_f32<QUAD, DO_D, kFY>(a, blockIdx.x);
  else
    fused_tile<T, QUAD, DO_D, kFY>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Coarse cascade: the leading small levels of one job solved by a single
// 1024-thread block -- each level's transfer (the stages above, one after
// another), the smoother's initialisation and every iteration with its
// stopping test -- so they cost one launch instead of a dozen per level, and
// the coarse levels of a batch of images run side by side.  The scalar
// recurrences are the finalize functions of the multi-block passes, run by
// thread 0 on block-reduced partials (fixed order: deterministic) and on a
// solver state kept in LDS; the host does not follow these levels, so no
// progress word is published.
// ---------------------------------------------------------------------------
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseWaves = kCoarseThreads / 64;

// Sum NV per-thread values over the block; every thread gets the sums.
template <int NV>
__device__ __forceinline__ void coarse_reduce(double (&v)[NV]) {
  __shared__ double red[kCoarseWaves][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double a = red[0][i];
#pragma unroll
    for (int w = 1; w < kCoarseWaves; ++w) a += red[w][i];
    v[i] = a;
  }
  __syncthreads();
}

// Every sweep hands each thread kCoarseU pixels at a time (k, k + 1024, ...)
// and issues all of their loads before using any, so one block keeps enough
// memory requests in flight on the small levels.
constexpr int kCoarseU = 4;

struct Px {
  int i, j;
  bool ok;   // inside the level (k < h w)
  size_t o;  // pitched offset (of pixel 0 when !ok)
};

__device__ __forceinline__ Px px_at(int k, int n, int w, int P) {
  Px p;
  p.ok = k < n;
  const int kk = p.ok ? k : 0;
  p.i = kk / w;
  p.j = kk - p.i * w;
  p.o = (size_t)p.i * P + p.j;
  return p;
}

template <int U = kCoarseU, typename F>
__device__ __forceinline__ void coarse_sweep(int n, int w, int P, F body) {
  for (int k0 = threadIdx.x; k0 < n; k0 += U * kCoarseThreads) {
    Px px[U];
#pragma unroll
    for (int m = 0; m < U; ++m) px[m] = px_at(k0 + m * kCoarseThreads, n, w, P);
    body(px);
  }
}

// (H x)(i, j) = sum_{a,b} psf(a,b) x(i-a, j-b), zero outside the image, from
// the full (2R+1)^2 taps (H^T: the flipped taps), for kCoarseU pixels: each
// tap's loads (from clamped, always valid positions) are issued together.
template <typename T>
__device__ __forceinline__ void coarse_conv(const T* __restrict__ x, int pitch, int h, int w,
                                            const T* __restrict__ taps, int R, const Px (&px)[kCoarseU],
                                            T (&acc)[kCoarseU]) {
  const int n = 2 * R + 1;
#pragma unroll
  for (int m = 0; m < kCoarseU; ++m) acc[m] = T(0);
  for (int a = -R; a <= R; ++a) {
    for (int b = -R; b <= R; ++b) {
      const T wt = taps[(a + R) * n + (b + R)];
      T v[kCoarseU];
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) {
        const int y = px[m].i - a, xx = px[m].j - b;
        const bool in = y >= 0 && y < h && xx >= 0 && xx < w;
        const T t = x[(size_t)min(max(y, 0), h - 1) * pitch + min(max(xx, 0), w - 1)];
        v[m] = in ? t : T(0);
      }
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) acc[m] = fma(wt, v[m], acc[m]);
    }
  }
}

// One transfer stage over its destination grid, then a block barrier.  The
// point operators keep a few dozen values live each, so the stages take two
// pixels at a time (S, the largest, one).
template <typename T, int OP>
__device__ __forceinline__ void coarse_stage(const JobDesc& d, int src, int dst) {
  constexpr int U = OP == kXfSmooth ? 1 : 2;
  const XArgs x = make_xargs<OP>(d, src, dst);
  coarse_sweep<U>(x.hd * x.wd, x.wd, x.pd, [&](const Px (&px)[U]) {
    double v[U];
#pragma unroll
    for (int m = 0; m < U; ++m) {
      if (OP == kXfExtrap)
        v[m] = pi_value<T>(x, px[m].i, px[m].j);
      else if (OP == kXfQuad)
        v[m] = quad_at<T>(x, px[m].i, px[m].j);
      else if (OP == kXfLinear)
        v[m] = linear_at<T>(x, px[m].i, px[m].j);
      else if (OP == kXfSmooth)
        v[m] = smooth_at<T>(x, px[m].i, px[m].j);
      else
        v[m] = pm_at<T>(x, px[m].i, px[m].j);
    }
#pragma unroll
    for (int m = 0; m < U; ++m)
      if (px[m].ok) ((T*)x.dst)[px[m].o] = to_t<T>(v[m]);
  });
  __syncthreads();
}

// Transfer into the level (the stage sequence of the multi-level engine).
template <typename T>
__device__ void coarse_transfer(const JobDesc& d) {
  const int l = d.level, n = d.pm_steps;
  int src;
  if (d.cascade == kCascadeEecmg) {
    if (l < 2) return;  // the two coarsest levels start from zero
    coarse_stage<T, kXfExtrap>(d, -1, kBufT2);
    src = kBufT2;
  } else {
    if (l < 1) return;
    src = kBufUB;
  }
  if (d.cascade == kCascadeIecmgL)
    coarse_stage<T, kXfLinear>(d, src, kBufT1);
  else
    coarse_stage<T, kXfQuad>(d, src, kBufT1);
  coarse_stage<T, kXfSmooth>(d, kBufT1, n == 0 ? kBufU : kBufT2);
  for (int s = 0; s < n; ++s) {
    const int a = (s % 2 == 0) ? kBufT2 : kBufT1;
    const int b = (s == n - 1) ? kBufU : ((s % 2 == 0) ? kBufT1 : kBufT2);
    coarse_stage<T, kXfPm>(d, a, b);
  }
}

// CGLS on one level: the arithmetic of the multi-block passes (init, pass A
// with p = s + beta p and q = H p, pass B with r -= alpha q, u += alpha p and
// s = H^T r), with a block barrier between dependent sweeps.
template <typename T>
__device__ void coarse_cgls(const JobDesc& d) {
  const int h = d.h, w = d.w, P = d.pitch, R = d.rad, n = h * w;
  const T* __restrict__ g = (const T*)d.g;
  T* __restrict__ u = (T*)d.u;
  T* __restrict__ r = (T*)d.r[0];
  T* __restrict__ p = (T*)d.p[0];
  T* __restrict__ s = (T*)d.s;
  T* __restrict__ q = (T*)d.q[0];
  const T* __restrict__ tp = (const T*)d.taps;
  const T* __restrict__ tt = (const T*)d.taps_t;
  __shared__ SolverState state;  // the level's scalars stay on chip
  SolverState* st = &state;
  __shared__ double sc[2];
  __shared__ int done;
  // a one-tap blur (R = 0, the coarse levels of most PSFs) is pointwise:
  // sweeps that only chain blurs then run as one, with the same expressions
  // (the tap product as fma(w, x, 0), as the tap loop forms it), so the
  // results are the same bits
  const bool pw = R == 0;
  const T w0 = tp[0], wt0 = tt[0];
  double v[2] = {0.0, 0.0};
  if (pw) {
    coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
      T gv[kCoarseU], uv[kCoarseU];
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) {
        gv[m] = g[px[m].o];
        uv[m] = u[px[m].o];
      }
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m)
        if (px[m].ok) {
          const T rv = gv[m] - fma(w0, uv[m], T(0));
          const T sv = fma(wt0, rv, T(0));
          r[px[m].o] = rv;
          s[px[m].o] = sv;
          p[px[m].o] = sv;
          v[0] += (double)rv * (double)rv;
          v[1] += (double)sv * (double)sv;
        }
    });
  } else {
    coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
      T hv[kCoarseU], gv[kCoarseU];
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) gv[m] = g[px[m].o];
      coarse_conv(u, P, h, w, tp, R, px, hv);
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m)
        if (px[m].ok) {
          const T rv = gv[m] - hv[m];
          r[px[m].o] = rv;
          v[0] += (double)rv * (double)rv;
        }
    });
    __syncthreads();
    coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
      T sv[kCoarseU];
      coarse_conv(r, P, h, w, tt, R, px, sv);
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m)
        if (px[m].ok) {
          s[px[m].o] = sv[m];
          p[px[m].o] = sv[m];
          v[1] += (double)sv[m] * (double)sv[m];
        }
    });
  }
  coarse_reduce(v);
  if (threadIdx.x == 0) {
    fin_cg_init(d, st, v, false);
    done = st->done;
  }
  __syncthreads();
  bool first = true;
  while (!done) {
    if (!first && !pw) {
      const T beta = (T)sc[1];
      coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
        T a[kCoarseU], b[kCoarseU];
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m) {
          a[m] = p[px[m].o];
          b[m] = s[px[m].o];
        }
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m)
          if (px[m].ok) p[px[m].o] = fma(beta, a[m], b[m]);
      });
      __syncthreads();
    }
    double e[1] = {0.0};
    if (pw) {
      const bool upd = !first;
      const T beta = upd ? (T)sc[1] : T(0);
      coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
        T a[kCoarseU], b[kCoarseU];
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m) {
          a[m] = p[px[m].o];
          b[m] = s[px[m].o];
        }
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m)
          if (px[m].ok) {
            const T pv = upd ? fma(beta, a[m], b[m]) : a[m];
            const T qv = fma(w0, pv, T(0));
            if (upd) p[px[m].o] = pv;
            q[px[m].o] = qv;
            e[0] += (double)qv * (double)qv;
          }
      });
    } else {
      coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
        T qv[kCoarseU];
        coarse_conv(p, P, h, w, tp, R, px, qv);
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m)
          if (px[m].ok) {
            q[px[m].o] = qv[m];
            e[0] += (double)qv[m] * (double)qv[m];
          }
      });
    }
    first = false;
    coarse_reduce(e);
    if (threadIdx.x == 0) {
      fin_cg_a(d, st, e, false);
      done = st->done;
      sc[0] = st->alpha;
    }
    __syncthreads();
    if (done) break;
    const T alpha = (T)sc[0];
    double b[2] = {0.0, 0.0};
    coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
      T qv[kCoarseU], rv[kCoarseU], pv[kCoarseU], uv[kCoarseU];
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) {
        qv[m] = q[px[m].o];
        rv[m] = r[px[m].o];
        pv[m] = p[px[m].o];
        uv[m] = u[px[m].o];
      }
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m)
        if (px[m].ok) {
          const T rn = fma(-alpha, qv[m], rv[m]);
          r[px[m].o] = rn;
          u[px[m].o] = fma(alpha, pv[m], uv[m]);
          b[0] += (double)rn * (double)rn;
          if (pw) {
            const T sv = fma(wt0, rn, T(0));
            s[px[m].o] = sv;
            b[1] += (double)sv * (double)sv;
          }
        }
    });
    if (!pw) {
      __syncthreads();
      coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
        T sv[kCoarseU];
        coarse_conv(r, P, h, w, tt, R, px, sv);
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m)
          if (px[m].ok) {
            s[px[m].o] = sv[m];
            b[1] += (double)sv[m] * (double)sv[m];
          }
      });
    }
    coarse_reduce(b);
    if (threadIdx.x == 0) {
      fin_cg_b(d, st, b, false);
      done = st->done;
      sc[1] = st->beta;
    }
    __syncthreads();
  }
}

// MR on one level (the arithmetic of the multi-block MR pass).
template <typename T>
__device__ void coarse_mr(const JobDesc& d) {
  const int h = d.h, w = d.w, P = d.pitch, R = d.rad, n = h * w;
  const T* __restrict__ g = (const T*)d.g;
  T* __restrict__ u = (T*)d.u;
  T* __restrict__ r = (T*)d.r[0];
  T* __restrict__ q = (T*)d.q[0];
  const T* __restrict__ tp = (const T*)d.taps;
  __shared__ SolverState state;  // the level's scalars stay on chip
  SolverState* st = &state;
  __shared__ double sc[1];
  __shared__ int done, pending;
  double v[1] = {0.0};
  coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
    T hv[kCoarseU], gv[kCoarseU];
#pragma unroll
    for (int m = 0; m < kCoarseU; ++m) gv[m] = g[px[m].o];
    coarse_conv(u, P, h, w, tp, R, px, hv);
#pragma unroll
    for (int m = 0; m < kCoarseU; ++m)
      if (px[m].ok) {
        const T rv = gv[m] - hv[m];
        r[px[m].o] = rv;
        v[0] += (double)rv * (double)rv;
      }
  });
  coarse_reduce(v);
  if (threadIdx.x == 0) {
    fin_mr_init(d, st, v, false);
    done = st->done;
    pending = 0;
  }
  __syncthreads();
  while (!done) {
    if (pending) {
      const T alpha = (T)sc[0];
      coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
        T rv[kCoarseU], qv[kCoarseU], uv[kCoarseU];
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m) {
          rv[m] = r[px[m].o];
          qv[m] = q[px[m].o];
          uv[m] = u[px[m].o];
        }
#pragma unroll
        for (int m = 0; m < kCoarseU; ++m)
          if (px[m].ok) {
            u[px[m].o] = fma(alpha, rv[m], uv[m]);
            r[px[m].o] = fma(-alpha, qv[m], rv[m]);
          }
      });
      __syncthreads();
    }
    double mm[3] = {0.0, 0.0, 0.0};
    coarse_sweep(n, w, P, [&](const Px (&px)[kCoarseU]) {
      T qv[kCoarseU], rc[kCoarseU];
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m) rc[m] = r[px[m].o];
      coarse_conv(r, P, h, w, tp, R, px, qv);
#pragma unroll
      for (int m = 0; m < kCoarseU; ++m)
        if (px[m].ok) {
          q[px[m].o] = qv[m];
          mm[0] += (double)rc[m] * (double)qv[m];
          mm[1] += (double)rc[m] * (double)rc[m];
          mm[2] += (double)qv[m] * (double)qv[m];
        }
    });
    coarse_reduce(mm);
    if (threadIdx.x == 0) {
      fin_mr(d, st, mm, false);
      done = st->done;
      pending = st->pending;
      sc[0] = st->alpha;
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// Restriction (eq. 12-13), with the coarse levels solved in the same launch
// ---------------------------------------------------------------------------
// Every level's right-hand side g_l(i, j) = g(2^(L-l) i, 2^(L-l) j) and the
// starting solution of every level that receives no transfer (zero, or the
// given initial guess on the finest level); the other levels are written whole
// by their transfer before their smoother reads them.  One launch does this
// for a group of jobs, in blocks of kCoarseThreads threads: the head block of
// a job with coarse levels restricts those levels itself (a few thousand
// pixels) and then solves them (the coarse cascade above), while tiles
// restrict the remaining levels in one pass over the dense input, so that
// pass runs beside the one-block cascade instead of before it.
// Rows of the dense input the restriction visits: every row when the finest
// level gets a pitched copy or a starting value, else only the even rows,
// which are all that feed the coarser levels.
constexpr int kRH = 16;  // visited rows per wave of a restriction tile
__host__ __device__ inline int restrict_row_step(const JobDesc& d) {
  const bool copy_fine = d.g_lv[d.L - 1] != d.g_in;
  const bool init_fine = (d.zero_u >> (d.L - 1)) & 1;
  return (copy_fine || init_fine) ? 1 : 2;
}

// Restriction tiles of a job (64 input columns x kRH * kCoarseWaves visited
// rows each) for its levels C .. L - 1.  The launch has one head block per job
// first (the coarse cascade, or nothing), then every job's tiles.
__host__ __device__ inline int restrict_tiles(const JobDesc& d) {
  const int C = d.coarse_levels, rs = restrict_row_step(d);
  if (C >= d.L || (rs == 2 && d.L == 1)) return 0;
  const int th = kRH * kCoarseWaves;
  return ((d.H + rs - 1) / rs + th - 1) / th * ((d.W + kXW - 1) / kXW);
}

// The levels 0 .. C-1 of a job, by its head block (the finest level among
// them only when every level is coarse), in one sweep over level C-1 that
// also writes the coarser levels' pixels: kCoarseU pixels per thread at a
// time, their loads first.  (Not inlined, like restrict_tile: the coarse
// cascade after it already needs nearly every register a 1024-thread block
// may have.)
template <typename T>
__device__ __noinline__ void restrict_coarse(const JobDesc& d, int C) {
  const int W = d.W, NL = d.L, top = C - 1, sh = NL - 1 - top, zero = d.zero_u;
  const bool fine = top == NL - 1;
  const bool copy = !fine || d.g_lv[top] != d.g_in;
  const bool ztop = (zero >> top) & 1;
  const T* gin = (const T*)d.g_in;
  const T* uin = (const T*)d.u_in;
  T* const gt = (T*)d.g_lv[top];
  T* const ut = (T*)d.u_lv[top];
  coarse_sweep(d.lh[top] * d.lw[top], d.lw[top], fine ? d.fine_pitch : d.lp[top], [&](const Px (&px)[kCoarseU]) {
    T gv[kCoarseU], uv[kCoarseU];
#pragma unroll
    for (int m = 0; m < kCoarseU; ++m) {
      const size_t fo = (size_t)(px[m].i << sh) * W + (px[m].j << sh);
      gv[m] = gin[fo];
      uv[m] = (ztop && fine && uin) ? uin[fo] : T(0);
    }
#pragma unroll
    for (int m = 0; m < kCoarseU; ++m) {
      if (!px[m].ok) continue;
      if (copy) gt[px[m].o] = gv[m];
      if (ztop) ut[px[m].o] = uv[m];
      for (int l = top - 1; l >= 0; --l) {
        const int s = top - l, msk = (1 << s) - 1;
        if ((px[m].i & msk) || (px[m].j & msk)) break;
        const size_t o = (size_t)(px[m].i >> s) * d.lp[l] + (px[m].j >> s);
        ((T*)d.g_lv[l])[o] = gv[m];
        if ((zero >> l) & 1) ((T*)d.u_lv[l])[o] = T(0);
      }
    }
  });
  __syncthreads();
}

// Restriction tile t of the levels C .. L-1: each lane one input column, each
// wave kRH visited rows, all loaded before any store.
template <typename T>
__device__ __noinline__ void restrict_tile(const JobDesc& d, int t, int C) {
  const int H = d.H, W = d.W, NL = d.L;
  const int rs = restrict_row_step(d);
  const int tiles_x = (W + kXW - 1) / kXW;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int x = tx * kXW + (threadIdx.x & 63);
  if (x >= W) return;
  const T* gin = (const T*)d.g_in;
  const T* uin = (const T*)d.u_in;
  const int zero = d.zero_u;
  // the finest level reads the dense input in place when its rows already
  // have the level's pitch; otherwise it gets a pitched copy
  const bool copy_fine = d.g_lv[NL - 1] != d.g_in;
  const bool init_fine = (zero >> (NL - 1)) & 1;
  // tile row r covers input row r * rs
  T vals[kRH];
  int ys[kRH];
#pragma unroll
  for (int k = 0; k < kRH; ++k) {
    const int y = (ty * (kRH * kCoarseWaves) + (threadIdx.x >> 6) * kRH + k) * rs;
    ys[k] = y;
    vals[k] = gin[(size_t)min(y, H - 1) * W + x];
  }
  for (int k = 0; k < kRH; ++k) {
    const int y = ys[k];
    if (y >= H) break;
    const size_t fo = (size_t)y * W + x;
    const T v = vals[k];
    const size_t of = (size_t)y * d.fine_pitch + x;
    if (copy_fine) ((T*)d.g_lv[NL - 1])[of] = v;
    if (init_fine) ((T*)d.u_lv[NL - 1])[of] = uin ? uin[fo] : T(0);
    for (int l = NL - 2; l >= C; --l) {
      const int sh = NL - 1 - l, m = (1 << sh) - 1;
      if ((y & m) || (x & m)) break;
      const size_t o = (size_t)(y >> sh) * d.lp[l] + (x >> sh);
      ((T*)d.g_lv[l])[o] = v;
      if ((zero >> l) & 1) ((T*)d.u_lv[l])[o] = T(0);
    }
  }
}

// descs[ll.job[e]] is level 0 of job e.  Blocks 0 .. ll.n - 1 are the jobs'
// head blocks, so every coarse cascade starts at once; the tiles follow, as
// ll.start counts them.
template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_restrict(LaunchList ll, const JobDesc* __restrict__ descs) {
  if ((int)blockIdx.x >= ll.n) {
    const Loc L = locate(ll, blockIdx.x - ll.n);
    const JobDesc& d = descs[L.d];
    restrict_tile<T>(d, L.t, d.coarse_levels);
    return;
  }
  const int d0 = ll.job[blockIdx.x];
  const int C = descs[d0].coarse_levels;
  if (C == 0) return;
  restrict_coarse<T>(descs[d0], C);
  for (int l = 0; l < C; ++l) {
    const JobDesc& dl = descs[d0 + l];
    coarse_transfer<T>(dl);
    if (dl.smoother == kSmootherMr)
      coarse_mr<T>(dl);
    else
      coarse_cgls<T>(dl);
    __syncthreads();
  }
}

constexpr int kFlushChunkBytes = 16;  // k_flush_u: bytes of a row per thread

// The deferred solution updates of a lazy_u level (see k_cg_b): terms are
// applied in groups of G = kPRing - 1 consecutive iterations, in order,
// u = (..(u + alpha_j p_j) + ..) + alpha_k p_k, rounded to T after each term
// exactly as single updates.  ll.kf[e] >= 0: the launch follows pass B of
// iteration j = ll.kf[e] (the last of its group; the host issues it before
// the next pass A could overwrite the group's oldest slot) and applies that
// group if the level got that far; -1: the level has ended and the last,
// incomplete group is applied.  Which terms exist follows from st->na alone
// (the iterations whose pass B ran), so every block agrees.
template <typename T>
__global__ __launch_bounds__(256) void k_flush_u(LaunchList ll, const JobDesc* __restrict__ descs) {
  constexpr int G = kPRing - 1;
  constexpr int E = kFlushChunkBytes / sizeof(T);  // elements per 16-byte chunk
  typedef T V __attribute__((ext_vector_type(E)));
  const Loc L = locate(ll, remap_xcd(blockIdx.x, gridDim.x));
  const JobDesc& d = descs[L.d];
  const SolverState* st = d.st;
  if (!__builtin_amdgcn_readfirstlane(d.lazy_u)) return;
  const int na = __builtin_amdgcn_readfirstlane(st->na);
  const int j = ll.kf[L.e];
  int t0, t1;
  if (j >= 0) {
    if (na < j + 1) return;  // the level stopped before this pass B
    t0 = j + 1 - G;
    t1 = j + 1;
  } else {
    t0 = na - na % G;
    t1 = na;
  }
  if (t0 >= t1) return;
  // one 16-byte chunk of a row per thread (rows start 256-byte aligned)
  const int cw = (d.w + E - 1) / E;
  const int i = L.t * 256 + (int)threadIdx.x;
  if (i >= d.h * cw) return;
  const int y = i / cw, x = (i - y * cw) * E;
  const size_t o = (size_t)y * d.pitch + x;
  const int nt = t1 - t0;
  T a[G];
  const T* p[G];
#pragma unroll
  for (int m = 0; m < G; ++m) {
    const int t = m < nt ? t0 + m : t0;  // (unused terms re-read the first one)
    a[m] = (T)st->alph[t % kPRing];
    p[m] = (const T*)((const char*)d.p[0] + (size_t)((t + 1) % kPRing) * (size_t)((char*)d.p[1] - (char*)d.p[0]));
  }
  T* u = (T*)d.u;
  if (x + E <= d.w) {
    V v[G];
#pragma unroll
    for (int m = 0; m < G; ++m) v[m] = *(const V*)(p[m] + o);
    V acc = *(const V*)(u + o);
#pragma unroll
    for (int m = 0; m < G; ++m)
      if (m < nt) {
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = fma(a[m], v[m][e], acc[e]);
      }
    *(V*)(u + o) = acc;
  } else {
    for (int e = 0; x + e < d.w; ++e) {
      T acc = u[o + e];
      for (int m = 0; m < nt; ++m) acc = fma(a[m], p[m][o + e], acc);
      u[o + e] = acc;
    }
  }
}

// Descriptors and PSF taps of newly admitted jobs, one block per job, read
// straight from pinned host memory: a step that admits many jobs costs one
// launch instead of two copies per job.
__global__ __launch_bounds__(256) void k_upload(UploadList ul, const JobDesc* __restrict__ hdesc,
                                                JobDesc* __restrict__ ddesc, const char* __restrict__ htaps,
                                                size_t taps_stride) {
  const int s = ul.slot[blockIdx.x];
  const JobDesc* src = hdesc + (size_t)s * kMaxLevels;
  const int L = src->L;
  const int tb = src->taps_bytes;
  uint32_t* tdst = (uint32_t*)const_cast<void*>(src->taps);
  // every load of a round is issued before any store (host memory is far)
  auto copy = [](uint32_t* __restrict__ dst, const uint32_t* __restrict__ from, int n) {
    constexpr int B = 8;
    for (int base = threadIdx.x; base < n; base += B * 256) {
      uint32_t v[B];
#pragma unroll
      for (int m = 0; m < B; ++m) v[m] = base + m * 256 < n ? from[base + m * 256] : 0u;
#pragma unroll
      for (int m = 0; m < B; ++m)
        if (base + m * 256 < n) dst[base + m * 256] = v[m];
    }
  };
  copy((uint32_t*)(ddesc + (size_t)s * kMaxLevels), (const uint32_t*)src, L * (int)(sizeof(JobDesc) / 4));
  copy(tdst, (const uint32_t*)(htaps + (size_t)s * taps_stride), tb / 4);
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_zero_words(void* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_upload(const UploadList& ul, const JobDesc* hdesc, JobDesc* ddesc, const char* htaps,
                         size_t taps_stride, hipStream_t s) {
  if (ul.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upload, dim3(ul.n), dim3(256), 0, s, ul, hdesc, ddesc, htaps, taps_stride);
  return hipGetLastError();
}

// Output copy: the finest level's (pitched) solution into the dense output.
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
hipError_t sm_f32_sep(Stage st, int R, int sm, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_f32_sym(Stage st, bool disk, int R, int sm, const LaunchList& ll, const JobDesc* descs,
                      hipStream_t s);
hipError_t sm_f64_sep(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_f64_sym(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_gen(Stage st, bool f64, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t sm_gen_short(Stage st, bool f64, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t opc_f32_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f32_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f64_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_f64_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t opc_gen(bool f64, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);
hipError_t sm_box(Stage st, bool f64, int R, int sm, const LaunchList& ll, const JobDesc* descs, hipStream_t s);
hipError_t opc_box(bool f64, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s);

int rmax_class_for(int r) { return r <= 3 ? 3 : (r <= 6 ? 6 : 12); }

static int tiles2(int h, int w, int th, int tw) { return ((h + th - 1) / th) * ((w + tw - 1) / tw); }

int blocks_for_stage(Stage st, const JobDesc& d) {
  switch (st) {
    case kRestrict: return restrict_tiles(d);
    case kOutCopy: return tiles2(d.H, d.W, kXH, kXW);
    case kCgInit1:
    case kCgInit2:
    case kCgA:
    case kMrInit:
    case kMrPass: return d.ntiles;
    case kCgB: return d.ntiles;
    case kCgFinInit:
    case kCgFinA:
    case kCgFinB:
    case kMrFinInit:
    case kMrFin: return 1;
    case kXfExtrap: return tiles2((d.hB + 1) / 2, (d.wB + 1) / 2, kPiTH, kXW);  // 2 x 2 outputs per thread
    case kXfFused: return d.f64 ? tiles2(d.h, d.w, kFY, kFX) : tiles2(d.h, d.w, kFY32, sgeo_ow(d.pm_steps >= 1));
    case kXfFusedSmall: return tiles2(d.h, d.w, kFYSmall, d.f64 ? kFX : sgeo_ow(d.pm_steps >= 1));
    case kFlushU: {  // one 16-byte chunk per thread
      const long chunks = (long)d.h * ((d.w + kFlushChunkBytes / (d.f64 ? 8 : 4) - 1) / (kFlushChunkBytes / (d.f64 ? 8 : 4)));
      return (int)((chunks + 255) / 256);
    }
    default: return tiles2(d.h, d.w, kXH, kXW);
  }
}

static hipError_t launch_smoother(Stage st, bool f64, int variant, const LaunchList& ll, const JobDesc* descs,
                                  hipStream_t s) {
  const int kind = variant_kind(variant), R = variant_r(variant);
  const int tall = variant_strip_mode(variant);  // strip mode: 0 usual, 1 tall, 2 short
  if (tall && (f64 || kind == kConvGeneral || kind == kConvGenShort)) return hipErrorInvalidValue;
  switch (kind) {
    case kConvGeneral: return sm_gen(st, f64, R, ll, descs, s);
    case kConvGenShort: return sm_gen_short(st, f64, R, ll, descs, s);
    case kConvSep: return f64 ? sm_f64_sep(st, R, ll, descs, s) : sm_f32_sep(st, R, tall, ll, descs, s);
    case kConvSymSquare:
      return f64 ? sm_f64_sym(st, false, R, ll, descs, s) : sm_f32_sym(st, false, R, tall, ll, descs, s);
    case kConvSymDisk:
      return f64 ? sm_f64_sym(st, true, R, ll, descs, s) : sm_f32_sym(st, true, R, tall, ll, descs, s);
    case kConvBoxDisk: return sm_box(st, f64, R, tall, ll, descs, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int TY>
static hipError_t launch_fused(int variant, dim3 grid, const LaunchList& ll, const JobDesc* descs, int src, int dst,
                               hipStream_t s) {
  const dim3 block(256);
  switch (variant & 3) {
    case 0: hipLaunchKernelGGL((k_xfer_fused<T, false, false, TY>), grid, block, 0, s, ll, descs, src, dst); break;
    case 1: hipLaunchKernelGGL((k_xfer_fused<T, true, false, TY>), grid, block, 0, s, ll, descs, src, dst); break;
    case 2: hipLaunchKernelGGL((k_xfer_fused<T, false, true, TY>), grid, block, 0, s, ll, descs, src, dst); break;
    default: hipLaunchKernelGGL((k_xfer_fused<T, true, true, TY>), grid, block, 0, s, ll, descs, src, dst); break;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_typed(Stage st, int variant, const LaunchList& ll, const JobDesc* descs, int src, int dst,
                               hipStream_t s) {
  const dim3 grid(ll.total), block(256);
  switch (st) {
    case kRestrict:  // the head blocks, then the tiles
      hipLaunchKernelGGL(k_restrict<T>, dim3(ll.n + ll.total), dim3(kCoarseThreads), 0, s, ll, descs);
      return hipGetLastError();
    case kOutCopy: hipLaunchKernelGGL(k_out_copy<T>, grid, block, 0, s, ll, descs); return hipGetLastError();
    case kFlushU: hipLaunchKernelGGL(k_flush_u<T>, grid, block, 0, s, ll, descs); return hipGetLastError();
    case kXfExtrap:
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL(k_pi2_f32, grid, block, 0, s, ll, descs, dst);
      else
        hipLaunchKernelGGL(k_pi2_f64, grid, block, 0, s, ll, descs, dst);
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
    case kXfFused: return launch_fused<T, sizeof(T) == 8 ? kFY : kFY32>(variant, grid, ll, descs, src, dst, s);
    case kXfFusedSmall: return launch_fused<T, kFYSmall>(variant, grid, ll, descs, src, dst, s);
    default: break;
  }
  return launch_smoother(st, sizeof(T) == 8, variant, ll, descs, s);
}

hipError_t launch_stage(Stage st, bool f64, int variant, const LaunchList& ll, const JobDesc* descs, int src,
                        int dst, hipStream_t s) {
  if (ll.n <= 0) return hipSuccess;
  const dim3 block(256);
  switch (st) {
    case kCgFinInit: hipLaunchKernelGGL(k_fin_cg_init, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kCgFinA: hipLaunchKernelGGL(k_fin_cg_a, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kCgFinB: hipLaunchKernelGGL(k_fin_cg_b, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kMrFinInit: hipLaunchKernelGGL(k_fin_mr_init, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
    case kMrFin: hipLaunchKernelGGL(k_fin_mr, dim3(ll.n), block, 0, s, ll, descs); return hipGetLastError();
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
    case kConvBoxDisk: return opc_box(f64, x, y, H, W, taps, R, s);
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

template <typename T>
static void launch_fused_op(const FArgs& a, bool quad, bool denoise, hipStream_t s) {
  const dim3 grid(tiles2(a.h, a.w, kFY, sizeof(T) == 8 ? kFX : sgeo_ow(denoise))), block(256);
  if (quad && denoise)
    hipLaunchKernelGGL((k_xfer_fused_op<T, true, true>), grid, block, 0, s, a);
  else if (quad)
    hipLaunchKernelGGL((k_xfer_fused_op<T, true, false>), grid, block, 0, s, a);
  else if (denoise)
    hipLaunchKernelGGL((k_xfer_fused_op<T, false, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_xfer_fused_op<T, false, false>), grid, block, 0, s, a);
}

hipError_t op_fused_transfer(const void* uB, int HC, int WC, void* uC, bool quad, double smooth_h, bool denoise,
                             double k, double tau, bool f64, hipStream_t s) {
  FArgs a{};
  a.src = uB;
  a.hB = (HC + 1) / 2;
  a.wB = (WC + 1) / 2;
  a.pB = a.wB;
  a.dst = uC;
  a.h = HC;
  a.w = WC;
  a.pitch = WC;
  a.smooth_h = smooth_h;
  a.pm_k = k;
  a.tau = tau;
  if (f64)
    launch_fused_op<double>(a, quad, denoise, s);
  else
    launch_fused_op<float>(a, quad, denoise, s);
  return hipGetLastError();
}

}  // namespace eecmg
