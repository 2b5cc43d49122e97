/*
 * EECMG oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, FP64 CPU implementation of the extrapolation economy cascadic
 * multigrid (EECMG) image restoration method of Chu, Yan and Li (arXiv
 * 2311.03010), written from the paper with no blocking, fusion or reordering.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the HIP
 * path, and the HIP path never calls it.
 *
 * Conventions
 *   - Images are dense row-major H x W arrays of doubles, index (i, j) =
 *     row i, column j, 0-based.  Level 1 is the coarsest, level L the finest.
 *   - A PSF of radius r is a (2r+1) x (2r+1) row-major array;
 *     psf[(a+r)*(2r+1) + (b+r)] is the weight at offset (a, b).
 *   - Inner products use Neumaier-compensated serial summation, so results do
 *     not depend on the OpenMP thread count (OpenMP only splits the pixel
 *     loops of the stencils; each output pixel is computed by one thread in a
 *     fixed order).
 *
 * Readings of points the paper leaves open are marked "reading:"; each one is
 * listed with its justification in the design notes of the repository.
 *
 * Parity status: every exported function is pinned by a CPU test against an
 * independent statement (dense matrices, closed forms, invariants, library
 * least squares), except the complete cascade's PSNR, which the paper reports
 * only for a test image that is not available: "parity unpinned" for the
 * paper's PSNR tables.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* stop reasons of the smoother */
#define OR_STOP_NONE 0
#define OR_STOP_DISCREPANCY 1 /* ||g - H u|| <= c delta  (Section 2, stopping rule) */
#define OR_STOP_CAP 2         /* m_l iterations done (Section 2, iteration-count rule) */
#define OR_STOP_GUARD 3       /* converged to rounding: gradient norm vanished */

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated summation                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s, c;
} or_nsum;

static void ns_add(or_nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

/* <x, y> over n entries, compensated. */
double or_dot(const double* x, const double* y, long n) {
  or_nsum a = {0.0, 0.0};
  for (long i = 0; i < n; ++i) ns_add(&a, x[i] * y[i]);
  return a.s + a.c;
}

/* The RMS norm of eq. (10): (1/m sum v_i^2)^(1/2). */
double or_rms(const double* x, long n) {
  if (n <= 0) return 0.0;
  return sqrt(or_dot(x, x, n) / (double)n);
}

/* PSNR of Section 5: 20 log10(255 / ||u - u_hat||) with the RMS norm. */
double or_psnr(const double* u_true, const double* u_hat, long n) {
  or_nsum a = {0.0, 0.0};
  for (long i = 0; i < n; ++i) {
    double d = u_true[i] - u_hat[i];
    ns_add(&a, d * d);
  }
  double rms = sqrt((a.s + a.c) / (double)n);
  return 20.0 * log10(255.0 / rms);
}

/* ------------------------------------------------------------------------ */
/* Grid hierarchy (Section 2, nested grids; eq. 12-14)                       */
/* ------------------------------------------------------------------------ */

/* Level sizes, coarsest first.  Reading: n_{l-1} = ceil(n_l / 2) per axis,
 * which covers both the odd case ((sqrt(N)+1)^2/4) and the even case (N/4)
 * of the paper for square images, and extends to non-square ones.  Every
 * level must keep at least 3 nodes per axis.  Returns 0 or OR_EINVAL. */
int or_level_sizes(int H, int W, int L, int* hs, int* ws) {
  if (L < 1 || H < 1 || W < 1) return OR_EINVAL;
  hs[L - 1] = H;
  ws[L - 1] = W;
  for (int l = L - 1; l >= 1; --l) {
    hs[l - 1] = (hs[l] + 1) / 2;
    ws[l - 1] = (ws[l] + 1) / 2;
  }
  for (int l = 0; l < L; ++l)
    if (hs[l] < 3 || ws[l] < 3) return OR_EINVAL;
  return OR_OK;
}

/* Economic iteration counts m_l (Section 2, after Algorithm 2):
 *   l >  L0: m_l = ceil(m0 (L - L0)^2 beta^(L-l))
 *   l <= L0: m_l = ceil(sqrt(m_*) (L - (2 - eps0) l) h_l^(-2))
 * with L0 = L/2, m0 = 1, beta = 4, m_* = 1, eps0 = 1/2, h_l = (1/2)^(l-1);
 * the bracket [t] is read as ceil(t), and a cap is never below 1.
 * Reading: l > L0 is compared as reals (L0 may be a half-integer). */
int or_iteration_caps(int L, int* m) {
  if (L < 1) return OR_EINVAL;
  const double m0 = 1.0, beta = 4.0, mstar = 1.0, eps0 = 0.5;
  const double L0 = 0.5 * (double)L;
  for (int l = 1; l <= L; ++l) {
    double t;
    if ((double)l > L0) {
      t = m0 * (L - L0) * (L - L0) * pow(beta, (double)(L - l));
    } else {
      double hl = pow(0.5, (double)(l - 1));
      t = sqrt(mstar) * ((double)L - (2.0 - eps0) * (double)l) / (hl * hl);
    }
    double c = ceil(t);
    if (c < 1.0) c = 1.0;
    m[l - 1] = (int)c;
  }
  return OR_OK;
}

/* Restriction R_l by injection (eq. 12-13).  Reading: applied per axis, so
 * the coarse node (i, j) takes the fine value at (2i, 2j). */
void or_restrict(const double* gf, int Hf, int Wf, double* gc, int Hc, int Wc) {
  (void)Hf;
  for (int i = 0; i < Hc; ++i)
    for (int j = 0; j < Wc; ++j) gc[(long)i * Wc + j] = gf[(long)(2 * i) * Wf + 2 * j];
}

/* Coarse-level PSF for H_l = R_l H_{l+1} R_l^* (eq. 14).  The coarse operator
 * keeps every second tap of the fine PSF: psf_c(a, b) = s * psf(2a, 2b) with
 * radius floor(r/2).  Reading of the adjoint's scale s:
 *   mode 0 (default): sum-preserving, s = sum(psf) / sum_{a,b} psf(2a, 2b)
 *   mode 1: s = 4 (adjoint under the level-normalised inner product of eq. 10)
 *   mode 2: s = 1 (Euclidean adjoint of injection)
 * Returns OR_EINVAL if mode 0 meets a zero decimated sum. */
int or_coarse_psf(const double* psf, int r, int mode, double* psf_c) {
  int n = 2 * r + 1, rc = r / 2, nc = 2 * rc + 1;
  double tot = 0.0, sub = 0.0;
  for (int a = -r; a <= r; ++a)
    for (int b = -r; b <= r; ++b) tot += psf[(a + r) * n + (b + r)];
  for (int a = -rc; a <= rc; ++a)
    for (int b = -rc; b <= rc; ++b) sub += psf[(2 * a + r) * n + (2 * b + r)];
  double s;
  if (mode == 0) {
    if (sub == 0.0) return OR_EINVAL;
    s = tot / sub;
  } else if (mode == 1) {
    s = 4.0;
  } else if (mode == 2) {
    s = 1.0;
  } else {
    return OR_EINVAL;
  }
  for (int a = -rc; a <= rc; ++a)
    for (int b = -rc; b <= rc; ++b)
      psf_c[(a + rc) * nc + (b + rc)] = s * psf[(2 * a + r) * n + (2 * b + r)];
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Blur operator (eq. 1, 7, 9; Section 5)                                    */
/* ------------------------------------------------------------------------ */

/* y = H x: (H x)(i,j) = sum_{|a|,|b|<=r} psf(a,b) x(i-a, j-b), with x = 0
 * outside the image (zero boundary condition).  transpose != 0 gives
 * y = H^T x: (H^T x)(i,j) = sum psf(a,b) x(i+a, j+b). */
void or_conv(const double* x, int H, int W, const double* psf, int r, int transpose, double* y) {
  int n = 2 * r + 1;
  int sg = transpose ? 1 : -1;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      double acc = 0.0;
      for (int a = -r; a <= r; ++a) {
        int ii = i + sg * a;
        if (ii < 0 || ii >= H) continue;
        for (int b = -r; b <= r; ++b) {
          int jj = j + sg * b;
          if (jj < 0 || jj >= W) continue;
          acc += psf[(a + r) * n + (b + r)] * x[(long)ii * W + jj];
        }
      }
      y[(long)i * W + j] = acc;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Smoothers C_l^{m_l} (Section 2)                                           */
/* ------------------------------------------------------------------------ */

/* Reading: the paper's "CG" smoother is CG on the normal equations
 * H^T H u = H^T g (CGLS): two operator products per iteration.
 *
 *   r = g - H u0, s = H^T r, p = s, gamma = <s,s>, gamma0 = gamma, k = 0
 *   repeat:
 *     stop if (stop_rule and ||r|| <= c delta)      [discrepancy principle]
 *     stop if k == cap                               [m_l]
 *     stop if gamma == 0 or gamma <= eps^2 gamma0    [converged]
 *     q = H p, eta = <q,q>; stop if eta == 0
 *     alpha = gamma/eta, u += alpha p, r -= alpha q
 *     s = H^T r, gamma' = <s,s>, p = s + (gamma'/gamma) p, gamma = gamma', k++
 *
 * u holds u0 on entry and the result on exit.  rms_hist (length cap+1, may
 * be NULL) receives ||r_k|| (eq. 10) for k = 0..iters. */
int or_cgls(const double* g, int H, int W, const double* psf, int r, double* u, int cap, int stop_rule,
            double cdelta, double eps, int* iters_out, double* rms_hist, int* reason_out) {
  long N = (long)H * W;
  double* res = (double*)malloc(sizeof(double) * N);
  double* s = (double*)malloc(sizeof(double) * N);
  double* p = (double*)malloc(sizeof(double) * N);
  double* q = (double*)malloc(sizeof(double) * N);
  if (!res || !s || !p || !q) {
    free(res); free(s); free(p); free(q);
    return OR_ENOMEM;
  }
  or_conv(u, H, W, psf, r, 0, q);
  for (long t = 0; t < N; ++t) res[t] = g[t] - q[t];
  or_conv(res, H, W, psf, r, 1, s);
  memcpy(p, s, sizeof(double) * N);
  double gamma = or_dot(s, s, N), gamma0 = gamma;
  double rms = or_rms(res, N);
  int k = 0, reason = OR_STOP_NONE;
  if (rms_hist) rms_hist[0] = rms;
  for (;;) {
    if (stop_rule && rms <= cdelta) { reason = OR_STOP_DISCREPANCY; break; }
    if (k >= cap) { reason = OR_STOP_CAP; break; }
    if (gamma == 0.0 || gamma <= eps * eps * gamma0) { reason = OR_STOP_GUARD; break; }
    or_conv(p, H, W, psf, r, 0, q);
    double eta = or_dot(q, q, N);
    if (eta == 0.0) { reason = OR_STOP_GUARD; break; }
    double alpha = gamma / eta;
    for (long t = 0; t < N; ++t) {
      u[t] += alpha * p[t];
      res[t] -= alpha * q[t];
    }
    or_conv(res, H, W, psf, r, 1, s);
    double gnew = or_dot(s, s, N);
    double beta = gnew / gamma;
    for (long t = 0; t < N; ++t) p[t] = s[t] + beta * p[t];
    gamma = gnew;
    ++k;
    rms = or_rms(res, N);
    if (rms_hist) rms_hist[k] = rms;
  }
  free(res); free(s); free(p); free(q);
  if (iters_out) *iters_out = k;
  if (reason_out) *reason_out = reason;
  return OR_OK;
}

/* Reading: the paper's "MR" smoother is the minimal-residual iteration
 * (one operator product per iteration; steepest descent on ||g - H u||
 * along the residual direction):
 *
 *   r = g - H u0, k = 0
 *   repeat:
 *     stop if (stop_rule and ||r|| <= c delta); stop if k == cap
 *     stop if <r,r> == 0 or <r,r> <= eps^2 <r0,r0>
 *     q = H r, eta = <q,q>; stop if eta == 0
 *     alpha = <r,q>/eta, u += alpha r, r -= alpha q, k++
 */
int or_mr(const double* g, int H, int W, const double* psf, int r, double* u, int cap, int stop_rule,
          double cdelta, double eps, int* iters_out, double* rms_hist, int* reason_out) {
  long N = (long)H * W;
  double* res = (double*)malloc(sizeof(double) * N);
  double* q = (double*)malloc(sizeof(double) * N);
  if (!res || !q) {
    free(res); free(q);
    return OR_ENOMEM;
  }
  or_conv(u, H, W, psf, r, 0, q);
  for (long t = 0; t < N; ++t) res[t] = g[t] - q[t];
  double rr = or_dot(res, res, N), rr0 = rr;
  double rms = sqrt(rr / (double)N);
  int k = 0, reason = OR_STOP_NONE;
  if (rms_hist) rms_hist[0] = rms;
  for (;;) {
    if (stop_rule && rms <= cdelta) { reason = OR_STOP_DISCREPANCY; break; }
    if (k >= cap) { reason = OR_STOP_CAP; break; }
    if (rr == 0.0 || rr <= eps * eps * rr0) { reason = OR_STOP_GUARD; break; }
    or_conv(res, H, W, psf, r, 0, q);
    double eta = or_dot(q, q, N);
    if (eta == 0.0) { reason = OR_STOP_GUARD; break; }
    double alpha = or_dot(res, q, N) / eta;
    for (long t = 0; t < N; ++t) {
      u[t] += alpha * res[t];
      res[t] -= alpha * q[t];
    }
    ++k;
    rr = or_dot(res, res, N);
    rms = sqrt(rr / (double)N);
    if (rms_hist) rms_hist[k] = rms;
  }
  free(res); free(q);
  if (iters_out) *iters_out = k;
  if (reason_out) *reason_out = reason;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Prolongation operators (Section 3.1, 3.2)                                 */
/* ------------------------------------------------------------------------ */

/* Quadratic extrapolation of one virtual node from the three before it:
 * v_n = 3 v_{n-1} - 3 v_{n-2} + v_{n-3}; exact for quadratics. */
static double qext(double v1, double v2, double v3) { return 3.0 * v1 - 3.0 * v2 + v3; }

/* New extrapolation Pi (Section 3.2, 1-D rule and its 2-D form).
 * A = level l-1 (HA x WA), B = level l (HB x WB), HA = ceil(HB/2).
 * d(a, b) = uB(2a, 2b) - uA(a, b); the result on B is
 *   (even, even) uB + d/4                                 [(5 uB - uA)/4]
 *   (even, odd)  uB + (d(a,b) + d(a,b+1))/8               [edge midpoint]
 *   (odd, even)  uB + (d(a,b) + d(a+1,b))/8               [edge midpoint]
 *   (odd, odd)   uB + (d(a,b)+d(a+1,b)+d(a,b+1)+d(a+1,b+1))/16
 * Reading (cell centres, not given in the paper): the bilinear mean of the
 * four corner corrections, which continues the node and edge rules.
 * Reading (even n_B): d gets one virtual node per such axis by quadratic
 * extrapolation, first along j for the real rows, then along i. */
int or_extrapolate(const double* uA, int HA, int WA, const double* uB, int HB, int WB, double* ut) {
  if (HA != (HB + 1) / 2 || WA != (WB + 1) / 2 || HA < 3 || WA < 3) return OR_EINVAL;
  int ei = (HB % 2 == 0), ej = (WB % 2 == 0);
  int DH = HA + ei, DW = WA + ej;
  double* d = (double*)malloc(sizeof(double) * DH * DW);
  if (!d) return OR_ENOMEM;
  for (int a = 0; a < HA; ++a)
    for (int b = 0; b < WA; ++b) d[a * DW + b] = uB[(long)(2 * a) * WB + 2 * b] - uA[(long)a * WA + b];
  if (ej)
    for (int a = 0; a < HA; ++a)
      d[a * DW + WA] = qext(d[a * DW + WA - 1], d[a * DW + WA - 2], d[a * DW + WA - 3]);
  if (ei)
    for (int b = 0; b < DW; ++b)
      d[HA * DW + b] = qext(d[(HA - 1) * DW + b], d[(HA - 2) * DW + b], d[(HA - 3) * DW + b]);
  for (int p = 0; p < HB; ++p) {
    for (int q = 0; q < WB; ++q) {
      int a = p / 2, b = q / 2;
      double corr;
      if (p % 2 == 0 && q % 2 == 0)
        corr = d[a * DW + b] / 4.0;
      else if (p % 2 == 0)
        corr = (d[a * DW + b] + d[a * DW + b + 1]) / 8.0;
      else if (q % 2 == 0)
        corr = (d[a * DW + b] + d[(a + 1) * DW + b]) / 8.0;
      else
        corr = (d[a * DW + b] + d[(a + 1) * DW + b] + d[a * DW + b + 1] + d[(a + 1) * DW + b + 1]) / 16.0;
      ut[(long)p * WB + q] = uB[(long)p * WB + q] + corr;
    }
  }
  free(d);
  return OR_OK;
}

/* One axis of the quadratic interpolation P (Section 3.2): fine index I on
 * the next level, coarse values e[] with e[p] at node p of the B grid.  The
 * B nodes pair up into panels (2a, 2a+1, 2a+2) below one coarse cell of the
 * level before; the quarter points take the Lagrange weights (3/8, 3/4,
 * -1/8) and (-1/8, 3/4, 3/8). */
static double quad_axis(const double* e, long stride, int I) {
  int p = I / 2;
  if (I % 2 == 0) return e[(long)p * stride];
  if (p % 2 == 0) /* I = 4a + 1 */
    return 0.375 * e[(long)p * stride] + 0.75 * e[(long)(p + 1) * stride] - 0.125 * e[(long)(p + 2) * stride];
  /* I = 4a + 3, p = 2a + 1 */
  return -0.125 * e[(long)(p - 1) * stride] + 0.75 * e[(long)p * stride] + 0.375 * e[(long)(p + 1) * stride];
}

/* Quadratic interpolation prolongation P (Section 3.2): ut on level l
 * (HB x WB) -> uC on level l+1 (HC x WC), HB = ceil(HC/2).  Tensor product:
 * first along i, then along j.  Reading (border): where the panel of the
 * last fine nodes reaches past the B grid, ut is extended by two virtual
 * nodes per axis by quadratic extrapolation (along j for the real rows, then
 * along i), i.e. the quadratic through the last three real nodes. */
int or_prolong_quad(const double* ut, int HB, int WB, double* uC, int HC, int WC) {
  if (HB != (HC + 1) / 2 || WB != (WC + 1) / 2 || HB < 3 || WB < 3) return OR_EINVAL;
  int EH = HB + 2, EW = WB + 2;
  double* e = (double*)malloc(sizeof(double) * EH * EW);
  double* t = (double*)malloc(sizeof(double) * HC * EW);
  if (!e || !t) {
    free(e); free(t);
    return OR_ENOMEM;
  }
  for (int p = 0; p < HB; ++p) {
    for (int q = 0; q < WB; ++q) e[p * EW + q] = ut[(long)p * WB + q];
    e[p * EW + WB] = qext(e[p * EW + WB - 1], e[p * EW + WB - 2], e[p * EW + WB - 3]);
    e[p * EW + WB + 1] = qext(e[p * EW + WB], e[p * EW + WB - 1], e[p * EW + WB - 2]);
  }
  for (int q = 0; q < EW; ++q) {
    e[HB * EW + q] = qext(e[(HB - 1) * EW + q], e[(HB - 2) * EW + q], e[(HB - 3) * EW + q]);
    e[(HB + 1) * EW + q] = qext(e[HB * EW + q], e[(HB - 1) * EW + q], e[(HB - 2) * EW + q]);
  }
  for (int I = 0; I < HC; ++I)
    for (int q = 0; q < EW; ++q) t[(long)I * EW + q] = quad_axis(e + q, EW, I);
  for (int I = 0; I < HC; ++I)
    for (int J = 0; J < WC; ++J) uC[(long)I * WC + J] = quad_axis(t + (long)I * EW, 1, J);
  free(e); free(t);
  return OR_OK;
}

/* Linear prolongation L (eq. 15), 0-based: nodes copy, edge midpoints take
 * the mean of their two ends, cell centres the mean along the (a,b)-(a+1,b+1)
 * diagonal.  Reading (border): one virtual node per axis by linear
 * extrapolation (2 v_{n-1} - v_{n-2}), along j first, then along i. */
int or_prolong_linear(const double* uB, int HB, int WB, double* uC, int HC, int WC) {
  if (HB != (HC + 1) / 2 || WB != (WC + 1) / 2 || HB < 2 || WB < 2) return OR_EINVAL;
  int EH = HB + 1, EW = WB + 1;
  double* e = (double*)malloc(sizeof(double) * EH * EW);
  if (!e) return OR_ENOMEM;
  for (int p = 0; p < HB; ++p) {
    for (int q = 0; q < WB; ++q) e[p * EW + q] = uB[(long)p * WB + q];
    e[p * EW + WB] = 2.0 * e[p * EW + WB - 1] - e[p * EW + WB - 2];
  }
  for (int q = 0; q < EW; ++q) e[HB * EW + q] = 2.0 * e[(HB - 1) * EW + q] - e[(HB - 2) * EW + q];
  for (int I = 0; I < HC; ++I) {
    for (int J = 0; J < WC; ++J) {
      int a = I / 2, b = J / 2;
      double v;
      if (I % 2 == 0 && J % 2 == 0)
        v = e[a * EW + b];
      else if (I % 2 == 0)
        v = 0.5 * (e[a * EW + b] + e[a * EW + b + 1]);
      else if (J % 2 == 0)
        v = 0.5 * (e[a * EW + b] + e[(a + 1) * EW + b]);
      else
        v = 0.5 * (e[a * EW + b] + e[(a + 1) * EW + b + 1]);
      uC[(long)I * WC + J] = v;
    }
  }
  free(e);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local smoothing S (Section 3.3, eq. 18-19)                                */
/* ------------------------------------------------------------------------ */

/* For every pixel, fit a0 + a1 s + a2 t to the 3x3 neighbourhood with weights
 * w(s,t) = exp(-((u(i,j) - u(i+s,j+t)) / h)^2) and output a0.
 * Readings: h = 1 is the paper's literal (unscaled) weight; the centre
 * (weight 1) is part of the fit; neighbours outside the image are dropped;
 * weights are exactly 0 once (delta/h)^2 > 30; all pixels read the input
 * image (out of place).
 * Solution: a0 is the fitted value at the centre, unique for every
 * minimiser because the centre has positive weight.  The data are taken
 * relative to the centre value, a0 is eliminated through the weighted
 * centroid (a0 = vbar - a1 sbar - a2 tbar), and the centred 2x2 system
 * S (a1, a2) = rhs is solved through its eigen-decomposition, dropping
 * eigenvalues below 1e-12 of the largest (pseudo-inverse).  Near-collinear
 * weight patterns make S nearly singular; this form keeps a0 accurate
 * there, where Cramer's rule would not. */
void or_local_smooth(const double* u, int H, int W, double h, double* out) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      double uc = u[(long)i * W + j];
      double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0, b0 = 0, b1 = 0, b2 = 0;
      for (int s = -1; s <= 1; ++s) {
        for (int t = -1; t <= 1; ++t) {
          int ii = i + s, jj = j + t;
          if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
          double v = u[(long)ii * W + jj] - uc;
          double z = v / h;
          double e = z * z;
          double w = (e > 30.0) ? 0.0 : exp(-e);
          m00 += w; m01 += w * s; m02 += w * t;
          m11 += w * s * s; m12 += w * s * t; m22 += w * t * t;
          b0 += w * v; b1 += w * s * v; b2 += w * t * v;
        }
      }
      double sb = m01 / m00, tb = m02 / m00, vb = b0 / m00;
      /* centred normal equations */
      double S11 = m11 - m01 * sb, S12 = m12 - m01 * tb, S22 = m22 - m02 * tb;
      double r1 = b1 - m01 * vb, r2 = b2 - m02 * vb;
      /* eigen-decomposition of the symmetric 2x2 S by one plane rotation */
      double th = 0.5 * atan2(2.0 * S12, S11 - S22);
      double cs = cos(th), sn = sin(th);
      double l1 = S11 * cs * cs + 2.0 * S12 * cs * sn + S22 * sn * sn;
      double l2 = S11 * sn * sn - 2.0 * S12 * cs * sn + S22 * cs * cs;
      double lmax = fabs(l1) > fabs(l2) ? fabs(l1) : fabs(l2);
      double corr = 0.0; /* (sbar, tbar) . S^+ rhs */
      if (l1 > 1e-12 * lmax && l1 > 0.0) corr += (sb * cs + tb * sn) * (r1 * cs + r2 * sn) / l1;
      if (l2 > 1e-12 * lmax && l2 > 0.0) corr += (-sb * sn + tb * cs) * (-r1 * sn + r2 * cs) / l2;
      out[(long)i * W + j] = uc + (vb - corr);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Edge-preserving denoising D (Section 4, eq. 21, 23-26)                    */
/* ------------------------------------------------------------------------ */

/* One explicit Perona-Malik step u^{n+1} = u^n + tau A(u^n) u^n (eq. 25):
 *   out(i,j) = u + tau sum_{nb in Q(i,j)} (c(nb) + c(i,j))/2 (u(nb) - u(i,j))
 * with c = 1 / (1 + |grad u|^2 / k^2) (eq. 21).
 * Readings: |grad u| from central differences with the border replicated;
 * neighbours outside the image drop out of the sum (zero-flux boundary). */
void or_pm_step(const double* u, int H, int W, double k, double tau, double* out) {
  long N = (long)H * W;
  double* c = (double*)malloc(sizeof(double) * N);
  if (!c) return;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      int ip = i + 1 < H ? i + 1 : H - 1, im = i > 0 ? i - 1 : 0;
      int jp = j + 1 < W ? j + 1 : W - 1, jm = j > 0 ? j - 1 : 0;
      double ux = 0.5 * (u[(long)ip * W + j] - u[(long)im * W + j]);
      double uy = 0.5 * (u[(long)i * W + jp] - u[(long)i * W + jm]);
      double g2 = ux * ux + uy * uy;
      c[(long)i * W + j] = 1.0 / (1.0 + g2 / (k * k));
    }
  }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < H; ++i) {
    for (int j = 0; j < W; ++j) {
      long o = (long)i * W + j;
      double uc = u[o], cc = c[o], acc = 0.0;
      if (i + 1 < H) acc += 0.5 * (c[o + W] + cc) * (u[o + W] - uc);
      if (i > 0) acc += 0.5 * (c[o - W] + cc) * (u[o - W] - uc);
      if (j + 1 < W) acc += 0.5 * (c[o + 1] + cc) * (u[o + 1] - uc);
      if (j > 0) acc += 0.5 * (c[o - 1] + cc) * (u[o - 1] - uc);
      out[o] = uc + tau * acc;
    }
  }
  free(c);
}

/* ------------------------------------------------------------------------ */
/* Cascades (Algorithm 1 IECMG, Algorithm 2 EECMG)                           */
/* ------------------------------------------------------------------------ */

#define OR_MAX_LEVELS 32

static int run_smoother(int smoother, const double* g, int H, int W, const double* psf, int r, double* u, int cap,
                        int stop_rule, double cdelta, double eps, int* it, double* fin_rms, int* reason) {
  double* hist = (double*)malloc(sizeof(double) * ((size_t)cap + 1));
  if (!hist) return OR_ENOMEM;
  int rc = smoother == 1 ? or_mr(g, H, W, psf, r, u, cap, stop_rule, cdelta, eps, it, hist, reason)
                         : or_cgls(g, H, W, psf, r, u, cap, stop_rule, cdelta, eps, it, hist, reason);
  if (rc == OR_OK && fin_rms) *fin_rms = hist[*it];
  free(hist);
  return rc;
}

/* Restore u from g_delta (H x W).
 *   cascade: 0 = EECMG (Algorithm 2), 1 = IECMG-L, 2 = IECMG-P (Algorithm 1)
 *   smoother: 0 = CGLS, 1 = MR
 *   caps: n_levels iteration caps (coarsest first) or NULL for the m_l rule
 * Readings (Algorithm 2): levels 1 and 2 start from zero; the transfer loop
 * runs l = 2..L-1 and produces u_{l+1}; L = 1 is one smoother run on the
 * finest grid.  S is applied once, then D pm_steps times.  The stopping rule
 * uses the same delta on every level.
 * Outputs: u_out (H x W); per level iterations, final residual RMS, stop
 * reason and PSF radius (each of length n_levels, may be NULL). */
int or_restore(const double* g_delta, int H, int W, const double* psf, int r, int n_levels, const int* caps_in,
               double k, int stop_rule, double delta, double c, double tau, int pm_steps, double smooth_h,
               int coarse_psf_mode, double guard_eps, int smoother, int cascade, double* u_out, int* iters_out,
               double* rms_out, int* reason_out, int* radius_out) {
  int L = n_levels;
  if (L < 1 || L > OR_MAX_LEVELS || r < 0 || k <= 0.0 || tau <= 0.0 || tau > 0.25 || pm_steps < 0 ||
      smooth_h <= 0.0 || (stop_rule && c <= 1.0) || cascade < 0 || cascade > 2 || smoother < 0 || smoother > 1)
    return OR_EINVAL;
  int hs[OR_MAX_LEVELS], ws[OR_MAX_LEVELS], rad[OR_MAX_LEVELS], caps[OR_MAX_LEVELS];
  if (or_level_sizes(H, W, L, hs, ws) != OR_OK) return OR_EINVAL;
  if (caps_in)
    for (int l = 0; l < L; ++l) caps[l] = caps_in[l];
  else
    or_iteration_caps(L, caps);
  for (int l = 0; l < L; ++l)
    if (caps[l] < 0) return OR_EINVAL;

  double* psfs[OR_MAX_LEVELS] = {0};
  double* gs[OR_MAX_LEVELS] = {0};
  double* us[OR_MAX_LEVELS] = {0};
  double *t1 = NULL, *t2 = NULL;
  int rc = OR_OK;

  /* PSF pyramid, finest first (eq. 14) */
  rad[L - 1] = r;
  psfs[L - 1] = (double*)malloc(sizeof(double) * (2 * r + 1) * (2 * r + 1));
  if (!psfs[L - 1]) { rc = OR_ENOMEM; goto done; }
  memcpy(psfs[L - 1], psf, sizeof(double) * (2 * r + 1) * (2 * r + 1));
  for (int l = L - 2; l >= 0; --l) {
    rad[l] = rad[l + 1] / 2;
    psfs[l] = (double*)malloc(sizeof(double) * (2 * rad[l] + 1) * (2 * rad[l] + 1));
    if (!psfs[l]) { rc = OR_ENOMEM; goto done; }
    rc = or_coarse_psf(psfs[l + 1], rad[l + 1], coarse_psf_mode, psfs[l]);
    if (rc != OR_OK) goto done;
  }
  /* right-hand sides (eq. 12-13) and solutions */
  for (int l = 0; l < L; ++l) {
    gs[l] = (double*)malloc(sizeof(double) * hs[l] * ws[l]);
    us[l] = (double*)calloc((size_t)hs[l] * ws[l], sizeof(double));
    if (!gs[l] || !us[l]) { rc = OR_ENOMEM; goto done; }
  }
  memcpy(gs[L - 1], g_delta, sizeof(double) * H * W);
  for (int l = L - 2; l >= 0; --l) or_restrict(gs[l + 1], hs[l + 1], ws[l + 1], gs[l], hs[l], ws[l]);
  t1 = (double*)malloc(sizeof(double) * H * W);
  t2 = (double*)malloc(sizeof(double) * H * W);
  if (!t1 || !t2) { rc = OR_ENOMEM; goto done; }

  double cdelta = c * delta;
  double eps = guard_eps;
  int fine_start; /* first level reached by a transfer */
  double frms;
  int it, why;
  if (cascade == 0) {
    /* Algorithm 2, Step 1: levels 1 and 2 from zero */
    int nstart = L >= 2 ? 2 : 1;
    for (int l = 0; l < nstart; ++l) {
      rc = run_smoother(smoother, gs[l], hs[l], ws[l], psfs[l], rad[l], us[l], caps[l], stop_rule, cdelta, eps, &it,
                        &frms, &why);
      if (rc != OR_OK) goto done;
      if (iters_out) iters_out[l] = it;
      if (rms_out) rms_out[l] = frms;
      if (reason_out) reason_out[l] = why;
    }
    fine_start = 2; /* 0-based index of level 3 */
  } else {
    /* Algorithm 1, Step 1: level 1 from zero */
    rc = run_smoother(smoother, gs[0], hs[0], ws[0], psfs[0], rad[0], us[0], caps[0], stop_rule, cdelta, eps, &it,
                      &frms, &why);
    if (rc != OR_OK) goto done;
    if (iters_out) iters_out[0] = it;
    if (rms_out) rms_out[0] = frms;
    if (reason_out) reason_out[0] = why;
    fine_start = 1;
  }
  for (int lc = fine_start; lc < L; ++lc) {
    /* lc: 0-based index of the level being built */
    int lb = lc - 1;
    if (cascade == 0) {
      int la = lc - 2;
      rc = or_extrapolate(us[la], hs[la], ws[la], us[lb], hs[lb], ws[lb], t2);
      if (rc != OR_OK) goto done;
      rc = or_prolong_quad(t2, hs[lb], ws[lb], t1, hs[lc], ws[lc]);
    } else if (cascade == 1) {
      rc = or_prolong_linear(us[lb], hs[lb], ws[lb], t1, hs[lc], ws[lc]);
    } else {
      rc = or_prolong_quad(us[lb], hs[lb], ws[lb], t1, hs[lc], ws[lc]);
    }
    if (rc != OR_OK) goto done;
    or_local_smooth(t1, hs[lc], ws[lc], smooth_h, us[lc]);
    for (int st = 0; st < pm_steps; ++st) {
      or_pm_step(us[lc], hs[lc], ws[lc], k, tau, t1);
      memcpy(us[lc], t1, sizeof(double) * hs[lc] * ws[lc]);
    }
    rc = run_smoother(smoother, gs[lc], hs[lc], ws[lc], psfs[lc], rad[lc], us[lc], caps[lc], stop_rule, cdelta, eps,
                      &it, &frms, &why);
    if (rc != OR_OK) goto done;
    if (iters_out) iters_out[lc] = it;
    if (rms_out) rms_out[lc] = frms;
    if (reason_out) reason_out[lc] = why;
  }
  memcpy(u_out, us[L - 1], sizeof(double) * H * W);
  if (radius_out)
    for (int l = 0; l < L; ++l) radius_out[l] = rad[l];

done:
  for (int l = 0; l < L; ++l) {
    free(psfs[l]);
    free(gs[l]);
    free(us[l]);
  }
  free(t1);
  free(t2);
  return rc;
}

/* Thread count of the pixel loops (results do not depend on it). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int or_num_threads(void) { return 1; }
void or_set_num_threads(int n) { (void)n; }
#endif
