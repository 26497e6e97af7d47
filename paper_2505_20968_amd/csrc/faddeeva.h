// FP64 Faddeeva function w(z) = exp(-z^2) erfc(-i z) for Im z >= 0, usable on
// host and device.  The paper (Sect. 2.4) writes W(a, v) = w(v + i a).
//
// Two published methods are combined:
//  * |z| < 15: J.A.C. Weideman, "Computation of the complex error function",
//    SIAM J. Numer. Anal. 31 (1994) 1497-1518: with L = sqrt(N/sqrt(2)) and
//    Z = (L + i z)/(L - i z),
//        w(z) = 2 p(Z)/(L - i z)^2 + 1/(sqrt(pi) (L - i z)),
//    p a polynomial of degree N-1 whose coefficients are the Fourier
//    coefficients of exp(-t^2)(L^2 + t^2) on t = L tan(theta/2).  Here
//    N = 40, a relative error of about 1.7e-14 inside |z| = 15 (N = 36 gives
//    2.4e-14 and is spread wider, enough to move formal solutions through
//    optically thick slabs by 1e-12); the coefficients are computed on the
//    host at library load (faddeeva_init) by a direct discrete Fourier
//    transform and copied to constant memory.
//  * |z| >= 15: the Laplace continued fraction (Gautschi 1970; Jones, Thron &
//    Waadeland 1981) w(z) = (i/sqrt(pi)) / (z - (1/2)/(z - 1/(z - (3/2)/(z - ...)))),
//    evaluated bottom-up.  The depth falls with |z|: the truncation error
//    of n levels shrinks roughly like (n / (2|z|^2))^n, so ten levels reach
//    FP64 rounding at |z| = 15 and three beyond |z| ~ 3000.  The depth table
//    below keeps one to two levels above the smallest depth that agrees with a
//    40-level evaluation to rounding on both half-plane axes and in between.
#pragma once

#include <hip/hip_runtime.h>

namespace trap {

constexpr int kWeidemanN = 40;

struct FaddeevaCoef {
  double L;
  double a[kWeidemanN];   // highest power first (Horner order)
};

// Host-side computation of the Weideman coefficients.
void faddeeva_coefficients(FaddeevaCoef* out);

// 1/d for a positive normal d: the hardware estimate and two Newton steps
// (each doubles the number of correct bits), within a few ulp, in five vector
// instructions instead of the IEEE division sequence.
__device__ __forceinline__ double fad_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Depth of the continued fraction at |z|^2 = r2 >= 225.
__device__ __forceinline__ int fad_cf_depth(double r2) {
  return r2 < 400.0 ? 10 : r2 < 900.0 ? 9 : r2 < 2500.0 ? 8 : r2 < 1e4 ? 7
       : r2 < 4e4 ? 6 : r2 < 2.5e5 ? 5 : r2 < 1e7 ? 4 : 3;
}

// w(x_j + i y), y >= 0, at K points that share y.  The K evaluations run side
// by side (independent dependency chains, each polynomial coefficient fetched
// once for all K): a lane takes the rational form if any of its points lies
// inside |z| = 15 and the continued fraction if any lies outside, the latter
// with the deepest level its points need (more levels only bring the
// truncated fraction closer to its limit), and keeps per point the branch
// that point belongs to.
template <int K>
__device__ inline void faddeeva_wk(const double (&x)[K], double y, const FaddeevaCoef& C, double2 (&w)[K]) {
  bool near[K];
  bool any_near = false, any_far = false;
  int depth = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double r2 = fma(x[j], x[j], y * y);
    near[j] = r2 < 225.0;
    any_near |= near[j];
    any_far |= !near[j];
    if (!near[j]) depth = max(depth, fad_cf_depth(r2));
  }
  if (any_near) {
    // Weideman rational form: t = L - i z = (L + y) - i x,
    // Z = (L + i z)/(L - i z) with L + i z = (L - y) + i x
    const double tr = C.L + y, nr = C.L - y;
    double Zr[K], Zi[K], itd[K], pr[K], pi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      itd[j] = fad_rcp(fma(x[j], x[j], tr * tr));
      // (nr + i x)(tr + i x) / |t|^2
      Zr[j] = fma(-x[j], x[j], nr * tr) * itd[j];
      Zi[j] = x[j] * (tr + nr) * itd[j];
      pr[j] = C.a[0];
      pi[j] = 0.0;
    }
    for (int k = 1; k < kWeidemanN; ++k) {
      const double ak = C.a[k];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double qr = fma(pr[j], Zr[j], fma(-pi[j], Zi[j], ak));
        pi[j] = fma(pr[j], Zi[j], pi[j] * Zr[j]);
        pr[j] = qr;
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (!near[j]) continue;
      // 1/t = (tr + i x) / |t|^2 for t = tr - i x, and 1/t^2
      const double ir = tr * itd[j], ii = x[j] * itd[j];
      const double i2r = fma(ir, ir, -ii * ii), i2i = 2.0 * ir * ii;
      w[j].x = fma(2.0, fma(pr[j], i2r, -pi[j] * i2i), 0.56418958354775628695 * ir);
      w[j].y = fma(2.0, fma(pr[j], i2i, pi[j] * i2r), 0.56418958354775628695 * ii);
    }
  }
  if (any_far) {
    // continued fraction, bottom-up: f_k = z - (k/2)/f_{k+1}, w = (i/sqrt(pi))/f_1
    double fr[K], fi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      fr[j] = x[j];
      fi[j] = y;
    }
    for (int k = depth; k >= 1; --k) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double c = (0.5 * k) * fad_rcp(fma(fr[j], fr[j], fi[j] * fi[j]));
        fr[j] = fma(-c, fr[j], x[j]);
        fi[j] = fma(c, fi[j], y);
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (near[j]) continue;
      const double s = 0.56418958354775628695 * fad_rcp(fma(fr[j], fr[j], fi[j] * fi[j]));   // 1/sqrt(pi)
      w[j].x = s * fi[j];
      w[j].y = s * fr[j];
    }
  }
}

__device__ inline double2 faddeeva_w(double x, double y, const FaddeevaCoef& C) {
  // returns w(x + i y), y >= 0
  const double xs[1] = {x};
  double2 w[1];
  faddeeva_wk<1>(xs, y, C, w);
  return w[0];
}

}  // namespace trap
