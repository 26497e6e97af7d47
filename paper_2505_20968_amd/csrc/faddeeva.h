// FP64 Faddeeva function w(z) = exp(-z^2) erfc(-i z) for Im z >= 0, usable on
// host and device.  The paper (Sect. 2.4) writes W(a, v) = w(v + i a).
//
// Two published methods are combined:
//  * |z| < 15: J.A.C. Weideman, "Computation of the complex error function",
//    SIAM J. Numer. Anal. 31 (1994) 1497-1518: with L = sqrt(N/sqrt(2)) and
//    Z = (L + i z)/(L - i z),
//        w(z) = 2 p(Z)/(L - i z)^2 + 1/(sqrt(pi) (L - i z)),
//    p a polynomial of degree N-1 whose coefficients are the Fourier
//    coefficients of exp(-t^2)(L^2 + t^2) on t = L tan(theta/2).  Here N = 40;
//    the coefficients are computed on the host at library load (faddeeva_init)
//    by a direct discrete Fourier transform and copied to constant memory.
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

__host__ __device__ inline double2 faddeeva_w(double x, double y, const FaddeevaCoef& C) {
  // returns w(x + i y), y >= 0
  const double r2 = x * x + y * y;
  if (r2 >= 225.0) {
    // continued fraction, bottom-up: f_k = z - (k/2)/f_{k+1}
    const int depth = r2 < 400.0 ? 10 : r2 < 900.0 ? 9 : r2 < 2500.0 ? 8 : r2 < 1e4 ? 7
                    : r2 < 4e4 ? 6 : r2 < 2.5e5 ? 5 : r2 < 1e7 ? 4 : 3;
    double fr = x, fi = y;       // f = z
    for (int k = depth; k >= 1; --k) {
      // f = z - (k/2) / f
      const double d = fr * fr + fi * fi;
      const double c = 0.5 * k / d;
      fr = x - c * fr;
      fi = y + c * fi;
    }
    // w = (i/sqrt(pi)) / f
    const double d = fr * fr + fi * fi;
    const double s = 0.56418958354775628695 / d;   // 1/sqrt(pi)
    return make_double2(s * fi, s * fr);
  }
  // Weideman rational form: t = L - i z = (L + y) - i x
  const double tr = C.L + y, ti = -x;
  // Z = (L + i z)/(L - i z); L + i z = (L - y) + i x
  const double nr = C.L - y, ni = x;
  const double itd = 1.0 / (tr * tr + ti * ti);
  const double Zr = (nr * tr + ni * ti) * itd;
  const double Zi = (ni * tr - nr * ti) * itd;
  double pr = C.a[0], pi = 0.0;
  for (int k = 1; k < kWeidemanN; ++k) {
    const double qr = pr * Zr - pi * Zi + C.a[k];
    const double qi = pr * Zi + pi * Zr;
    pr = qr;
    pi = qi;
  }
  // 1/t and 1/t^2
  const double ir = tr * itd, ii = -ti * itd;
  const double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
  const double wr = 2.0 * (pr * i2r - pi * i2i) + 0.56418958354775628695 * ir;
  const double wi = 2.0 * (pr * i2i + pi * i2r) + 0.56418958354775628695 * ii;
  return make_double2(wr, wi);
}

}  // namespace trap
