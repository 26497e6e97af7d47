// Host-side problem setup in FP64: grids, scattering-angle table, sublevel
// structure and dipole vectors, coefficient tables, spline coefficient map.
//
// Physics (paper Sects. 2.2-2.3, App. B, Sect. 6.1):
//  * dnu_D(z) = (nu0/c) sqrt(2 k T/M + xi^2); u = x lam(z), lam = dnu_D_ref/dnu_D.
//  * a = (G_R + G_I + G_E)/(4 pi dnu_D), eps = G_I/(G_R + G_I), G_E = r_E (G_R + G_I).
//  * alpha_{u u'} = G_R/(G_R+G_I+G_E + 2 pi i nu_{u u'}),
//    beta_{u u'}  = G_R/(G_R+G_I + 2 pi i nu_{u u'}).
//  * Upper term: zeta (L.S + c) + nu_L (M_L + 2 M_S) in the uncoupled basis
//    (Paschen-Back), diagonalised per height; lower term nu_L (M_L + 2 M_S);
//    two-level atom: nu_L g M.  Dipoles from the Wigner-Eckart theorem on L.
//  * Stokes tensors Acart_j = sum_ab (A_j)_ab e_a e_b^T with
//    A = (1, sigma_z, sigma_x, -sigma_y) in the (e_a, e_b) ray basis.
#include <algorithm>
#include <cmath>
#include <complex>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "faddeeva.h"
#include "trap_internal.h"

namespace trap {


namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 2.99792458e10;
constexpr double kKB = 1.380649e-16;
constexpr double kAMU = 1.66053906660e-24;
constexpr double kLarmorPerG = 1.39962449361e6;

// ---------------------------------------------------------------- Gauss-Legendre on [0,1]
void gauss_legendre01(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      double dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // final derivative for the weight
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? z : p1;
        pm = (n == 1) ? 1.0 : p0;
        dp = n * (z * pn - pm) / (z * z - 1.0);
        t[i] = 0.5 * (1.0 - z);                       // ascending on [0,1]
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);       // half of the [-1,1] weight
        break;
      }
    }
  }
}

// ---------------------------------------------------------------- Wigner 3j (Racah formula)
// log n!, tabulated once
double lfact(int n) {
  static const std::vector<double> tab = [] {
    std::vector<double> t(256);
    for (int k = 0; k < 256; ++k) t[k] = std::lgamma(k + 1.0);
    return t;
  }();
  return n < 256 ? tab[n] : std::lgamma(n + 1.0);
}

double wigner3j(double j1, double j2, double j3, double m1, double m2, double m3) {
  auto I = [](double v) { return static_cast<int>(std::lround(v)); };
  if (std::fabs(m1 + m2 + m3) > 1e-9) return 0.0;
  if (std::fabs(m1) > j1 + 1e-9 || std::fabs(m2) > j2 + 1e-9 || std::fabs(m3) > j3 + 1e-9) return 0.0;
  if (j3 > j1 + j2 + 1e-9 || j3 < std::fabs(j1 - j2) - 1e-9) return 0.0;
  const int a1 = I(j1 + j2 - j3), a2 = I(j1 - j2 + j3), a3 = I(-j1 + j2 + j3), a4 = I(j1 + j2 + j3 + 1);
  double ltri = 0.5 * (lfact(a1) + lfact(a2) + lfact(a3) - lfact(a4));
  double lm = 0.5 * (lfact(I(j1 + m1)) + lfact(I(j1 - m1)) + lfact(I(j2 + m2)) + lfact(I(j2 - m2)) +
                     lfact(I(j3 + m3)) + lfact(I(j3 - m3)));
  int kmin = std::max({0, I(j2 - j3 - m1), I(j1 - j3 + m2)});
  int kmax = std::min({I(j1 + j2 - j3), I(j1 - m1), I(j2 + m2)});
  double sum = 0.0;
  for (int k = kmin; k <= kmax; ++k) {
    double ld = lfact(k) + lfact(I(j3 - j2 + k + m1)) + lfact(I(j3 - j1 + k - m2)) +
                lfact(I(j1 + j2 - j3 - k)) + lfact(I(j1 - k - m1)) + lfact(I(j2 - k + m2));
    sum += ((k & 1) ? -1.0 : 1.0) * std::exp(ltri + lm - ld);
  }
  int ph = I(j1 - j2 - m3);
  return ((ph & 1) ? -1.0 : 1.0) * sum;
}

// ---------------------------------------------------------------- Jacobi eigensolver (real symmetric)
void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& evals, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  // sort ascending, eigenvectors in columns of V
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return A[i * n + i] < A[j * n + j]; });
  evals.resize(n);
  std::vector<double> Vs(n * n);
  for (int c = 0; c < n; ++c) {
    evals[c] = A[idx[c] * n + idx[c]];
    for (int r = 0; r < n; ++r) Vs[r * n + c] = V[r * n + idx[c]];
  }
  V.swap(Vs);
}

struct TermBasis {
  std::vector<double> ml, ms;
};

TermBasis term_basis(double L, double S) {
  TermBasis b;
  for (int i = 0; i <= static_cast<int>(std::lround(2 * L)); ++i)
    for (int j = 0; j <= static_cast<int>(std::lround(2 * S)); ++j) {
      b.ml.push_back(-L + i);
      b.ms.push_back(-S + j);
    }
  return b;
}

std::vector<double> term_hamiltonian(const TermBasis& b, double L, double S, double zeta,
                                     double shift, double nuL, double gL, double gS) {
  const int n = static_cast<int>(b.ml.size());
  std::vector<double> H(n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    H[a * n + a] = zeta * (b.ml[a] * b.ms[a] + shift) + nuL * (gL * b.ml[a] + gS * b.ms[a]);
    for (int c = 0; c < n; ++c) {
      // (L+ S- + L- S+)/2 between |ml, ms> (column a) and |ml', ms'> (row c)
      if (std::fabs(b.ml[c] - b.ml[a] - 1) < 1e-9 && std::fabs(b.ms[c] - b.ms[a] + 1) < 1e-9) {
        double v = std::sqrt(L * (L + 1) - b.ml[a] * (b.ml[a] + 1)) *
                   std::sqrt(S * (S + 1) - b.ms[a] * (b.ms[a] - 1));
        H[c * n + a] += 0.5 * zeta * v;
      }
      if (std::fabs(b.ml[c] - b.ml[a] + 1) < 1e-9 && std::fabs(b.ms[c] - b.ms[a] - 1) < 1e-9) {
        double v = std::sqrt(L * (L + 1) - b.ml[a] * (b.ml[a] - 1)) *
                   std::sqrt(S * (S + 1) - b.ms[a] * (b.ms[a] + 1));
        H[c * n + a] += 0.5 * zeta * v;
      }
    }
  }
  return H;
}

struct Sublevels {
  std::vector<double> Eu, El;       // Hz relative to nu0
  std::vector<cd> d;                // [nu][nl][3] atmospheric frame
  double c_abs = 0, c_sc = 0;
};

Sublevels sublevels(const trap_atom_desc& at, double Bg, double thB, double chB, double dnuD_ref) {
  Sublevels s;
  const double nuL = kLarmorPerG * Bg;
  double Lu, Ll, S, zeta = 0.0, shift = 0.0, gLu, gSu, gLl, gSl;
  if (at.kind == 0) {
    Lu = at.J_u;
    Ll = at.J_l;
    S = 0.0;
    gLu = at.g_u;
    gSu = 0.0;
    gLl = at.g_l;
    gSl = 0.0;
  } else {
    Lu = at.L_u;
    Ll = at.L_l;
    S = at.S;
    auto ls = [&](double J) { return 0.5 * (J * (J + 1) - Lu * (Lu + 1) - S * (S + 1)); };
    double Jhi = Lu + S, Jlo = std::fabs(Lu - S);
    double gap = ls(Jhi) - ls(Jlo);
    zeta = (gap != 0.0) ? at.fs_split_x * dnuD_ref / gap : 0.0;
    shift = -0.5 * (ls(Jhi) + ls(Jlo));
    gLu = 1.0;
    gSu = 2.0;
    gLl = 1.0;
    gSl = 2.0;
  }
  TermBasis bu = term_basis(Lu, S), bl = term_basis(Ll, S);
  const int nu = static_cast<int>(bu.ml.size()), nl = static_cast<int>(bl.ml.size());
  std::vector<double> Vu, Vl;
  jacobi_eigen(nu, term_hamiltonian(bu, Lu, S, zeta, shift, nuL, gLu, gSu), s.Eu, Vu);
  jacobi_eigen(nl, term_hamiltonian(bl, Ll, S, 0.0, 0.0, nuL, gLl, gSl), s.El, Vl);
  // spherical components q = -1, 0, 1 in the uncoupled basis
  std::vector<double> Dq(3 * nu * nl, 0.0);
  for (int a = 0; a < nu; ++a)
    for (int b = 0; b < nl; ++b) {
      if (std::fabs(bu.ms[a] - bl.ms[b]) > 1e-9) continue;
      for (int iq = 0; iq < 3; ++iq) {
        const double q = iq - 1.0;
        const int ph = static_cast<int>(std::lround(Lu - bu.ml[a]));
        Dq[(iq * nu + a) * nl + b] =
            std::sqrt(3.0) * ((ph & 1) ? -1.0 : 1.0) * wigner3j(Lu, 1.0, Ll, -bu.ml[a], q, bl.ml[b]);
      }
    }
  // magnetic-frame unit vectors in the atmospheric frame
  const double st = std::sin(thB), ct = std::cos(thB), sc = std::sin(chB), cc = std::cos(chB);
  const double xB[3] = {ct * cc, ct * sc, -st}, yB[3] = {-sc, cc, 0.0}, zB[3] = {st * cc, st * sc, ct};
  // e_q^* for q = -1, 0, +1 (e_{+-1} = -+(x + i y)/sqrt2 -> conj)
  const double r2 = 1.0 / std::sqrt(2.0);
  cd econj[3][3];
  for (int k = 0; k < 3; ++k) {
    econj[0][k] = cd(xB[k] * r2, -yB[k] * r2);     // e_{-1}^* = (x - i y)^*/sqrt2 ... see below
    econj[1][k] = cd(zB[k], 0.0);
    econj[2][k] = cd(-xB[k] * r2, yB[k] * r2);
  }
  // e_{-1} = (x - i y)/sqrt2 -> conj = (x + i y)/sqrt2 ; e_{+1} = -(x + i y)/sqrt2 -> conj = -(x - i y)/sqrt2
  for (int k = 0; k < 3; ++k) {
    econj[0][k] = cd(xB[k] * r2, yB[k] * r2);
    econj[2][k] = cd(-xB[k] * r2, yB[k] * r2);
  }
  s.d.assign(nu * nl * 3, cd(0.0, 0.0));
  for (int ku = 0; ku < nu; ++ku)
    for (int kl = 0; kl < nl; ++kl) {
      for (int iq = 0; iq < 3; ++iq) {
        double val = 0.0;   // <u_ku| D_q | l_kl> with real eigenvectors
        for (int a = 0; a < nu; ++a) {
          if (Vu[a * nu + ku] == 0.0) continue;
          for (int b = 0; b < nl; ++b) val += Vu[a * nu + ku] * Dq[(iq * nu + a) * nl + b] * Vl[b * nl + kl];
        }
        for (int k = 0; k < 3; ++k) s.d[(ku * nl + kl) * 3 + k] += val * econj[iq][k];
      }
    }
  double tot = 0.0;
  std::vector<double> Du(nu, 0.0);
  for (int ku = 0; ku < nu; ++ku)
    for (int kl = 0; kl < nl; ++kl)
      for (int k = 0; k < 3; ++k) {
        double v = std::norm(s.d[(ku * nl + kl) * 3 + k]);
        tot += v;
        Du[ku] += v;
      }
  s.c_abs = 3.0 / tot;
  s.c_sc = 3.0 * s.c_abs / (2.0 * Du[0]);
  return s;
}

// d1^T Acart_j d2^* with Acart_j = sum_ab (A_j)_ab e_a e_b^T
// projections of a dipole vector on the two polarisation axes of a direction
void stokes_proj(const cd* d, const double* ea, const double* eb, cd* pa, cd* pb) {
  cd a(0, 0), b(0, 0);
  for (int k = 0; k < 3; ++k) {
    a += d[k] * ea[k];
    b += d[k] * eb[k];
  }
  *pa = a;
  *pb = b;
}

// Stokes component j of the pair (d1, d2) from the projections of d1 and the
// conjugated projections of d2 (ea, eb real, so those are the conjugates of
// d2's projections, exactly)
cd stokes_pair(int j, cd pa1, cd pb1, cd pa2, cd pb2) {
  const cd I(0.0, 1.0);
  switch (j) {
    case 0: return pa1 * pa2 + pb1 * pb2;
    case 1: return pa1 * pa2 - pb1 * pb2;
    case 2: return pa1 * pb2 + pb1 * pa2;
    default: return I * pa1 * pb2 - I * pb1 * pa2;
  }
}

// Not-a-knot cubic spline coefficient map on nodes x: on interval k with
// t = (y - x_k)/h_k the interpolant of values v is sum_p P[k][p][m] v_m t^p.
// sig_out (optional) receives the second-derivative map Sig[i][m] = d s_i / d v_m.
std::vector<double> spline_map(const std::vector<double>& x, std::vector<double>* sig_out = nullptr) {
  const int n = static_cast<int>(x.size());
  std::vector<double> h(n - 1);
  for (int k = 0; k < n - 1; ++k) h[k] = x[k + 1] - x[k];
  // system for second derivatives s (n unknowns), RHS = R v (n x n)
  std::vector<double> A(n * n, 0.0), R(n * n, 0.0);
  // not-a-knot at the left: (s1 - s0)/h0 = (s2 - s1)/h1
  A[0 * n + 0] = -h[1];
  A[0 * n + 1] = h[0] + h[1];
  A[0 * n + 2] = -h[0];
  for (int k = 1; k < n - 1; ++k) {
    A[k * n + k - 1] = h[k - 1];
    A[k * n + k] = 2.0 * (h[k - 1] + h[k]);
    A[k * n + k + 1] = h[k];
    R[k * n + k + 1] += 6.0 / h[k];
    R[k * n + k] += -6.0 / h[k] - 6.0 / h[k - 1];
    R[k * n + k - 1] += 6.0 / h[k - 1];
  }
  A[(n - 1) * n + n - 3] = -h[n - 2];
  A[(n - 1) * n + n - 2] = h[n - 3] + h[n - 2];
  A[(n - 1) * n + n - 1] = -h[n - 3];
  // solve A S = R by Gaussian elimination with partial pivoting.  A is banded
  // (tridiagonal plus the two not-a-knot rows), so each row operation only
  // runs to the pivot row's last nonzero column: the skipped terms are exact
  // zeros, the result is the same as the dense elimination.
  std::vector<double> S = R;
  std::vector<double> M = A;
  auto last_nz = [&](int r) {
    int k = n - 1;
    while (k > 0 && M[r * n + k] == 0.0) --k;
    return k;
  };
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[c * n + k], M[piv * n + k]);
        std::swap(S[c * n + k], S[piv * n + k]);
      }
    const int hi = last_nz(c);
    for (int r = c + 1; r < n; ++r) {
      double f = M[r * n + c] / M[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k <= hi; ++k) M[r * n + k] -= f * M[c * n + k];
      for (int k = 0; k < n; ++k) S[r * n + k] -= f * S[c * n + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    const int hi = last_nz(c);
    for (int k = 0; k < n; ++k) {
      double v = S[c * n + k];
      for (int j = c + 1; j <= hi; ++j) v -= M[c * n + j] * S[j * n + k];
      S[c * n + k] = v / M[c * n + c];
    }
  }
  if (sig_out) *sig_out = S;
  // S[i][m] = d s_i / d v_m.  Coefficients in t:
  //   c0 = v_k, c1 = v_{k+1} - v_k - h^2 (2 s_k + s_{k+1})/6, c2 = h^2 s_k/2, c3 = h^2 (s_{k+1} - s_k)/6
  std::vector<double> P((n - 1) * 4 * n, 0.0);
  for (int k = 0; k < n - 1; ++k) {
    const double h2 = h[k] * h[k];
    for (int m = 0; m < n; ++m) {
      const double sk = S[k * n + m], sk1 = S[(k + 1) * n + m];
      const double vk = (m == k) ? 1.0 : 0.0, vk1 = (m == k + 1) ? 1.0 : 0.0;
      P[(k * 4 + 0) * n + m] = vk;
      P[(k * 4 + 1) * n + m] = vk1 - vk - h2 * (2.0 * sk + sk1) / 6.0;
      P[(k * 4 + 2) * n + m] = 0.5 * h2 * sk;
      P[(k * 4 + 3) * n + m] = h2 * (sk1 - sk) / 6.0;
    }
  }
  return P;
}

}  // namespace

void gauss_legendre_unit(int n, std::vector<double>& t, std::vector<double>& w) { gauss_legendre01(n, t, w); }

// Angular grid (double Gauss-Legendre mu x trapezoidal chi, Sect. 4.2), the
// distinct scattering angles, the (incoming direction, Theta) slots, the pair
// lists per slot and the slot groups of the fused Sigma kernel.
static void angular_setup(Problem& P, std::vector<double>& dirs, std::vector<double>& ea,
                          std::vector<double>& eb) {
  const int nd = P.nd;
  const bool aa = P.prd_mode == TRAP_PRD_AA;
  std::vector<double> gt, gw;
  gauss_legendre01(P.nmu / 2, gt, gw);
  std::vector<double> mu1, wmu1;
  for (int i = P.nmu / 2 - 1; i >= 0; --i) {
    mu1.push_back(-gt[i]);
    wmu1.push_back(gw[i]);
  }
  for (int i = 0; i < P.nmu / 2; ++i) {
    mu1.push_back(gt[i]);
    wmu1.push_back(gw[i]);
  }
  // off-grid lines of sight: rings of zero weight after the quadrature
  for (double m : P.los_mu) {
    mu1.push_back(m);
    wmu1.push_back(0.0);
  }
  P.mu.resize(nd);
  P.w.resize(nd);
  dirs.assign(3 * nd, 0.0);
  ea.assign(3 * nd, 0.0);
  eb.assign(3 * nd, 0.0);
  for (int i = 0; i < P.nmu + P.nlos; ++i)
    for (int k = 0; k < P.nchi; ++k) {
      const int o = i * P.nchi + k;
      const double chi = 2.0 * kPi * k / P.nchi, mu = mu1[i], st = std::sqrt(1.0 - mu * mu);
      P.mu[o] = mu;
      P.w[o] = wmu1[i] / (2.0 * P.nchi);
      dirs[3 * o + 0] = st * std::cos(chi);
      dirs[3 * o + 1] = st * std::sin(chi);
      dirs[3 * o + 2] = mu;
      ea[3 * o + 0] = -std::sin(chi);
      ea[3 * o + 1] = std::cos(chi);
      ea[3 * o + 2] = 0.0;
      // e_b = Omega x e_a
      eb[3 * o + 0] = dirs[3 * o + 1] * ea[3 * o + 2] - dirs[3 * o + 2] * ea[3 * o + 1];
      eb[3 * o + 1] = dirs[3 * o + 2] * ea[3 * o + 0] - dirs[3 * o + 0] * ea[3 * o + 2];
      eb[3 * o + 2] = dirs[3 * o + 0] * ea[3 * o + 1] - dirs[3 * o + 1] * ea[3 * o + 0];
    }
  // ---- scattering-angle table and slots
  std::vector<double> cosv(nd * nd);
  for (int o = 0; o < nd; ++o)
    for (int i = 0; i < nd; ++i) {
      double c = dirs[3 * o] * dirs[3 * i] + dirs[3 * o + 1] * dirs[3 * i + 1] + dirs[3 * o + 2] * dirs[3 * i + 2];
      c = std::min(1.0, std::max(-1.0, c));
      if (std::fabs(c - 1.0) < 1e-12) c = 1.0;
      if (std::fabs(c + 1.0) < 1e-12) c = -1.0;
      cosv[o * nd + i] = c;
    }
  std::vector<double> sorted(cosv);
  std::sort(sorted.begin(), sorted.end(), std::greater<double>());
  std::vector<double> reps{sorted[0]};
  for (size_t k = 1; k < sorted.size(); ++k)
    if (reps.back() - sorted[k] > 1e-10) reps.push_back(sorted[k]);
  // angle-averaged PRD (Sect. 5.2, Eq. R_AA): one kernel for every pair, so a
  // single "angle" class holds every incoming direction as a slot; its kernel
  // is the average of the rows at the 25 Gauss-Legendre angles of App. C
  if (aa) reps.assign(1, 1.0);
  P.nth = static_cast<int>(reps.size());
  P.theta.resize(P.nth);
  for (int t = 0; t < P.nth; ++t) {
    P.theta[t] = (reps[t] == 1.0) ? 0.0 : (reps[t] == -1.0 ? kPi : std::acos(reps[t]));
  }
  P.pair_theta.resize(nd * nd);
  for (int k = 0; k < nd * nd; ++k) {
    int best = 0;
    for (int t = 1; t < P.nth; ++t)
      if (std::fabs(reps[t] - cosv[k]) < std::fabs(reps[best] - cosv[k])) best = t;
    P.pair_theta[k] = best;
  }
  if (aa) {
    std::vector<double> gt, gw;
    gauss_legendre01(25, gt, gw);
    P.theta_rows.resize(25);
    P.theta_rw.resize(25);
    for (int g = 0; g < 25; ++g) {
      P.theta_rows[g] = kPi * gt[g];
      P.theta_rw[g] = kPi * gw[g] * 0.5 * std::sin(P.theta_rows[g]);
    }
  } else {
    P.theta_rows = P.theta;
    P.theta_rw.clear();
  }
  P.nth_rows = static_cast<int>(P.theta_rows.size());
  // slots: for each theta the incoming directions that occur with it
  std::vector<std::vector<int>> used(P.nth, std::vector<int>(nd, -1));
  for (int o = 0; o < nd; ++o)
    for (int i = 0; i < nd; ++i) used[P.pair_theta[o * nd + i]][i] = 1;
  P.slot_off.assign(P.nth + 1, 0);
  P.slot_dir.clear();
  P.slot_theta.clear();
  for (int t = 0; t < P.nth; ++t) {
    P.slot_off[t] = static_cast<int>(P.slot_dir.size());
    for (int i = 0; i < nd; ++i)
      if (used[t][i] == 1) {
        used[t][i] = static_cast<int>(P.slot_dir.size());
        P.slot_dir.push_back(i);
        P.slot_theta.push_back(t);
      }
    P.max_slots_per_theta = std::max(P.max_slots_per_theta,
                                     static_cast<int>(P.slot_dir.size()) - P.slot_off[t]);
  }
  P.slot_off[P.nth] = static_cast<int>(P.slot_dir.size());
  P.nslot = static_cast<int>(P.slot_dir.size());
  P.pair_slot.resize(nd * nd);
  for (int o = 0; o < nd; ++o)
    for (int i = 0; i < nd; ++i) P.pair_slot[o * nd + i] = used[P.pair_theta[o * nd + i]][i];
  // pairs (o, o') listed per slot (slot-major), and slot groups per theta for the fused kernel
  P.pair_off.assign(P.nslot + 1, 0);
  for (int k = 0; k < nd * nd; ++k) ++P.pair_off[P.pair_slot[k] + 1];
  for (int sl = 0; sl < P.nslot; ++sl) P.pair_off[sl + 1] += P.pair_off[sl];
  P.pair_o.assign(nd * nd, 0);
  {
    std::vector<int> fill(P.pair_off.begin(), P.pair_off.end() - 1);
    for (int o = 0; o < nd; ++o)
      for (int i = 0; i < nd; ++i) P.pair_o[fill[P.pair_slot[o * nd + i]]++] = o;
  }
  P.pair_dir.assign(nd * nd, 0);
  for (int sl = 0; sl < P.nslot; ++sl)
    for (int q = P.pair_off[sl]; q < P.pair_off[sl + 1]; ++q) P.pair_dir[q] = P.slot_dir[sl];
  P.pair_index.assign(nd * nd, 0);
  for (int q = 0; q < nd * nd; ++q) P.pair_index[P.pair_o[q] * nd + P.pair_dir[q]] = q;
  // contraction column groups: the slots of one theta in groups of at most 32
  // (FP32) or 16 (FP64); FP32 groups are split into two classes by size so
  // each class runs with its own number of column tiles
  for (int pi = 0; pi < 2; ++pi) {
    const int cg = pi == 0 ? 16 : 32;
    std::vector<int> wide, narrow;
    for (int t = 0; t < P.nth; ++t)
      for (int s0 = P.slot_off[t]; s0 < P.slot_off[t + 1]; s0 += cg) {
        const int cnt = std::min(cg, P.slot_off[t + 1] - s0);
        auto& dst = cnt > 16 ? wide : narrow;
        dst.push_back(t);
        dst.push_back(s0);
        dst.push_back(cnt);
      }
    P.cgrp_n8[pi] = static_cast<int>(wide.size() / 3);
    P.cgrp[pi] = wide;
    P.cgrp[pi].insert(P.cgrp[pi].end(), narrow.begin(), narrow.end());
  }

  // a group holds at most sg slots of one theta and at most 2 sg pairs
  for (int pi = 0; pi < 2; ++pi) {
    const int sg = pi == 0 ? 8 : 16;
    P.grp[pi].clear();
    P.grp_maxpairs[pi] = 0;
    for (int t = 0; t < P.nth; ++t) {
      int s0 = P.slot_off[t];
      while (s0 < P.slot_off[t + 1]) {
        int cnt = 0;
        while (s0 + cnt < P.slot_off[t + 1] && cnt < sg &&
               P.pair_off[s0 + cnt + 1] - P.pair_off[s0] <= 2 * sg)
          ++cnt;
        cnt = std::max(cnt, 1);
        P.grp_maxpairs[pi] = std::max(P.grp_maxpairs[pi], P.pair_off[s0 + cnt] - P.pair_off[s0]);
        P.grp[pi].push_back(t);
        P.grp[pi].push_back(s0);
        P.grp[pi].push_back(cnt);
        s0 += cnt;
      }
    }
  }
}

PrecompLayout precomp_layout(int nz, int nn, int ldm, int nt, int nthr, bool aa, const double* x,
                             const double* lam) {
  PrecompLayout L;
  L.h = (x[nn - 1] - x[0]) / (nn - 1);
  L.uniform = true;
  for (int k = 0; k + 1 < nn; ++k)
    if (std::fabs(x[k + 1] - x[k] - L.h) > 1e-12 * std::fabs(L.h)) L.uniform = false;
  // the widest kernel support has half-width 6.6 * 2 sin(Theta/2) / lam <= 13.2 / lam
  if (L.uniform) {
    double lmin = lam[0];
    for (int z = 1; z < nz; ++z) lmin = std::min(lmin, lam[z]);
    L.ntail = (int)std::min<double>(std::ceil(13.2 / (lmin * L.h)) + 2.0, 8.0 * nn);
  }
  L.nd2 = 2 * nn - 1 + 2 * L.ntail;
  const size_t tab_per_z = (size_t)nthr * L.nd2 * 16 * (sizeof(double) + nt * 2 * sizeof(double));
  const size_t rows_per_z = (size_t)nthr * nt * 2 * nn;
  const size_t lg_per_z = rows_per_z * ldm * sizeof(double) * (aa ? 3 : 2);
  size_t zc_lim = std::max<size_t>(1, (size_t(1) << 30) / lg_per_z);
  if (L.uniform) zc_lim = std::min(zc_lim, std::max<size_t>(1, (size_t(192) << 20) / tab_per_z));
  L.zc_tab = (int)std::min<size_t>(nz, zc_lim);
  L.bytes = (size_t)L.zc_tab * (lg_per_z + (L.uniform ? tab_per_z : 0));
  return L;
}

// ---------------------------------------------------------------- banded kernel store
// Largest k with x[k] <= v (-1 below the grid, nn - 1 at or past its end):
// the interval search of the kernel-row precompute.
static int upper_node(const std::vector<double>& x, double v) {
  const int nn = static_cast<int>(x.size());
  if (v < x[0]) return -1;
  if (v >= x[nn - 1]) return nn - 1;
  int lo = 0, hi = nn - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// f(i0, i1) over [0, n) in contiguous ranges on up to 16 host threads (one
// when the work is small); f must only write what its range owns.
template <typename F>
static void host_parallel(size_t n, size_t min_per_thread, F f) {
  const size_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t nt = std::max<size_t>(1, std::min(hw, n / std::max<size_t>(1, min_per_thread)));
  if (nt <= 1) {
    f(size_t(0), n);
    return;
  }
  std::vector<std::thread> pool;
  pool.reserve(nt - 1);
  const size_t per = (n + nt - 1) / nt;
  for (size_t k = 1; k < nt; ++k) {
    const size_t a = std::min(n, k * per), b = std::min(n, a + per);
    pool.emplace_back([=, &f]() { f(a, b); });
  }
  f(size_t(0), std::min(n, per));
  for (auto& t : pool) t.join();
}

void kernel_bands(Problem& P, const std::vector<double>& sig) {
  const int nz = P.nz, nn = P.nn, nth = P.nth, np = 2 * P.nt;
  const bool aa = P.prd_mode == TRAP_PRD_AA;
  // reach of the spline map: column m of M = L + Gam Sig receives node j's
  // weight through Sig[j][m], which decays geometrically away from j; beyond
  // `reach` nodes every entry is below 1e-13 of its row's largest
  int reach = 0;
  for (int j = 0; j < nn; ++j) {
    double mx = 0.0;
    for (int m = 0; m < nn; ++m) mx = std::max(mx, std::fabs(sig[(size_t)j * nn + m]));
    for (int m = 0; m < nn; ++m)
      if (std::fabs(sig[(size_t)j * nn + m]) > 1e-13 * mx) reach = std::max(reach, std::abs(m - j));
  }
  P.band_reach = reach;
  // the FP32 operator keeps less: a value below about 1e-9 of its row's
  // largest is below the resolution of the FP32 sum (2^-24 ~ 6e-8), so its
  // window takes the knot intervals within kCut32 Gaussian widths
  // (exp(-4.6^2) ~ 6.5e-10) and the reach where Sig falls below 1e-9
  constexpr double kCut = 6.6, kCut32 = 4.6;
  int reach32 = 0;
  for (int j = 0; j < nn; ++j) {
    double mx = 0.0;
    for (int m = 0; m < nn; ++m) mx = std::max(mx, std::fabs(sig[(size_t)j * nn + m]));
    for (int m = 0; m < nn; ++m)
      if (std::fabs(sig[(size_t)j * nn + m]) > 1e-9 * mx) reach32 = std::max(reach32, std::abs(m - j));
  }
  reach32 = std::min(reach32, reach);
  P.band_reach32 = reach32;
  // Gaussian half-width factor of each stored angle: sin(Theta/2) (1 at
  // Theta = pi, 0 at Theta = 0: the diagonal row); the angle average takes
  // its widest node
  std::vector<double> sg(nth);
  for (int t = 0; t < nth; ++t) {
    if (aa) {
      double th = 0.0;
      for (double v : P.theta_rows) th = std::max(th, v);
      sg[t] = th >= kPi ? 1.0 : std::sin(0.5 * th);
    } else {
      const double th = P.theta[t];
      sg[t] = th == 0.0 ? 0.0 : (th >= kPi ? 1.0 : std::sin(0.5 * th));
    }
  }
  std::vector<int> nslots(nth);
  for (int t = 0; t < nth; ++t) nslots[t] = P.slot_off[t + 1] - P.slot_off[t];
  // band [lo, hi) of every row n of every (z, theta): the knot intervals within
  // 6.6 Gaussian widths 2 sin(Theta/2)/lam of x_n (what the kernel-row
  // precompute integrates), one node of margin for rounding, then the spline's
  // reach; the in-band entries are the algorithmic work
  // (every entry is written below, by the thread that owns its (z, theta):
  // no zero fill, and the first touch of each page happens in that thread)
  // (the FP32 window [blo32, bhi32) likewise, inside [blo, bhi))
  std::unique_ptr<short[]> blo(new short[(size_t)nz * nth * nn]), bhi(new short[(size_t)nz * nth * nn]);
  std::unique_ptr<short[]> blo32(new short[(size_t)nz * nth * nn]), bhi32(new short[(size_t)nz * nth * nn]);
  std::vector<long long> cnt_zt((size_t)nz * nth), cnt32_zt((size_t)nz * nth);
  const size_t nzt = (size_t)nz * nth;
  host_parallel(nzt, 64, [&](size_t zt0, size_t zt1) {
    for (size_t zt = zt0; zt < zt1; ++zt) {
      const int z = static_cast<int>(zt / nth), t = static_cast<int>(zt % nth);
      long long cnt = 0, cnt32 = 0;
      // x_n - R and x_n + R increase with n: the interval searches walk forward
      struct Walk {
        double R;
        int rch, plo = -1, phi = -1;
      } wk[2] = {{kCut * 2.0 * sg[t] / P.lam[z], reach}, {kCut32 * 2.0 * sg[t] / P.lam[z], reach32}};
      for (int n = 0; n < nn; ++n) {
        int lo[2], hi[2];
        for (int v = 0; v < 2; ++v) {
          Walk& w = wk[v];
          if (sg[t] == 0.0) {
            lo[v] = n;
            hi[v] = n + 1;
            continue;
          }
          const double xn = P.x[n], a = xn - w.R, b = xn + w.R;
          if (n == 0) {
            w.plo = upper_node(P.x, a);
            w.phi = upper_node(P.x, b);
          } else {
            while (w.plo + 1 < nn && P.x[w.plo + 1] <= a) ++w.plo;
            while (w.phi + 1 < nn && P.x[w.phi + 1] <= b) ++w.phi;
          }
          int ph = w.phi;
          if (ph >= 0 && ph < nn - 1 && P.x[ph] >= b) ph -= 1;
          const int jlo = std::max(w.plo, 0), jhi = std::min(ph + 1, nn - 1);
          lo[v] = std::max(0, jlo - 1 - w.rch);
          hi[v] = std::min(nn, jhi + 2 + w.rch);
        }
        lo[1] = std::max(lo[1], lo[0]);
        hi[1] = std::max(lo[1], std::min(hi[1], hi[0]));
        blo[zt * nn + n] = static_cast<short>(lo[0]);
        bhi[zt * nn + n] = static_cast<short>(hi[0]);
        blo32[zt * nn + n] = static_cast<short>(lo[1]);
        bhi32[zt * nn + n] = static_cast<short>(hi[1]);
        cnt += hi[0] - lo[0];
        cnt32 += hi[1] - lo[1];
      }
      cnt_zt[zt] = cnt;
      cnt32_zt[zt] = cnt32;
    }
  });
  P.kflops_z.assign(nz, 0.0);
  P.kflops32_z.assign(nz, 0.0);
  P.band_nnz = 0.0;
  P.band_nnz32 = 0.0;
  for (size_t zt = 0; zt < nzt; ++zt) {
    P.band_nnz += (double)P.nt * cnt_zt[zt];
    P.band_nnz32 += (double)P.nt * cnt32_zt[zt];
    P.kflops_z[zt / nth] += 16.0 * P.nt * (double)cnt_zt[zt] * nslots[zt % nth];
    P.kflops32_z[zt / nth] += 16.0 * P.nt * (double)cnt32_zt[zt] * nslots[zt % nth];
  }
  // wave tiles in both row layouts; the one with less column work is kept:
  // every wave of a block steps through the block's column range (the union
  // of its eight tiles' ranges), times the incoming slots of the angle
  // tiles(pad, row0, qk, qk32, work): the column work of a layout, and with
  // qk / qk32 given, every tile's range and FP32 window (the layout is first
  // chosen by its work alone, then only the chosen one is filled)
  auto tiles = [&](bool pad, std::vector<int>& row0, host_vec<unsigned>* qk, host_vec<unsigned>* qk32,
                   double* work) {
    const int nnp = pad ? (nn + 15) / 16 * 16 : nn;
    const int rows = np * nnp;
    const int nq = (rows + 15) / 16;
    row0.assign(nq, 0);
    for (int q = 0; q < nq; ++q) row0[q] = pad ? (q % np) * nnp + 16 * (q / np) : 16 * q;
    if (qk) qk->resize((size_t)nz * nth * nq);         // every entry written below
    if (qk32) qk32->resize((size_t)nz * nth * nq);
    std::vector<double> work_zt(nzt, 0.0);
    // the band ends never decrease with n, so a run of rows n_a..n_b of one
    // plane spans [lo(n_a), hi(n_b))
    host_parallel(nzt, 64, [&](size_t zt0, size_t zt1) {
      std::vector<unsigned> qz(nq);                    // this (z, theta)'s tile ranges
      for (size_t zt = zt0; zt < zt1; ++zt) {
        const short* bl = &blo[zt * nn];
        const short* bh = &bhi[zt * nn];
        const short* bl32 = &blo32[zt * nn];
        const short* bh32 = &bhi32[zt * nn];
        for (int q = 0; q < nq; ++q) {
          int lo = P.ldm, hi = 0, lo32 = P.ldm, hi32 = 0;
          const int r1 = std::min(row0[q] + 16, rows);
          for (int r = row0[q]; r < r1;) {
            const int p = r / nnp, n = r - p * nnp;
            const int run = std::min(r1 - r, nnp - n);        // rows left in this plane
            const int nb = std::min(n + run, nn) - 1;
            if (nb >= n) {
              lo = std::min(lo, (int)bl[n]);
              hi = std::max(hi, (int)bh[nb]);
              lo32 = std::min(lo32, (int)bl32[n]);
              hi32 = std::max(hi32, (int)bh32[nb]);
            }
            r += run;
          }
          if (hi <= lo) lo = hi = 0;
          lo = lo / 8 * 8;
          hi = std::min((hi + 7) / 8 * 8, P.ldm);
          qz[q] = (unsigned)lo | ((unsigned)hi << 16);
          if (qk) (*qk)[zt * nq + q] = qz[q];
          if (qk32) {
            // inside the tile's range (rounded the same way)
            lo32 = std::max(lo, lo32 / 8 * 8);
            hi32 = std::min(hi, (hi32 + 7) / 8 * 8);
            if (hi32 <= lo32) lo32 = hi32 = lo;
            (*qk32)[zt * nq + q] = (unsigned)lo32 | ((unsigned)hi32 << 16);
          }
        }
        for (int q0 = 0; q0 < nq; q0 += 8) {
          int lo = P.ldm, hi = 0;
          for (int q = q0; q < std::min(q0 + 8, nq); ++q) {
            const unsigned v = qz[q];
            if ((v >> 16) > (v & 0xffffu)) {
              lo = std::min(lo, (int)(v & 0xffffu));
              hi = std::max(hi, (int)(v >> 16));
            }
          }
          if (hi > lo) work_zt[zt] += 8.0 * (hi - lo) * nslots[zt % nth];
        }
      }
    });
    *work = 0.0;
    for (double w : work_zt) *work += w;
    return nnp;
  };
  std::vector<int> r0a, r0b;
  double wa = 0.0, wb = 0.0;
  const int nnpa = tiles(false, r0a, nullptr, nullptr, &wa);
  const int nnpb = tiles(true, r0b, nullptr, nullptr, &wb);
  const bool pad = wb < wa;
  P.qpad = pad ? 1 : 0;
  P.nnp = pad ? nnpb : nnpa;
  double wsel = 0.0;
  tiles(pad, pad ? r0b : r0a, &P.qk, &P.qk32, &wsel);
  P.qrow0 = std::move(pad ? r0b : r0a);
  P.nq = static_cast<int>(P.qrow0.size());
  P.nqb = (P.nq + 7) / 8;
  // tile offsets: tiles of (z, theta) back to back in block order, each
  // [16][hi - lo]
  // (all four are written in full below)
  P.tofs.resize((size_t)nz * nth * P.nq);
  P.td.resize((size_t)nz * nth * P.nq);
  P.kbase.resize((size_t)nz * nth);
  P.qb.resize((size_t)nz * nth * P.nqb);
  P.qb32.resize((size_t)nz * nth * P.nqb);
  std::vector<long long> ent32_zt(nzt);
  // per (z, theta): tile offsets and size, then the running base, then the
  // descriptors and block ranges
  std::vector<long long> size_zt(nzt);
  host_parallel(nzt, 256, [&](size_t zt0, size_t zt1) {
    for (size_t zt = zt0; zt < zt1; ++zt) {
      int off = 0;
      for (int q = 0; q < P.nq; ++q) {
        const unsigned v = P.qk[zt * P.nq + q];
        P.tofs[zt * P.nq + q] = off;
        off += 16 * (int)((v >> 16) - (v & 0xffffu));
      }
      size_zt[zt] = off;
    }
  });
  long long total = 0;
  for (size_t zt = 0; zt < nzt; ++zt) {
    P.kbase[zt] = total;
    total += size_zt[zt];
  }
  host_parallel(nzt, 256, [&](size_t zt0, size_t zt1) {
    for (size_t zt = zt0; zt < zt1; ++zt) {
      for (int q = 0; q < P.nq; ++q) {
        const unsigned v = P.qk[zt * P.nq + q];
        P.td[zt * P.nq + q] = TileDesc{P.kbase[zt] + P.tofs[zt * P.nq + q], (int)(v & 0xffffu), (int)(v >> 16)};
      }
      for (int bq = 0; bq < P.nqb; ++bq) {
        unsigned lo = 0xffffu, hi = 0;
        for (int q = 8 * bq; q < std::min(8 * bq + 8, P.nq); ++q) {
          const unsigned v = P.qk[zt * P.nq + q];
          if ((v >> 16) > (v & 0xffffu)) {
            lo = std::min(lo, v & 0xffffu);
            hi = std::max(hi, v >> 16);
          }
        }
        if (hi <= lo) lo = hi = 0;
        P.qb[zt * P.nqb + bq] = lo | (hi << 16);
        unsigned lo32 = 0xffffu, hi32 = 0;
        for (int q = 8 * bq; q < std::min(8 * bq + 8, P.nq); ++q) {
          const unsigned v = P.qk32[zt * P.nq + q];
          if ((v >> 16) > (v & 0xffffu)) {
            lo32 = std::min(lo32, v & 0xffffu);
            hi32 = std::max(hi32, v >> 16);
          }
        }
        if (hi32 <= lo32) lo32 = hi32 = 0;
        P.qb32[zt * P.nqb + bq] = lo32 | (hi32 << 16);
      }
      long long e32 = 0;
      for (int q = 0; q < P.nq; ++q) {
        const unsigned v = P.qk32[zt * P.nq + q];
        e32 += 16LL * (int)((v >> 16) - (v & 0xffffu));
      }
      ent32_zt[zt] = e32;
    }
  });
  P.kentries = (size_t)total;
  P.kent32_z.assign(nz, 0.0);
  for (size_t zt = 0; zt < nzt; ++zt) P.kent32_z[zt / nth] += (double)ent32_zt[zt];
  {
    // FP32 column groups by decreasing matrix-core work (window entries of the
    // theta over all heights x column tiles): the resident-field contraction
    // hands its work units out in this order
    std::vector<double> eth(nth, 0.0);
    for (size_t zt = 0; zt < nzt; ++zt) eth[zt % nth] += (double)ent32_zt[zt];
    const int ng = (int)P.cgrp[1].size() / 3;
    std::vector<double> wg(ng);
    P.cord.resize(ng);
    for (int g = 0; g < ng; ++g) {
      P.cord[g] = g;
      wg[g] = eth[P.cgrp[1][3 * g]] * (g < P.cgrp_n8[1] ? 8 : 4);
    }
    std::stable_sort(P.cord.begin(), P.cord.end(), [&](int a, int b) { return wg[a] > wg[b]; });
    P.unit_ctr.assign(2, 0);
    const int ng0 = (int)P.cgrp[0].size() / 3;
    P.cord0.resize(ng0);
    for (int g = 0; g < ng0; ++g) P.cord0[g] = g;
    std::stable_sort(P.cord0.begin(), P.cord0.end(),
                     [&](int a, int b) { return eth[P.cgrp[0][3 * a]] > eth[P.cgrp[0][3 * b]]; });
  }
}

static int zero_field_classes(const trap_atom_desc& at, double dnuD_ref, std::vector<double>* dE,
                              std::vector<int>* cls);

// Direction counts: the n_mu x n_chi quadrature plus the zero-weight
// line-of-sight rings.  Returns an error message, or nullptr.
static const char* set_directions(Problem& P, const trap_problem_desc* pd) {
  if (pd->n_los < 0 || pd->n_los > 16) return "n_los must lie in [0, 16]";
  if (pd->n_los > 0 && !pd->los_mu) return "los_mu is NULL";
  P.nmu = pd->n_mu;
  P.nchi = pd->n_chi;
  P.nlos = pd->n_los;
  P.los_mu.assign(pd->los_mu, pd->los_mu + pd->n_los);
  for (double m : P.los_mu)
    if (!(m > 0.0 && m <= 1.0)) return "line-of-sight mu must lie in (0, 1]";
  P.ngrid = P.nmu * P.nchi;
  P.nd = (P.nmu + P.nlos) * P.nchi;
  return nullptr;
}

size_t estimate_bytes(const trap_atom_desc* atom, const trap_problem_desc* pd, int store_mask, int* err) {
  *err = 0;
  if (!atom || !pd || pd->n_z < 2 || pd->n_nu < 4 || pd->n_mu < 2 || pd->n_mu % 2 || pd->n_chi < 1 ||
      (atom->kind != 0 && atom->kind != 1) || !pd->x || !pd->T || !(atom->mass_amu > 0)) {
    *err = 1;
    return 0;
  }
  Problem P;
  P.nz = pd->n_z;
  P.nn = pd->n_nu;
  if (set_directions(P, pd)) {
    *err = 1;
    return 0;
  }
  P.ldm = (P.nn + 7) / 8 * 8;
  std::vector<double> dirs, ea, eb;
  angular_setup(P, dirs, ea, eb);
  size_t nu, nl;
  if (atom->kind == 0) {
    nu = static_cast<size_t>(std::lround(2 * atom->J_u)) + 1;
    nl = static_cast<size_t>(std::lround(2 * atom->J_l)) + 1;
  } else {
    nu = (2 * atom->L_u + 1) * static_cast<size_t>(std::lround(2 * atom->S) + 1);
    nl = (2 * atom->L_l + 1) * static_cast<size_t>(std::lround(2 * atom->S) + 1);
  }
  const size_t nt = nu * nl;
  const size_t nz = P.nz, nn = P.nn, nd = P.nd, nth = P.nth, nslot = P.nslot, ldm = P.ldm;
  const size_t N = 4 * nz * nd * nn;
  const int mask = store_mask | 1;
  // the banded kernel store: bands from the grids and the Doppler widths
  std::vector<double> lam_b(nz);
  {
    const double mass = atom->mass_amu * kAMU;
    const double Tref = pd->T_ref > 0 ? pd->T_ref : 6000.0;
    const double vref = std::sqrt(2.0 * kKB * Tref / mass);
    for (size_t z = 0; z < nz; ++z) {
      const double xi = pd->xi ? pd->xi[z] * 1e5 : 0.0;
      lam_b[z] = vref / std::sqrt(2.0 * kKB * pd->T[z] / mass + xi * xi);
    }
    P.x.assign(pd->x, pd->x + nn);
    for (size_t k = 0; k + 1 < nn; ++k)
      if (!(P.x[k + 1] > P.x[k])) {
        *err = 1;
        return 0;
      }
    P.lam = lam_b;
    P.nt = static_cast<int>(nt);
    std::vector<double> sig;
    spline_map(P.x, &sig);
    kernel_bands(P, sig);
  }
  const size_t cfe = nz * nd * nd * nt * 2 * nl * 16;    // angular coefficients per precision
  size_t b = 0;
  auto add = [&b](size_t bytes) { b += bytes ? bytes : 16; };   // one allocation
  auto add_vec = [&add](const auto& v) { add(v.size() * sizeof(v[0])); };
  add(P.kentries * 4);                                  // kernel values (FP32)
  add(P.kentries * 4);                                  //   and remainders
  for (int pi = 0; pi < 2; ++pi) {
    if (!(mask & (1 << pi))) continue;
    const size_t es = pi == 0 ? 8 : 4;
    add(cfe * es);
    for (int k = 0; k < 3; ++k) add(N * es);           // comoving field, two work vectors
    add(nz * nl * nl * nd * nn * 4 * es);               // eps_bar
  }
  // precompute outputs: K, eps_th, f, b; R_III weights and profiles
  add(nz * nd * nn * 8 * 8);
  add(nz * nd * nn * 4 * 8);
  add(nz * nd * nn * 8);
  add(nz * nd * nn * 4 * 8);
  add(nz * nt * nn * 16);
  add(nz * nt * nn * 16);
  // solver: Krylov basis (restart <= 40), r, x, scratch, reductions, FP32 vectors
  add(N * 8 * 41);
  for (int k = 0; k < 3; ++k) add(N * 8);
  add(nz * nt * nd * 4 * 16);                           // R_III factors Y, X
  add(nz * nu * nu * nl * 16);
  add(4096 * 8);
  add((1024 * 42 + 2 * 42) * 8);                       // reduction scratch (1024 blocks)
  add(N * 4);
  add(N * 4);
  // problem tables: one batch (grid and spline maps, per-height scalars,
  // angular tables, sublevel shifts, branching ratios, dipole tables) in the
  // order and alignment of build_problem's upload
  {
    UploadBatch up;
    auto item = [&up](size_t bytes) { up.add(nullptr, nullptr, bytes); };
    auto item_vec = [&item](const auto& v) { item(v.size() * sizeof(v[0])); };
    item(nn * 8);
    item((nn - 1) * 4 * nn * 8);
    item(nn * nn * 8);
    item(nn * nn * 8);
    for (int k = 0; k < 2; ++k) item(nd * 8);            // mu, w
    for (int k = 0; k < 6; ++k) item(nz * 8);            // tau, lam, a, eps, W_T, eta0
    item(nz * nd * 8);                                   // u_b
    item(nz * nt * 8);                                   // transition shifts
    item(nz * nl * nl * 8);                              // lower-level shifts
    item_vec(P.theta);
    item_vec(P.theta_rows);
    item_vec(P.theta_rw);
    item_vec(P.slot_theta);
    item_vec(P.slot_dir);
    item_vec(P.slot_off);
    item_vec(P.pair_slot);
    item_vec(P.pair_theta);
    item_vec(P.pair_off);
    item_vec(P.pair_o);
    item_vec(P.pair_dir);
    item_vec(P.pair_index);
    item_vec(P.grp[0]);
    item_vec(P.grp[1]);
    item_vec(P.cgrp[0]);
    item_vec(P.cgrp[1]);
    item_vec(P.cord);
    item_vec(P.unit_ctr);
    item_vec(P.cord0);
    item(nz * nd * 4 * nu * nu * nl * 16);               // E
    item(nz * nd * 4 * nu * nu * nl * 16);               // A
    item(nz * nu * nu * 16);                             // alpha
    item(nz * nu * nu * 16);                             // beta - alpha
    item(nz * nt * nd * 4 * 8);                          // g
    item_vec(P.td);                                      // banded store layout
    item_vec(P.qb);
    item_vec(P.qk32);                                    //   and the FP32 windows
    item_vec(P.qb32);
    if (pd->kappa_c || pd->sigma_c) {
      item(nz * nn * 8);                                 // kappa_c
      item(nz * nn * 8);                                 // sigma_c
      item(nd * 3 * 8);                                  // polarisation axes e_a
      item(nd * 3 * 8);                                  //   and e_b
    }
    add(up.total);
  }
  // precompute scratch (factor tables, row stores of one height chunk)
  {
    const double mass = atom->mass_amu * kAMU;
    const double Tref = pd->T_ref > 0 ? pd->T_ref : 6000.0;
    const double vref = std::sqrt(2.0 * kKB * Tref / mass);
    std::vector<double> lam(nz);
    for (size_t z = 0; z < nz; ++z) {
      const double xi = pd->xi ? pd->xi[z] * 1e5 : 0.0;
      lam[z] = vref / std::sqrt(2.0 * kKB * pd->T[z] / mass + xi * xi);
    }
    const PrecompLayout lay =
        precomp_layout((int)nz, (int)nn, (int)ldm, (int)nt, P.nth_rows, false, pd->x, lam.data());
    const size_t rows = (size_t)lay.zc_tab * P.nth_rows * nt * 2 * nn * ldm * 8;
    add(rows);                                          // L and Gamma row stores
    add(rows);
    add((size_t)lay.zc_tab * P.nth_rows * nt * nn * 8);  // node spans of the Gamma rows (int2 each)
    if (lay.uniform) {
      add((size_t)lay.zc_tab * P.nth_rows * lay.nd2 * 16 * 8);        // Gaussian factors
      add((size_t)lay.zc_tab * P.nth_rows * nt * lay.nd2 * 16 * 16);  // Faddeeva factors
    }
  }
  // the preconditioner (store_mask bit 2): its table upload, tables, kernel
  // scratch and sweep vectors, as run_precompute_precond and precond_apply
  // allocate them
  if (store_mask & 4) {
    const double mass = atom->mass_amu * kAMU;
    const double Tref = pd->T_ref > 0 ? pd->T_ref : 6000.0;
    const double nu0 = kC / (atom->lambda0_A * 1e-8);
    const double vref = std::sqrt(2.0 * kKB * Tref / mass);
    std::vector<double> lam(nz);
    for (size_t z = 0; z < nz; ++z) {
      const double xi = pd->xi ? pd->xi[z] * 1e5 : 0.0;
      lam[z] = vref / std::sqrt(2.0 * kKB * pd->T[z] / mass + xi * xi);
    }
    const size_t nk = (size_t)zero_field_classes(*atom, nu0 * vref / kC, nullptr, nullptr);
    const size_t ng = 25;
    UploadBatch up;
    auto item = [&up](size_t bytes) { up.add(nullptr, nullptr, bytes); };
    item(nz * nk * 8);                                   // class shifts
    item(nz * nk * 8);                                   // R_II weights (real plane)
    item(nz * nk * 8);                                   //   (imaginary plane)
    item(nz * 4 * nk * nk * 16);                         // R_III weights
    item(nz * nd * 4);                                   // directions by class
    item(nz * (nd + 1) * 4);                             // class offsets
    item(nz * 4);                                        // class counts
    item(nz * nd * 8);                                   // class shifts
    item(ng * 8);                                        // angles
    item(ng * 8);                                        // weights
    add(up.total);
    add(nz * nn * nn * 8);                               // Phi
    add(nz * nn * nn * 8);                               // C
    add(nz * nd * nn * 8);                               // local Lambda
    add(nz * nd * nn * 16);                              // scalar step coefficients
    add(nz * nn * nn * 3 * 8);                           // A and the elimination scratch
    add(nz * nk * 2 * nn * ldm * 8);                     // class kernels
    add(nz * nk * nn * 16);                              // R_III rows
    add(nz * nk * nn * 16);                              // profiles
    const PrecompLayout lay = precomp_layout((int)nz, (int)nn, (int)ldm, (int)nk, (int)ng, true, pd->x, lam.data());
    const size_t rows_per_z = ng * nk * 2 * nn;
    const size_t zc = std::max<size_t>(1, std::min<size_t>(nz, (size_t(32) << 20) / (rows_per_z * ldm * 8)));
    if (lay.uniform) {
      add(zc * ng * lay.nd2 * 16 * 8);
      add(zc * ng * nk * lay.nd2 * 16 * 16);
    }
    for (int k = 0; k < 3; ++k) add(zc * rows_per_z * ldm * 8);
    for (int k = 0; k < 3; ++k) add(nz * nd * nn * 8);  // sweep vectors
    add(nz * 2 * nn * 8);
    // per-class comoving sums: Doppler-shift classes per height as build_problem forms them
    int ncmax = 1;
    for (size_t z = 0; z < nz; ++z) {
      const double xi = pd->xi ? pd->xi[z] * 1e5 : 0.0;
      const double vth = std::sqrt(2.0 * kKB * pd->T[z] / mass + xi * xi);
      std::vector<double> cub;
      for (size_t o = 0; o < nd && pd->v; ++o) {
        const double vdot = pd->v[3 * z] * dirs[3 * o] + pd->v[3 * z + 1] * dirs[3 * o + 1] +
                            pd->v[3 * z + 2] * dirs[3 * o + 2];
        const double v = vdot * 1e5 / vth;
        if (std::find(cub.begin(), cub.end(), v) == cub.end()) cub.push_back(v);
      }
      ncmax = std::max(ncmax, (int)cub.size());
    }
    add(nz * (size_t)ncmax * nn * 8);
  }
  // the height-chunked Sigma path materialises W for one chunk of heights
  // (at most ~512 MiB in FP64, half that in FP32)
  {
    const size_t per_z = nt * nslot * 2 * (size_t)w_stride((int)nn) * 4;
    const size_t zc = std::max<size_t>(1, std::min<size_t>(nz, (size_t(1) << 29) / std::max<size_t>(per_z * 8, 1)));
    add(zc * per_z * 8);
    if (mask & 2) add(zc * per_z * 4);
  }
  return b;
}

// Transitions of the zero-field atom grouped by frequency: class energy
// differences (Hz) and the class of each transition (u, l) at u nl + l; the
// class count is returned.
static int zero_field_classes(const trap_atom_desc& at, double dnuD_ref, std::vector<double>* dE,
                              std::vector<int>* cls) {
  const Sublevels s0 = sublevels(at, 0.0, 0.0, 0.0, dnuD_ref);
  const int nu = static_cast<int>(s0.Eu.size()), nl = static_cast<int>(s0.El.size());
  std::vector<double> e_k;
  if (cls) cls->assign((size_t)nu * nl, 0);
  for (int u = 0; u < nu; ++u)
    for (int l = 0; l < nl; ++l) {
      const double e = s0.Eu[u] - s0.El[l];
      int k = 0;
      while (k < (int)e_k.size() && std::fabs(e_k[k] - e) > 1e-9 * std::max(1.0, std::fabs(e))) ++k;
      if (k == (int)e_k.size()) e_k.push_back(e);
      if (cls) (*cls)[(size_t)u * nl + l] = k;
    }
  if (dE) *dE = e_k;
  return static_cast<int>(e_k.size());
}

// Weights of the preconditioner's comoving coupling (Sect. 5.2, App. F): the
// comoving Stokes-I emissivity of the zero-field atom for an isotropic,
// unpolarised comoving field J (K = Q = 0).  With the angle-averaged kernels
// M_k and R_III rows R_k / profiles P_k of the zero-field transition classes k,
//   Phi J = sum_k (cr_k Re M_k + ci_k Im M_k) J
//         + sum_{a,b} Re[X1 P_a (R_b.J) + X2 conj(P_a) (R_b.J) + X3 P_a (conj R_b.J) + X4 conj(P_a) (conj R_b.J)].
// They follow from the scattering sums of Sigma (App. D) with the incoming
// factor summed over directions, which an isotropic field allows; the total
// is then the same for every outgoing direction, so direction 0 is used.
static void precond_weights(Problem& P, const trap_atom_desc& at, double dnuD_ref, const std::vector<double>& ea,
                            const std::vector<double>& eb, const std::vector<double>& ub, double rE) {
  const int nz = P.nz, nd = P.nd;
  const Sublevels s0 = sublevels(at, 0.0, 0.0, 0.0, dnuD_ref);
  const int nu = static_cast<int>(s0.Eu.size()), nl = static_cast<int>(s0.El.size()), nt = nu * nl;
  std::vector<int> cls(nt);
  const int nk = P.pc_nk = zero_field_classes(at, dnuD_ref, &P.pc_dE, &cls);
  // incoming factor summed over directions, SA[q][p][l] = sum_x w_x d_ql^T Acart_0(x)/2 d_pl^*,
  // and the outgoing factor of direction 0, E0[p][q][l'] = d_pl'^T Acart_0(0) d_ql'^*
  std::vector<cd> SA((size_t)nu * nu * nl, cd(0, 0)), E0((size_t)nu * nu * nl);
  std::vector<cd> pa(nt), pb(nt);
  for (int o = 0; o < nd; ++o) {
    for (int t = 0; t < nt; ++t) stokes_proj(&s0.d[t * 3], &ea[3 * o], &eb[3 * o], &pa[t], &pb[t]);
    for (int q = 0; q < nu; ++q)
      for (int p = 0; p < nu; ++p)
        for (int l = 0; l < nl; ++l) {
          const int tq = q * nl + l, tp = p * nl + l;
          SA[((size_t)q * nu + p) * nl + l] +=
              P.w[o] * 0.5 * stokes_pair(0, pa[tq], pb[tq], std::conj(pa[tp]), std::conj(pb[tp]));
          if (o == 0) E0[((size_t)p * nu + q) * nl + l] = stokes_pair(0, pa[tp], pb[tp], std::conj(pa[tq]), std::conj(pb[tq]));
        }
  }
  P.pc_cr.assign((size_t)nz * nk, 0.0);
  P.pc_ci.assign((size_t)nz * nk, 0.0);
  P.pc_X.assign((size_t)nz * 4 * nk * nk, make_double2(0.0, 0.0));
  for (int z = 0; z < nz; ++z) {
    const double gtot = 4.0 * kPi * P.a[z] * P.dnuD[z];
    const double gri = gtot / (1.0 + rE);
    const double gr = (1.0 - P.eps[z]) * gri;
    std::vector<cd> X(4 * nk * nk, cd(0, 0));
    for (int l = 0; l < nl; ++l)
      for (int lp = 0; lp < nl; ++lp)
        for (int q = 0; q < nu; ++q)
          for (int p = 0; p < nu; ++p) {
            const double nuqp = s0.Eu[q] - s0.Eu[p];
            const cd al = gr / cd(gtot, 2.0 * kPi * nuqp);
            const cd bma = gr / cd(gri, 2.0 * kPi * nuqp) - al;
            const cd C = P.c_sc * E0[((size_t)p * nu + q) * nl + lp] * SA[((size_t)q * nu + p) * nl + l];
            const cd g = C * al / (2.0 * kPi), h = C * bma / (4.0 * kPi);
            const int kp = cls[p * nl + l], kq = cls[q * nl + l];
            // R_II: g W_{p l} + g conj(W_{q l})
            P.pc_cr[z * nk + kp] += g.real();
            P.pc_ci[z * nk + kp] -= g.imag();
            P.pc_cr[z * nk + kq] += g.real();
            P.pc_ci[z * nk + kq] += g.imag();
            // R_III: h (y_p + conj y_q)(P_p + conj P_q)
            X[(0 * nk + kp) * nk + kp] += h;
            X[(1 * nk + kq) * nk + kp] += h;
            X[(2 * nk + kp) * nk + kq] += h;
            X[(3 * nk + kq) * nk + kq] += h;
          }
    for (int i = 0; i < 4 * nk * nk; ++i) P.pc_X[(size_t)z * 4 * nk * nk + i] = make_double2(X[i].real(), X[i].imag());
  }
  // directions of equal Doppler shift share the interpolation maps
  P.pc_mem.assign((size_t)nz * nd, 0);
  P.pc_moff.assign((size_t)nz * (nd + 1), 0);
  P.pc_cub.assign((size_t)nz * nd, 0.0);
  P.pc_ncls.assign(nz, 0);
  std::vector<int> dcls(nd);
  for (int z = 0; z < nz; ++z) {
    int nc = 0;
    for (int o = 0; o < nd; ++o) {
      const double v = ub[(size_t)z * nd + o];
      int c = 0;
      while (c < nc && P.pc_cub[(size_t)z * nd + c] != v) ++c;
      if (c == nc) P.pc_cub[(size_t)z * nd + nc++] = v;
      dcls[o] = c;
    }
    P.pc_ncls[z] = nc;
    int k = 0;
    for (int c = 0; c < nc; ++c) {
      P.pc_moff[(size_t)z * (nd + 1) + c] = k;
      for (int o = 0; o < nd; ++o)
        if (dcls[o] == c) P.pc_mem[(size_t)z * nd + k++] = o;
    }
    for (int c = nc; c <= nd; ++c) P.pc_moff[(size_t)z * (nd + 1) + c] = k;
  }
}

int build_problem(trap_ctx* ctx, const trap_atom_desc* at, const trap_problem_desc* pd) {
  if (!at || !pd) return fail(TRAP_EINVAL, "null descriptor");
  if (pd->n_z < 2 || pd->n_nu < 4 || pd->n_mu < 2 || (pd->n_mu & 1) || pd->n_chi < 1)
    return fail(TRAP_EINVAL, "grid sizes: need n_z>=2, n_nu>=4, even n_mu>=2, n_chi>=1");
  if (!pd->x || !pd->tau_line || !pd->T || !pd->a || !pd->eps || !pd->W_T || !pd->v || !pd->B)
    return fail(TRAP_EINVAL, "missing atmosphere array");
  if (at->kind != 0 && at->kind != 1) return fail(TRAP_EINVAL, "atom kind must be 0 or 1");
  if (!(at->lambda0_A > 0) || !(at->mass_amu > 0)) return fail(TRAP_EINVAL, "bad atomic constants");
  Problem& P = ctx->pb;
  P = Problem();
  {
    // the previous problem's table storage (kernel_bands resizes, keeping capacity)
    auto& hs = ctx->host_spare;
    P.td = std::move(hs.td);
    P.qk = std::move(hs.qk);
    P.qk32 = std::move(hs.qk32);
    P.qb = std::move(hs.qb);
    P.qb32 = std::move(hs.qb32);
    P.tofs = std::move(hs.tofs);
    P.td.clear();
    P.qk.clear();
    P.qk32.clear();
    P.qb.clear();
    P.qb32.clear();
    P.tofs.clear();
  }
  P.nz = pd->n_z;
  P.nn = pd->n_nu;
  if (const char* why = set_directions(P, pd)) return fail(TRAP_EINVAL, why);
  P.ldm = (P.nn + 7) / 8 * 8;
  const int nz = P.nz, nn = P.nn, nd = P.nd;
  P.x.assign(pd->x, pd->x + nn);
  for (int k = 0; k + 1 < nn; ++k)
    if (!(P.x[k + 1] > P.x[k])) return fail(TRAP_EINVAL, "frequency nodes must increase");
  if (!(P.x[0] < 0.0 && P.x[nn - 1] > 0.0)) return fail(TRAP_EINVAL, "frequency grid must bracket 0");
  P.tau.assign(pd->tau_line, pd->tau_line + nz);
  for (int z = 0; z < nz; ++z) {
    if (!(P.tau[z] > 0.0) || !std::isfinite(P.tau[z])) return fail(TRAP_EINVAL, "tau_line must be > 0");
    if (z > 0 && !(P.tau[z] < P.tau[z - 1])) return fail(TRAP_EINVAL, "tau_line must decrease upward");
    if (!(pd->a[z] > 0.0) || !std::isfinite(pd->a[z])) return fail(TRAP_EINVAL, "damping must be > 0");
    if (!(pd->eps[z] >= 0.0 && pd->eps[z] <= 1.0)) return fail(TRAP_EINVAL, "eps must be in [0,1]");
    if (!(pd->T[z] > 0.0)) return fail(TRAP_EINVAL, "temperature must be > 0");
    if (!std::isfinite(pd->W_T[z])) return fail(TRAP_EINVAL, "W_T not finite");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(pd->v[3 * z + k]) || !std::isfinite(pd->B[3 * z + k]))
        return fail(TRAP_EINVAL, "velocity/field not finite");
  }
  // ---- continuum
  P.has_cont = pd->kappa_c || pd->sigma_c;
  if (P.has_cont) {
    P.kc.assign((size_t)nz * nn, 0.0);
    P.sc.assign((size_t)nz * nn, 0.0);
    for (size_t i = 0; i < (size_t)nz * nn; ++i) {
      if (pd->kappa_c) P.kc[i] = pd->kappa_c[i];
      if (pd->sigma_c) P.sc[i] = pd->sigma_c[i];
      if (!(P.kc[i] >= 0.0) || !(P.sc[i] >= 0.0) || !std::isfinite(P.kc[i]) || !std::isfinite(P.sc[i]))
        return fail(TRAP_EINVAL, "continuum coefficients must be finite and >= 0");
    }
  }
  // ---- per-height scalars
  const double nu0 = kC / (at->lambda0_A * 1e-8);
  const double mass = at->mass_amu * kAMU;
  const double Tref = pd->T_ref > 0 ? pd->T_ref : 6000.0;
  const double dnuD_ref = nu0 * std::sqrt(2.0 * kKB * Tref / mass) / kC;
  P.lam.resize(nz);
  P.a.assign(pd->a, pd->a + nz);
  P.eps.assign(pd->eps, pd->eps + nz);
  P.WT.assign(pd->W_T, pd->W_T + nz);
  P.eta0.resize(nz);
  P.dnuD.resize(nz);
  std::vector<double> vth(nz);
  for (int z = 0; z < nz; ++z) {
    const double xi = pd->xi ? pd->xi[z] * 1e5 : 0.0;
    vth[z] = std::sqrt(2.0 * kKB * pd->T[z] / mass + xi * xi);
    P.dnuD[z] = nu0 * vth[z] / kC;
    P.lam[z] = dnuD_ref / P.dnuD[z];
    P.eta0[z] = std::exp(P.a[z] * P.a[z]) * std::erfc(P.a[z]) / std::sqrt(kPi);
  }
  // ---- angular grid, scattering angles, slots
  P.prd_mode = ctx->prd_mode;
  std::vector<double> dirs, ea, eb;
  angular_setup(P, dirs, ea, eb);
  // ---- sublevels per height
  std::vector<Sublevels> sub(nz);
  for (int z = 0; z < nz; ++z)
    sub[z] = sublevels(*at, pd->B[3 * z], pd->B[3 * z + 1], pd->B[3 * z + 2], dnuD_ref);
  P.nu = static_cast<int>(sub[0].Eu.size());
  P.nl = static_cast<int>(sub[0].El.size());
  P.nt = P.nu * P.nl;
  P.c_abs = sub[0].c_abs;
  P.c_sc = sub[0].c_sc;
  const int nu = P.nu, nl = P.nl, nt = P.nt;
  std::vector<double> st(nz * nt), sll(nz * nl * nl), ub(nz * nd);
  std::vector<double2> alpha(nz * nu * nu), bma(nz * nu * nu);
  // the large tables are written in full below: per-thread buffers that keep
  // their pages between calls (no zero fill, no first-touch faults per problem)
  static thread_local std::vector<double> g_buf;
  static thread_local std::vector<double2> E_buf, A_buf;
  const size_t n_g = (size_t)nz * nt * nd * 4, n_e = static_cast<size_t>(nz) * nd * 4 * nu * nu * nl;
  if (g_buf.size() < n_g) g_buf.resize(n_g);
  if (E_buf.size() < n_e) E_buf.resize(n_e);
  if (A_buf.size() < n_e) A_buf.resize(n_e);
  double* g = g_buf.data();
  double2* E = E_buf.data();
  double2* A = A_buf.data();
  const double rE = at->r_E;
  for (int z = 0; z < nz; ++z) {
    const Sublevels& s = sub[z];
    for (int u = 0; u < nu; ++u)
      for (int l = 0; l < nl; ++l) st[z * nt + u * nl + l] = (s.Eu[u] - s.El[l]) / P.dnuD[z];
    for (int l = 0; l < nl; ++l)
      for (int lp = 0; lp < nl; ++lp) sll[(z * nl + l) * nl + lp] = (s.El[l] - s.El[lp]) / P.dnuD[z];
    const double gtot = 4.0 * kPi * P.a[z] * P.dnuD[z];
    const double gri = gtot / (1.0 + rE);
    const double gr = (1.0 - P.eps[z]) * gri;
    for (int u = 0; u < nu; ++u)
      for (int up = 0; up < nu; ++up) {
        const double nuuu = s.Eu[u] - s.Eu[up];
        const cd al = gr / cd(gtot, 2.0 * kPi * nuuu);
        const cd be = gr / cd(gri, 2.0 * kPi * nuuu);
        alpha[(z * nu + u) * nu + up] = make_double2(al.real(), al.imag());
        bma[(z * nu + u) * nu + up] = make_double2((be - al).real(), (be - al).imag());
      }
    for (int o = 0; o < nd; ++o) {
      const double vdot = pd->v[3 * z] * dirs[3 * o] + pd->v[3 * z + 1] * dirs[3 * o + 1] +
                          pd->v[3 * z + 2] * dirs[3 * o + 2];
      ub[z * nd + o] = vdot * 1e5 / vth[z];
      // projections of every transition's dipole vector on this direction's axes
      std::vector<cd> pa(nt), pb(nt);
      for (int t = 0; t < nt; ++t) stokes_proj(&s.d[t * 3], &ea[3 * o], &eb[3 * o], &pa[t], &pb[t]);
      for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 4; ++j)
          g[((z * nt + t) * nd + o) * 4 + j] = stokes_pair(j, pa[t], pb[t], std::conj(pa[t]), std::conj(pb[t])).real();
      for (int i = 0; i < 4; ++i)
        for (int up = 0; up < nu; ++up)
          for (int u = 0; u < nu; ++u)
            for (int l = 0; l < nl; ++l) {
              const int t1 = up * nl + l, t2 = u * nl + l;
              // E[z][o][i][u'][u][l'] with l' = l here
              const cd e = stokes_pair(i, pa[t1], pb[t1], std::conj(pa[t2]), std::conj(pb[t2]));
              E[((((static_cast<size_t>(z) * nd + o) * 4 + i) * nu + up) * nu + u) * nl + l] = make_double2(e.real(), e.imag());
              // A[z][o][j][u][u'][l] with (u, u') = (up, u) index order: first upper index u
              const cd aa = 0.5 * e;
              A[((((static_cast<size_t>(z) * nd + o) * 4 + i) * nu + up) * nu + u) * nl + l] = make_double2(aa.real(), aa.imag());
            }
    }
  }
  precond_weights(P, *at, dnuD_ref, ea, eb, ub, rE);
  // ---- upload
  std::vector<double> sig;
  auto spl = spline_map(P.x, &sig);
  kernel_bands(P, sig);
  std::vector<double> sigT(sig.size());
  for (int i = 0; i < nn; ++i)
    for (int j = 0; j < nn; ++j) sigT[(size_t)j * nn + i] = sig[(size_t)i * nn + j];
  // one device allocation and one pinned copy for every table (the layout of
  // the batch is mirrored by estimate_bytes)
  UploadBatch up;
  up.add(&P.d_x, P.x);
  up.add(&P.d_P, spl);
  up.add(&P.d_Sig, sig);
  up.add(&P.d_SigT, sigT);
  up.add(&P.d_mu, P.mu);
  up.add(&P.d_w, P.w);
  up.add(&P.d_tau, P.tau);
  up.add(&P.d_lam, P.lam);
  up.add(&P.d_a, P.a);
  up.add(&P.d_eps, P.eps);
  up.add(&P.d_WT, P.WT);
  up.add(&P.d_eta0, P.eta0);
  up.add(&P.d_ub, ub);
  // mirror roles of the kernel rows (see Problem::row_role): the grid must be
  // exactly symmetric and a partner's shifts exactly the negated ones at every height
  P.row_role.clear();
  P.rows_mirrored = 0;
  {
    // symmetric to rounding (a grid built as start + k step is not bitwise
    // symmetric); the mirrored rows then differ from direct ones by far less
    // than the quadrature error
    const double xs = std::max(std::fabs(P.x[0]), std::fabs(P.x[nn - 1]));
    bool sym = true;
    for (int n = 0; n < nn && sym; ++n) sym = std::fabs(P.x[n] + P.x[nn - 1 - n]) <= 1e-13 * xs;
    if (sym) {
      std::vector<int> role(nt, -1);
      auto negated = [&](int t, int t2) {
        for (int z = 0; z < nz; ++z)
          if (st[z * nt + t2] != -st[z * nt + t]) return false;
        return true;
      };
      for (int t = 0; t < nt; ++t) {
        for (int t2 = 0; t2 < t && role[t] < 0; ++t2)
          if (role[t2] == -1 && negated(t, t2)) role[t] = t2;
        if (role[t] < 0 && negated(t, t)) role[t] = t;
      }
      bool any = false;
      for (int t = 0; t < nt; ++t) any = any || role[t] >= 0;
      if (any) P.row_role = role;
      for (int t = 0; t < nt; ++t)
        if (role[t] >= 0) P.rows_mirrored += (role[t] == t ? nn / 2 : nn);
    }
  }
  up.add(&P.d_st, st);
  up.add(&P.d_sll, sll);
  up.add(&P.d_theta, P.theta);
  up.add(&P.d_theta_rows, P.theta_rows);
  up.add(&P.d_theta_rw, P.theta_rw);
  up.add(&P.d_slot_theta, P.slot_theta);
  up.add(&P.d_slot_dir, P.slot_dir);
  up.add(&P.d_slot_off, P.slot_off);
  up.add(&P.d_pair_slot, P.pair_slot);
  up.add(&P.d_pair_theta, P.pair_theta);
  up.add(&P.d_pair_off, P.pair_off);
  up.add(&P.d_pair_o, P.pair_o);
  up.add(&P.d_pair_dir, P.pair_dir);
  up.add(&P.d_pair_index, P.pair_index);
  up.add(&P.d_grp[0], P.grp[0]);
  up.add(&P.d_grp[1], P.grp[1]);
  up.add(&P.d_cgrp[0], P.cgrp[0]);
  up.add(&P.d_cgrp[1], P.cgrp[1]);
  up.add(&P.d_cord, P.cord);
  up.add(&P.d_unit_ctr, P.unit_ctr);
  up.add(&P.d_cord0, P.cord0);
  up.add(reinterpret_cast<void**>(&P.d_E), E, n_e * sizeof(double2));
  up.add(reinterpret_cast<void**>(&P.d_A), A, n_e * sizeof(double2));
  up.add(&P.d_alpha, alpha);
  up.add(&P.d_bma, bma);
  up.add(reinterpret_cast<void**>(&P.d_g), g, n_g * sizeof(double));
  up.add(&P.d_td, P.td);
  up.add(&P.d_qb, P.qb);
  up.add(&P.d_qk32, P.qk32);
  up.add(&P.d_qb32, P.qb32);
  if (P.has_cont) {
    up.add(&P.d_kc, P.kc);
    up.add(&P.d_sc, P.sc);
    up.add(&P.d_ea, ea);
    up.add(&P.d_eb, eb);
  }
  TRAP_TRY(up.commit(ctx));
  return TRAP_OK;
}

}  // namespace trap
