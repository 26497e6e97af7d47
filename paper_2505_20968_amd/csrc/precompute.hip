// Device precompute for one problem (paper Sect. 4.3, App. C-E):
//  * propagation-matrix coefficients and thermal emissivity per (z, o, n);
//  * R_II kernel rows M[z][theta][t][n][:] = int F(Theta, u'+s_t, u_n+s_t) S_m(u') du'
//    by product integration of F against each cubic piece of the cardinal
//    spline basis (moments of F on every knot interval, then the spline map);
//  * R_III incoming weights r[z][t][m] = int W(a, u'+s_t) S_m(u') du' (the 1/u'
//    tail of Im W subtracted on both tails) and outgoing profiles on the grid;
//  * the normalisation factor f (App. E) and b = Lambda eps_th + t.
//
// Quadrature: Gauss-Legendre 16 on panels chosen per knot interval.  Panels
// grow geometrically away from the Voigt/Lorentz centre of F at
// u' = -u_n - 2 s_t (first width 2 max(cos(Theta/2), a)), and never exceed
// half the Gaussian width 2 sin(Theta/2); the Gaussian factor is cut where
// it falls below e^-43.
#include <cmath>
#include <vector>

#include "faddeeva.h"
#include "trap_internal.h"

namespace trap {

__constant__ FaddeevaCoef c_fad;
__constant__ double c_gl_t[16];
__constant__ double c_gl_w[16];

static constexpr double kSqrtPi = 1.7724538509055160273;
static constexpr double kInvSqrtPi = 0.56418958354775628695;
static constexpr double kPiD = 3.14159265358979323846;

__device__ inline double2 wz(double x, double y) { return faddeeva_w(x, y, c_fad); }

// F(Theta, up, u) in reduced units; pi_limit selects the Theta = pi form.
struct FParams {
  double sG, cG, inv_sinT, a;
  bool pi_limit;
};

__device__ inline double2 Ffun(const FParams& p, double up, double u) {
  if (p.pi_limit) {
    const double g = exp(-0.25 * (u - up) * (u - up));
    // i / (2 sqrt(pi) (m + i a)) = i (m - i a) / (2 sqrt(pi) (m^2 + a^2))
    const double m = 0.5 * (u + up);
    const double d = 2.0 * kSqrtPi * (m * m + p.a * p.a);
    return make_double2(g * p.a / d, g * m / d);
  }
  const double q = (u - up) / (2.0 * p.sG);
  const double g = exp(-q * q);
  if (g == 0.0) return make_double2(0.0, 0.0);
  const double2 w = wz((u + up) / (2.0 * p.cG), p.a / p.cG);
  return make_double2(g * w.x * p.inv_sinT, g * w.y * p.inv_sinT);
}

// ------------------------------------------------------------------ profiles
__global__ void k_profiles(int nz, int nd, int nn, int nt, const double* __restrict__ x,
                           const double* __restrict__ lam, const double* __restrict__ a,
                           const double* __restrict__ ub, const double* __restrict__ st,
                           const double* __restrict__ g, const double* __restrict__ eta0,
                           const double* __restrict__ eps, const double* __restrict__ WT,
                           double c_abs, double* __restrict__ K8, double* __restrict__ epsth) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long total = (long long)nz * nd * nn;
  if (id >= total) return;
  const int n = id % nn;
  const int o = (id / nn) % nd;
  const int z = id / ((long long)nn * nd);
  const double u = lam[z] * x[n] + ub[z * nd + o];
  double eta[4] = {0, 0, 0, 0}, rho[4] = {0, 0, 0, 0};
  for (int t = 0; t < nt; ++t) {
    const double2 w = wz(u + st[z * nt + t], a[z]);
    const double* gg = g + ((long long)(z * nt + t) * nd + o) * 4;
    for (int j = 0; j < 4; ++j) {
      eta[j] += w.x * gg[j];
      rho[j] += w.y * gg[j];
    }
  }
  const double sc = 0.5 * c_abs * kInvSqrtPi;
  for (int j = 0; j < 4; ++j) {
    eta[j] *= sc;
    rho[j] *= sc;
  }
  const double inv = 1.0 / eta[0];
  double* k = K8 + id * 8;
  k[0] = eta[1] * inv;
  k[1] = eta[2] * inv;
  k[2] = eta[3] * inv;
  k[3] = rho[1] * inv;
  k[4] = rho[2] * inv;
  k[5] = rho[3] * inv;
  k[6] = inv;
  k[7] = eta[0] / eta0[z];
  const double th = eps[z] * WT[z];
  for (int j = 0; j < 4; ++j) epsth[id * 4 + j] = th * eta[j];
}

// ------------------------------------------------------------------ panel integration helper
// Integrate f(x) * t^q (q = 0..nq-1, t = (x - x0)/h) over [pa, pb] with panels
// graded away from xc.  Accumulates into acc[q] (complex).
template <typename Fn>
__device__ void graded_integrate(double pa, double pb, double xc, double wc, double Lg, double x0,
                                 double invh, int nq, Fn f, double2* acc) {
  auto panel = [&](double l, double r) {
    const double hw = r - l;
    for (int i = 0; i < 16; ++i) {
      const double xx = l + hw * c_gl_t[i];
      const double2 v = f(xx);
      const double ww = hw * c_gl_w[i];
      double tp = ww;
      const double t = (xx - x0) * invh;
      for (int q = 0; q < nq; ++q) {
        acc[q].x += tp * v.x;
        acc[q].y += tp * v.y;
        tp *= t;
      }
    }
  };
  auto sweep = [&](double start, double end) {
    // from `start` (nearest the centre) towards `end`
    const double dir = end > start ? 1.0 : -1.0;
    double pos = start;
    int guard = 0;
    while (dir * (end - pos) > 0.0 && guard < 4096) {
      const double dist = fabs(pos - xc);
      double w = fmin(Lg, fmax(wc, dist));
      double nxt = pos + dir * w;
      if (dir * (end - nxt) < 0.25 * w) nxt = end;
      panel(fmin(pos, nxt), fmax(pos, nxt));
      pos = nxt;
      ++guard;
    }
  };
  if (pb <= pa) return;
  if (xc > pa && xc < pb) {
    sweep(xc, pa);
    sweep(xc, pb);
  } else if (fabs(pa - xc) <= fabs(pb - xc)) {
    sweep(pa, pb);
  } else {
    sweep(pb, pa);
  }
}

__device__ inline int upper_interval(const double* x, int nn, double v) {
  // largest k with x[k] <= v, clamped to [0, nn-1]
  int lo = 0, hi = nn - 1;
  if (v < x[0]) return -1;
  if (v >= x[nn - 1]) return nn - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------ R_II kernel rows
// One 64-thread block per row (z, theta, t, n).
__global__ void __launch_bounds__(64) k_kernel_rows(
    int nth, int nt, int nn, int ldm, const double* __restrict__ x, const double* __restrict__ P,
    const double* __restrict__ lam, const double* __restrict__ av, const double* __restrict__ st,
    const double* __restrict__ theta, double* __restrict__ M64, float* __restrict__ M32,
    long long row0) {
  extern __shared__ double2 mom[];     // [(nn+1)][4], piece index shifted by one
  const long long row = row0 + blockIdx.x;
  const int lane = threadIdx.x;
  const int n = row % nn;
  const int t = (row / nn) % nt;
  const int th = (row / ((long long)nn * nt)) % nth;
  const int z = row / ((long long)nn * nt * nth);
  const double L = lam[z], a = av[z], s = st[z * nt + t], Th = theta[th];
  const size_t base = (size_t)((((size_t)z * nth + th) * nt + t) * 2) * nn * ldm;
  const size_t rre = base + (size_t)n * ldm, rim = base + (size_t)nn * ldm + (size_t)n * ldm;
  if (Th == 0.0) {
    const double2 w = wz(L * x[n] + s, a);
    for (int m = lane; m < ldm; m += 64) {
      const double re = (m == n) ? kSqrtPi * w.x : 0.0, im = (m == n) ? kSqrtPi * w.y : 0.0;
      if (M64) { M64[rre + m] = re; M64[rim + m] = im; }
      if (M32) { M32[rre + m] = (float)re; M32[rim + m] = (float)im; }
    }
    return;
  }
  FParams fp;
  fp.pi_limit = (Th >= kPiD);
  fp.sG = fp.pi_limit ? 1.0 : sin(0.5 * Th);
  fp.cG = fp.pi_limit ? 0.0 : cos(0.5 * Th);
  fp.inv_sinT = fp.pi_limit ? 0.0 : 1.0 / sin(Th);
  fp.a = a;
  const double sigma = 2.0 * fp.sG / L;
  const double R = 6.6 * sigma;
  const double xn = x[n];
  const double lo = xn - R, hi = xn + R;
  const double xc = -xn - 2.0 * s / L;
  const double wc = 2.0 * fmax(fp.cG, a) / L;
  const double Lg = 0.5 * sigma;
  for (int i = lane; i < (nn + 1) * 4; i += 64) mom[i] = make_double2(0.0, 0.0);
  __syncthreads();
  // pieces: -1 left tail, 0..nn-2 knot intervals, nn-1 right tail
  int plo = upper_interval(x, nn, lo);          // -1 if lo < x0
  int phi = upper_interval(x, nn, hi);
  if (phi >= 0 && phi < nn - 1 && x[phi] >= hi) phi -= 1;
  const double un = L * xn + s;
  auto integrand = [&](double xp) {
    const double2 F = Ffun(fp, L * xp + s, un);
    return make_double2(L * F.x, L * F.y);
  };
  for (int p = plo + lane; p <= phi; p += 64) {
    double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (p < 0) {
      graded_integrate(lo, x[0], xc, wc, Lg, 0.0, 0.0, 1, integrand, acc);
    } else if (p >= nn - 1) {
      graded_integrate(x[nn - 1], hi, xc, wc, Lg, 0.0, 0.0, 1, integrand, acc);
    } else {
      const double pa = fmax(x[p], lo), pb = fmin(x[p + 1], hi);
      graded_integrate(pa, pb, xc, wc, Lg, x[p], 1.0 / (x[p + 1] - x[p]), 4, integrand, acc);
    }
    for (int q = 0; q < 4; ++q) mom[(p + 1) * 4 + q] = acc[q];
  }
  __syncthreads();
  const int klo = max(plo, 0), khi = min(phi, nn - 2);
  for (int m = lane; m < ldm; m += 64) {
    double re = 0.0, im = 0.0;
    if (m >= nn) {      // zero padding of the row
      if (M64) { M64[rre + m] = 0.0; M64[rim + m] = 0.0; }
      if (M32) { M32[rre + m] = 0.0f; M32[rim + m] = 0.0f; }
      continue;
    }
    for (int k = klo; k <= khi; ++k) {
      const double* pk = P + (size_t)k * 4 * nn + m;
      for (int q = 0; q < 4; ++q) {
        const double c = pk[(size_t)q * nn];
        const double2 mm = mom[(k + 1) * 4 + q];
        re += c * mm.x;
        im += c * mm.y;
      }
    }
    if (m == 0) { re += mom[0].x; im += mom[0].y; }
    if (m == nn - 1) { re += mom[nn * 4].x; im += mom[nn * 4].y; }
    if (M64) { M64[rre + m] = re; M64[rim + m] = im; }
    if (M32) { M32[rre + m] = (float)re; M32[rim + m] = (float)im; }
  }
}

// ------------------------------------------------------------------ R_III weights
__global__ void __launch_bounds__(64) k_r3_rows(int nt, int nn, const double* __restrict__ x,
                                                const double* __restrict__ P, const double* __restrict__ lam,
                                                const double* __restrict__ av, const double* __restrict__ st,
                                                double2* __restrict__ r3, double2* __restrict__ prof) {
  extern __shared__ double2 mom[];
  const int row = blockIdx.x;            // z * nt + t
  const int t = row % nt, z = row / nt;
  const int lane = threadIdx.x;
  const double L = lam[z], a = av[z], s = st[z * nt + t];
  for (int i = lane; i < (nn + 1) * 4; i += 64) mom[i] = make_double2(0.0, 0.0);
  __syncthreads();
  const double xc = -s / L, wc = 0.25 / L, Lg = 2.0 / L;
  auto integrand = [&](double xp) {
    const double2 w = wz(L * xp + s, a);
    return make_double2(L * w.x, L * w.y);
  };
  for (int p = lane; p < nn - 1; p += 64) {
    double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    graded_integrate(x[p], x[p + 1], xc, wc, Lg, x[p], 1.0 / (x[p + 1] - x[p]), 4, integrand, acc);
    for (int q = 0; q < 4; ++q) mom[(p + 1) * 4 + q] = acc[q];
  }
  // tails in u units: int [w(u'+s+ia) - i/(sqrt(pi) u')] du' over (-inf, u0] and [u1, inf)
  if (lane < 2) {
    const double uedge = (lane == 0) ? L * x[0] : L * x[nn - 1];
    const double sgn = (lane == 0) ? -1.0 : 1.0;
    const double sc = fabs(uedge);
    double2 acc = make_double2(0.0, 0.0);
    for (int pnl = 0; pnl < 32; ++pnl) {
      const double ta = pnl / 32.0, tb = (pnl + 1) / 32.0;
      for (int i = 0; i < 16; ++i) {
        const double tau = ta + (tb - ta) * c_gl_t[i];
        const double om = 1.0 - tau;
        const double up = uedge + sgn * sc * tau / om;
        const double2 w = wz(up + s, a);
        const double jac = sc / (om * om) * (tb - ta) * c_gl_w[i];
        acc.x += jac * w.x;
        acc.y += jac * (w.y - kInvSqrtPi / up);
      }
    }
    mom[(lane == 0 ? 0 : nn) * 4] = acc;
  }
  __syncthreads();
  for (int m = lane; m < nn; m += 64) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nn - 1; ++k) {
      const double* pk = P + (size_t)k * 4 * nn + m;
      for (int q = 0; q < 4; ++q) {
        const double c = pk[(size_t)q * nn];
        re += c * mom[(k + 1) * 4 + q].x;
        im += c * mom[(k + 1) * 4 + q].y;
      }
    }
    if (m == 0) { re += mom[0].x; im += mom[0].y; }
    if (m == nn - 1) { re += mom[nn * 4].x; im += mom[nn * 4].y; }
    r3[(size_t)row * nn + m] = make_double2(re, im);
    prof[(size_t)row * nn + m] = wz(L * x[m] + s, a);
  }
}

// ------------------------------------------------------------------ normalisation
__global__ void k_flat_field(long long total, int nd, int nn, const double* __restrict__ WT,
                             double* __restrict__ I) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int z = id / ((long long)nd * nn);
  double* v = I + id * 4;
  v[0] = WT[z];
  v[1] = 0.0;
  v[2] = 0.0;
  v[3] = 0.0;
}

__global__ void k_norm_factor(long long total, int nd, int nn, const double* __restrict__ eps,
                              const double* __restrict__ WT, const double* __restrict__ K8,
                              const double* __restrict__ num, double* __restrict__ f) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int z = id / ((long long)nd * nn);
  const double etaI = 1.0 / K8[id * 8 + 6];
  f[id] = (1.0 - eps[z]) * WT[z] * etaI / num[id * 4];
}

// ------------------------------------------------------------------ driver
int run_precompute(trap_ctx* ctx, int store_mask) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  hipStream_t s = ctx->stream;
  static bool coef_ready = false;
  static FaddeevaCoef hc;
  static double gt[16], gw[16];
  if (!coef_ready) {
    faddeeva_coefficients(&hc);
    // Gauss-Legendre 16 on [0,1] (Newton on P_16)
    const int n = 16;
    for (int i = 0; i < n; ++i) {
      double zz = cos(kPiD * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = zz;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * zz * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (zz * p1 - p0) / (zz * zz - 1.0);
        const double dz = p1 / dp;
        zz -= dz;
        if (fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = zz;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * zz * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (zz * p1 - p0) / (zz * zz - 1.0);
      gt[i] = 0.5 * (1.0 - zz);
      gw[i] = 1.0 / ((1.0 - zz * zz) * dp * dp);
    }
    coef_ready = true;
  }
  TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_fad), &hc, sizeof(hc)));
  TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_t), gt, sizeof(gt)));
  TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), gw, sizeof(gw)));
  const int nz = P.nz, nd = P.nd, nn = P.nn, nt = P.nt, nth = P.nth;
  const long long npt = (long long)nz * nd * nn;
  if (!C.d_K) {
    TRAP_TRY(dalloc_t(ctx, &C.d_K, npt * 8));
    TRAP_TRY(dalloc_t(ctx, &C.d_epsth, npt * 4));
    TRAP_TRY(dalloc_t(ctx, &C.d_f, npt));
    TRAP_TRY(dalloc_t(ctx, &C.d_r3, (size_t)nz * nt * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_prof, (size_t)nz * nt * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_b, npt * 4));
  }
  hipLaunchKernelGGL(k_profiles, dim3(ceil_div(npt, 256)), dim3(256), 0, s, nz, nd, nn, nt, P.d_x,
                     P.d_lam, P.d_a, P.d_ub, P.d_st, P.d_g, P.d_eta0, P.d_eps, P.d_WT, P.c_abs, C.d_K,
                     C.d_epsth);
  TRAP_HIP(hipGetLastError());
  const size_t kelems = (size_t)nz * nth * nt * 2 * nn * P.ldm;
  const int mask = store_mask | 1;     // FP64 kernels always exist (residual, f, b)
  if ((mask & 1) && !C.d_M64) TRAP_TRY(dalloc_t(ctx, &C.d_M64, kelems));
  if ((mask & 2) && !C.d_M32) TRAP_TRY(dalloc_t(ctx, &C.d_M32, kelems));
  C.store_mask = mask;
  const long long nrows = (long long)nz * nth * nt * nn;
  const size_t lds = (size_t)(nn + 1) * 4 * sizeof(double2);
  if (lds > 64 * 1024) return fail(TRAP_EINVAL, "frequency grid too large for the kernel precompute");
  const long long chunk = 1 << 20;
  const int pr = prof_begin(ctx, TRAP_STAGE_KERNEL_ROWS);
  for (long long r0 = 0; r0 < nrows; r0 += chunk) {
    const long long nr = std::min(chunk, nrows - r0);
    hipLaunchKernelGGL(k_kernel_rows, dim3((unsigned)nr), dim3(64), lds, s, nth, nt, nn, P.ldm, P.d_x, P.d_P,
                       P.d_lam, P.d_a, P.d_st, P.d_theta, (mask & 1) ? C.d_M64 : nullptr,
                       (mask & 2) ? C.d_M32 : nullptr, r0);
    TRAP_HIP(hipGetLastError());
  }
  prof_end(ctx, pr);
  hipLaunchKernelGGL(k_r3_rows, dim3(nz * nt), dim3(64), lds, s, nt, nn, P.d_x, P.d_P, P.d_lam, P.d_a,
                     P.d_st, C.d_r3, C.d_prof);
  TRAP_HIP(hipGetLastError());
  C.done = true;
  // normalisation factor f: one unnormalised FP64 Sigma apply on (W_T, 0, 0, 0)
  TRAP_TRY(ensure_work(ctx, TRAP_FP64));
  double* flat = ctx->wk.tmp64;
  double* num = ctx->wk.r;
  hipLaunchKernelGGL(k_flat_field, dim3(ceil_div(npt, 256)), dim3(256), 0, s, npt, nd, nn, P.d_WT, flat);
  TRAP_HIP(hipGetLastError());
  TRAP_TRY(sigma_apply(ctx, flat, num, TRAP_FP64, 0, 0));
  hipLaunchKernelGGL(k_norm_factor, dim3(ceil_div(npt, 256)), dim3(256), 0, s, npt, nd, nn, P.d_eps,
                     P.d_WT, C.d_K, num, C.d_f);
  TRAP_HIP(hipGetLastError());
  // right-hand side b = Lambda eps_th + t
  TRAP_TRY(formal_apply(ctx, C.d_epsth, C.d_b, 1, TRAP_FP64));
  TRAP_HIP(hipStreamSynchronize(s));
  return TRAP_OK;
}

void faddeeva_coefficients(FaddeevaCoef* out) {
  const int N = kWeidemanN, M = 2 * N;
  const double L = sqrt(N / sqrt(2.0));
  std::vector<double> aq(N + 1, 0.0);
  for (int q = 1; q <= N; ++q) {
    double sum = 0.0;
    for (int k = -M + 1; k <= M - 1; ++k) {
      const double th = k * kPiD / M;
      const double t = L * tan(0.5 * th);
      const double f = exp(-t * t) * (L * L + t * t);
      sum += f * cos(kPiD * q * k / M);
    }
    aq[q] = sum / (2.0 * M);
  }
  out->L = L;
  for (int i = 0; i < N; ++i) out->a[i] = aq[N - i];
}

}  // namespace trap
