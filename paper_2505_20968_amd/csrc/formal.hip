// Formal solution Lambda (paper Sect. 3): per ray (Omega, nu) a sweep along z,
// upward rays from the bottom (boundary (W_T(z_min), 0, 0, 0)), downward rays
// from the top (no incoming radiation).  Trapezoidal optical depth
//   dtau = (r_k + r_{k+1})/2 |tau_line(z_k) - tau_line(z_{k+1})| / |mu|,
// r = eta_I/eta_0, and DELO-linear steps
//   (Id + psi_c K'_c) I_c = (e^{-dtau} Id - psi_u K'_u) I_u + psi_u S_u + psi_c S_c,
// K' = K/eta_I - Id, S = eps/eta_I.  The weights
//   psi_u = [1 - e^{-x}(1 + x)]/x,  psi_c = [x - 1 + e^{-x}]/x
// cancel catastrophically for small x; below a precision-dependent threshold
// (0.1 in FP64, 1 in FP32) they are summed from their Taylor series
//   psi_u = sum_{m>=2} (-1)^m (m-1) x^(m-1)/m!,  psi_c = sum_{m>=2} (-1)^m x^(m-1)/m!.
// One thread per ray; arithmetic in the vector precision T.
#include <cmath>

#include "trap_internal.h"

namespace trap {

template <typename T>
__device__ inline void delo_weights(T x, T& pu, T& pc, T& ex) {
  ex = exp(-x);
  const T thr = sizeof(T) == 8 ? T(0.1) : T(1.0);
  if (x < thr) {
    // Horner-free accumulation with factorial recursion, 20 terms
    T p = x, fac = T(2), su = T(0), sc = T(0), sgn = T(1);
    for (int m = 2; m < 22; ++m) {
      if (m > 2) fac *= T(m);
      su += sgn * T(m - 1) * p / fac;
      sc += sgn * p / fac;
      p *= x;
      sgn = -sgn;
    }
    pu = su;
    pc = sc;
  } else {
    pu = (T(1) - ex * (T(1) + x)) / x;
    pc = (x - T(1) + ex) / x;
  }
}

// y = K' v with K' = [[0,kQ,kU,kV],[kQ,0,rV,-rU],[kU,-rV,0,rQ],[kV,rU,-rQ,0]]
template <typename T>
__device__ inline void kprime_mul(const T* k, const T* v, T* y) {
  y[0] = k[0] * v[1] + k[1] * v[2] + k[2] * v[3];
  y[1] = k[0] * v[0] + k[5] * v[2] - k[4] * v[3];
  y[2] = k[1] * v[0] - k[5] * v[1] + k[3] * v[3];
  y[3] = k[2] * v[0] + k[4] * v[1] - k[3] * v[2];
}

// solve (Id + p K') x = b, 4x4 Gaussian elimination with partial pivoting
template <typename T>
__device__ inline void delo_solve(const T* k, T p, const T* b, T* xout) {
  T A[4][5];
  A[0][0] = T(1); A[0][1] = p * k[0]; A[0][2] = p * k[1]; A[0][3] = p * k[2];
  A[1][0] = p * k[0]; A[1][1] = T(1); A[1][2] = p * k[5]; A[1][3] = -p * k[4];
  A[2][0] = p * k[1]; A[2][1] = -p * k[5]; A[2][2] = T(1); A[2][3] = p * k[3];
  A[3][0] = p * k[2]; A[3][1] = p * k[4]; A[3][2] = -p * k[3]; A[3][3] = T(1);
#pragma unroll
  for (int i = 0; i < 4; ++i) A[i][4] = b[i];
  // every index below is a compile-time constant (the pivot row is swapped in
  // by comparison, not by indexing), so the matrix stays in registers
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    T best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[r][c]) > best) {
        best = fabs(A[r][c]);
        piv = r;
      }
#pragma unroll
    for (int r = c + 1; r < 4; ++r)
      if (piv == r)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const T tmp = A[c][j];
          A[c][j] = A[r][j];
          A[r][j] = tmp;
        }
    const T inv = T(1) / A[c][c];
#pragma unroll
    for (int r = c + 1; r < 4; ++r) {
      const T fct = A[r][c] * inv;
#pragma unroll
      for (int j = c; j < 5; ++j) A[r][j] -= fct * A[c][j];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    T v = A[i][4];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) v -= A[i][j] * xout[j];
    xout[i] = v / A[i][i];
  }
}

// E_k = int_0^m t^k e^{-t} dt for k = 0, 1, 2: the closed forms, or below
// m = 0.5 (where they cancel) sum_j (-1)^j m^(k+j+1) / (j! (k+j+1)).  FP64.
__device__ inline void exp_moments(double m, double& E0, double& E1, double& E2) {
  if (m < 0.5) {
    // E_k = m^(k+1) sum_j t_j / (k + j + 1), t_j = (-m)^j / j!; 16 terms
    // leave a relative remainder below 1e-16 for m < 0.5 (unrolled, so the
    // divisors are constants)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, t = 1.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      s0 += t * (1.0 / (j + 1));
      s1 += t * (1.0 / (j + 2));
      s2 += t * (1.0 / (j + 3));
      t *= -m * (1.0 / (j + 1));
    }
    E0 = m * s0;
    E1 = m * m * s1;
    E2 = m * m * m * s2;
  } else {
    const double ex = exp(-m);
    E0 = 1.0 - ex;
    E1 = E0 - m * ex;
    E2 = 2.0 * E1 - m * m * ex;
  }
}

// DELOPAR (Sect. 3): the source S integrated against e^{-t} over the upwind
// interval [0, m] (t from the current point O back to the upwind point M)
// with the parabola through M (t = m), O (t = 0) and the downwind point P
// (t = -p):
//   w_M = (E2 + p E1) / (m (m + p)),   w_O = -(E2 + (p - m) E1 - m p E0) / (m p),
//   w_P = (E2 - m E1) / (p (m + p)).
__device__ inline void parabolic_weights(double m, double p, double& wM, double& wO, double& wP) {
  double E0, E1, E2;
  exp_moments(m, E0, E1, E2);
  wM = (E2 + p * E1) / (m * (m + p));
  wO = -(E2 + (p - m) * E1 - m * p * E0) / (m * p);
  wP = (E2 - m * E1) / (p * (m + p));
}

// BESSER (Sect. 3): S over the upwind interval is the quadratic Bezier curve
// from S_M to S_O with one control point c; its Bernstein factors (t/m)^2,
// 2 (t/m)(1 - t/m), (1 - t/m)^2 against e^{-t} give
//   w_M = E2/m^2,   w_C = 2 (E1/m - E2/m^2),   w_O = E0 - 2 E1/m + E2/m^2.
__device__ inline void bezier_weights(double m, double& wM, double& wC, double& wO) {
  double E0, E1, E2;
  exp_moments(m, E0, E1, E2);
  const double a = E1 / m, b = E2 / (m * m);
  wM = b;
  wC = 2.0 * (a - b);
  wO = E0 - 2.0 * a + b;
}

// The control point: the tangent at O of the parabola through M, O and P
// (slope zero where O is a local extremum of S), followed back half the
// upwind interval, and kept inside the range of S_M and S_O so that the
// curve does not overshoot.  hM, hP are the upwind and downwind optical steps.
template <typename T>
__device__ inline T besser_control(T SM, T SO, T SP, T hM, T hP) {
  const T dM = (SO - SM) / hM, dP = (SP - SO) / hP;
  const T dO = dM * dP > T(0) ? (hM * dP + hP * dM) / (hM + hP) : T(0);
  const T c = SO - T(0.5) * hM * dO;
  return fmin(fmax(c, fmin(SM, SO)), fmax(SM, SO));
}

// The BESSER step linearised about a reference source (its Jacobian): the
// branch taken at each point (zero slope at an extremum, the range limit
// towards S_M or S_O, or the tangent) is the one the reference source takes
// there, and that branch's linear weights are applied to the source S.
template <typename T>
__device__ inline T besser_control_lin(T SM, T SO, T SP, T RM, T RO, T RP, T hM, T hP) {
  const T rM = (RO - RM) / hM, rP = (RP - RO) / hP;
  const bool ext = !(rM * rP > T(0));
  const T rO = ext ? T(0) : (hM * rP + hP * rM) / (hM + hP);
  const T cr = RO - T(0.5) * hM * rO;
  const T lo = fmin(RM, RO), hi = fmax(RM, RO);
  if (cr < lo) return RM <= RO ? SM : SO;
  if (cr > hi) return RM >= RO ? SM : SO;
  if (ext) return SO;
  const T dM = (SO - SM) / hM, dP = (SP - SO) / hP;
  return SO - T(0.5) * hM * ((hM * dP + hP * dM) / (hM + hP));
}

// PAR: 0 = DELO-linear only, 1 = DELOPAR only, 2 = BESSER only, 3 = BESSER
// linearised about the reference emissivity eref, -1 = the scheme argument
// decides between DELO-linear and DELOPAR
template <typename T, int PAR>
__device__ __forceinline__ void formal_body(int bx, int nz, int nd, int nn, const double* __restrict__ mu,
                                            const double* __restrict__ tau, const double* __restrict__ K8,
                                            const double* __restrict__ WT, const T* __restrict__ eps,
                                            T* __restrict__ I, int with_boundary, int scheme,
                                            const T* __restrict__ eref = nullptr) {
  const int id = bx * blockDim.x + threadIdx.x;
  if (id >= nd * nn) return;
  const int o = id / nn, n = id % nn;
  const double m = mu[o];
  const bool up = m > 0.0;
  const long long zs = (long long)nd * nn;          // point stride between heights
  auto pidx = [&](int z) { return (long long)z * zs + (long long)o * nn + n; };
  int z = up ? 0 : nz - 1;
  const int dz = up ? 1 : -1;
  T Icur[4] = {T(0), T(0), T(0), T(0)};
  if (up && with_boundary) Icur[0] = T(WT[0]);
  T ku[6], Su[4], ru;
  double rud;
  T Ru[4];                                          // reference source (PAR 3)
  double tz = tau[z];
  {
    const long long p = pidx(z);
    const double* k = K8 + p * 8;
    for (int i = 0; i < 6; ++i) ku[i] = T(k[i]);
    const T inv = T(k[6]);
    ru = T(k[7]);
    rud = k[7];
    for (int s = 0; s < 4; ++s) Su[s] = eps[p * 4 + s] * inv;
    if constexpr (PAR == 3)
      for (int s = 0; s < 4; ++s) Ru[s] = eref[p * 4 + s] * inv;
    for (int s = 0; s < 4; ++s) I[p * 4 + s] = Icur[s];
  }
  // the raw data of the next height are loaded one step ahead, so their
  // latency overlaps the current step's arithmetic
  double kn[8], tn = 0.0;
  T en[4], enr[4];
  auto fetch = [&](int zz) {
    const long long p = pidx(zz);
    const double* k = K8 + p * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) kn[i] = k[i];
#pragma unroll
    for (int s = 0; s < 4; ++s) en[s] = eps[p * 4 + s];
    if constexpr (PAR == 3)
#pragma unroll
      for (int s = 0; s < 4; ++s) enr[s] = eref[p * 4 + s];
    tn = tau[zz];
  };
  if (nz > 1) fetch(z + dz);
  for (int step = 1; step < nz; ++step) {
    const int zc = z + dz;
    const long long p = pidx(zc);
    double kr[8];
    T er[4], err[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) kr[i] = kn[i];
#pragma unroll
    for (int s = 0; s < 4; ++s) er[s] = en[s];
    if constexpr (PAR == 3)
#pragma unroll
      for (int s = 0; s < 4; ++s) err[s] = enr[s];
    const double tzc = tn;
    if (step + 1 < nz) fetch(zc + dz);
    T kc[6], Sc[4];
    for (int i = 0; i < 6; ++i) kc[i] = T(kr[i]);
    const T inv = T(kr[6]);
    const T rc = T(kr[7]);
    for (int s = 0; s < 4; ++s) Sc[s] = er[s] * inv;
    T Rc[4];
    if constexpr (PAR == 3)
      for (int s = 0; s < 4; ++s) Rc[s] = err[s] * inv;
    // the step's optical depth and weights from the FP64 data in FP64 (one
    // rounding each into T): in FP32 the recurrence below then carries the
    // only rounding that accumulates along the ray
    const double xs = 0.5 * (rud + kr[7]) * fabs(tz - tzc) / fabs(m);
    double pu64, pc64, ex64;
    delo_weights<double>(xs, pu64, pc64, ex64);
    const T pu = T(pu64), pc = T(pc64), ex = T(ex64);
    T kv[4], b[4];
    kprime_mul<T>(ku, Icur, kv);
    const bool par = PAR == 1 || (PAR < 0 && scheme == TRAP_FORMAL_DELOPAR);
    if (PAR != 0 && par && step + 1 < nz) {
      // the downwind point's data are the ones just prefetched
      const double xd = 0.5 * (kr[7] + kn[7]) * fabs(tzc - tn) / fabs(m);
      double wM, wO, wP;
      parabolic_weights(0.5 * (double(ru) + kr[7]) * fabs(tz - tzc) / fabs(m), xd, wM, wO, wP);
      const T inP = T(kn[6]);
      for (int s = 0; s < 4; ++s)
        b[s] = ex * Icur[s] - pu * kv[s] + T(wM) * Su[s] + T(wO) * Sc[s] + T(wP) * (en[s] * inP);
    } else if ((PAR == 2 || PAR == 3) && step + 1 < nz) {
      const double hM = 0.5 * (double(ru) + kr[7]) * fabs(tz - tzc) / fabs(m);
      const double hP = 0.5 * (kr[7] + kn[7]) * fabs(tzc - tn) / fabs(m);
      double wM, wC, wO;
      bezier_weights(hM, wM, wC, wO);
      const T inP = T(kn[6]);
      for (int s = 0; s < 4; ++s) {
        T c;
        if constexpr (PAR == 3)
          c = besser_control_lin<T>(Su[s], Sc[s], en[s] * inP, Ru[s], Rc[s], enr[s] * inP, T(hM), T(hP));
        else
          c = besser_control<T>(Su[s], Sc[s], en[s] * inP, T(hM), T(hP));
        b[s] = ex * Icur[s] - pu * kv[s] + T(wM) * Su[s] + T(wC) * c + T(wO) * Sc[s];
      }
    } else {
      for (int s = 0; s < 4; ++s) b[s] = ex * Icur[s] - pu * kv[s] + pu * Su[s] + pc * Sc[s];
    }
    T Inew[4];
    delo_solve<T>(kc, pc, b, Inew);
    for (int s = 0; s < 4; ++s) {
      Icur[s] = Inew[s];
      I[p * 4 + s] = Inew[s];
      Su[s] = Sc[s];
    }
    if constexpr (PAR == 3)
      for (int s = 0; s < 4; ++s) Ru[s] = Rc[s];
    for (int i = 0; i < 6; ++i) ku[i] = kc[i];
    ru = rc;
    rud = kr[7];
    z = zc;
    tz = tzc;
  }
}

template <typename T, int PAR>
__global__ void __launch_bounds__(64) k_formal(int nz, int nd, int nn, const double* __restrict__ mu,
                         const double* __restrict__ tau, const double* __restrict__ K8,
                         const double* __restrict__ WT, const T* __restrict__ eps, T* __restrict__ I,
                         int with_boundary, const T* __restrict__ eref) {
  formal_body<T, PAR>(blockIdx.x, nz, nd, nn, mu, tau, K8, WT, eps, I, with_boundary, PAR, eref);
}

// one launch over several contexts: block b is context r's block b - off[r]
__global__ void __launch_bounds__(64) k_formal_grouped(const GFormal* __restrict__ A, const int* __restrict__ off, int n) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  const GFormal& a = A[lo];
  formal_body<float, -1>(blockIdx.x - off[lo], a.nz, a.nd, a.nn, a.mu, a.tau, a.K8, a.WT, a.eps, a.I, 0, a.scheme);
}

int launch_formal_grouped(hipStream_t s, const GFormal* args, const int* off, int n, int blocks) {
  hipLaunchKernelGGL(k_formal_grouped, dim3(blocks), dim3(64), 0, s, args, off, n);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

// ------------------------------------------------------------------ preconditioner (Sect. 5.2, App. F)
// Local Lambda of the unpolarised formal solution: along each ray the
// response of I at a height to the emissivity at that height is psi_c/eta_I
// of the step that ends there; zero at the first point of the sweep.
__global__ void __launch_bounds__(64) k_pc_local_lambda(int nz, int nd, int nn, const double* __restrict__ mu,
                                                        const double* __restrict__ tau, const double* __restrict__ K8,
                                                        double* __restrict__ L, double2* __restrict__ F) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nd * nn) return;
  const int o = id / nn, n = id % nn;
  const double m = mu[o];
  const bool up = m > 0.0;
  const double amu = fabs(m);
  const long long zs = (long long)nd * nn;
  int z = up ? 0 : nz - 1;
  const int dz = up ? 1 : -1;
  L[(long long)z * zs + id] = 0.0;
  F[(long long)z * zs + id] = make_double2(0.0, 0.0);
  double ru = K8[((long long)z * zs + id) * 8 + 7];
  double iu = K8[((long long)z * zs + id) * 8 + 6];
  for (int step = 1; step < nz; ++step) {
    const int zc = z + dz;
    const long long p = (long long)zc * zs + id;
    const double rc = K8[p * 8 + 7], ic = K8[p * 8 + 6];
    const double x = 0.5 * (ru + rc) * fabs(tau[z] - tau[zc]) / amu;
    double pu, pc, ex;
    delo_weights<double>(x, pu, pc, ex);
    L[p] = pc * ic;
    F[p] = make_double2(ex, pu * iu);
    ru = rc;
    iu = ic;
    z = zc;
  }
}

int launch_pc_local_lambda(trap_ctx* ctx) {
  Problem& P = ctx->pb;
  hipLaunchKernelGGL(k_pc_local_lambda, dim3(ceil_div((long long)P.nd * P.nn, 64)), dim3(64), 0, ctx->stream, P.nz,
                     P.nd, P.nn, P.d_mu, P.d_tau, ctx->pre.d_K, ctx->pre.d_pcL, ctx->pre.d_pcF);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

// Lambda* e for the Stokes-I emissivity e[z][o][n] (scalar DELO-linear steps,
// K' = 0, no incoming radiation) with the block-Jacobi residual fused:
// res = y - x + Lambda* e (y read with stride y_stride).  The step
// coefficients depend on the atmosphere only and are tabulated with the local
// Lambda: I_c = ex I_u + (psi_u/eta_u) e_u + (psi_c/eta_c) e_c, F = (ex,
// psi_u/eta_u), L = psi_c/eta_c.  Nothing but I itself depends on the
// previous step, so the loads of kSweepAhead steps are issued together.
constexpr int kSweepAhead = 4;

__device__ __forceinline__ void pc_lambda_sweep_body(int bx, int nz, int nd, int nn, const double* __restrict__ mu,
                                                     const double2* __restrict__ F, const double* __restrict__ L,
                                                     const double* __restrict__ e, const double* __restrict__ y,
                                                     int y_stride, const double* __restrict__ x,
                                                     double* __restrict__ res) {
  const int id = bx * blockDim.x + threadIdx.x;
  if (id >= nd * nn) return;
  const int o = id / nn;
  const bool up = mu[o] > 0.0;
  const long long zs = (long long)nd * nn;
  const int z0 = up ? 0 : nz - 1;
  const int dz = up ? 1 : -1;
  long long p = (long long)z0 * zs + id;
  double I = 0.0;
  double eu = e[p];
  res[p] = y[p * y_stride] - x[p];
  for (int s0 = 1; s0 < nz; s0 += kSweepAhead) {
    double2 f[kSweepAhead];
    double lc[kSweepAhead], ec[kSweepAhead], yr[kSweepAhead];
    long long pp[kSweepAhead];
#pragma unroll
    for (int j = 0; j < kSweepAhead; ++j) {
      const int st = min(s0 + j, nz - 1);
      pp[j] = (long long)(z0 + dz * st) * zs + id;
      f[j] = F[pp[j]];
      lc[j] = L[pp[j]];
      ec[j] = e[pp[j]];
      yr[j] = y[pp[j] * y_stride] - x[pp[j]];
    }
#pragma unroll
    for (int j = 0; j < kSweepAhead; ++j) {
      if (s0 + j < nz) {
        I = f[j].x * I + f[j].y * eu + lc[j] * ec[j];
        res[pp[j]] = yr[j] + I;
        eu = ec[j];
      }
    }
  }
}

__global__ void __launch_bounds__(64) k_pc_lambda_sweep(int nz, int nd, int nn, const double* __restrict__ mu,
                                                        const double2* __restrict__ F, const double* __restrict__ L,
                                                        const double* __restrict__ e, const double* __restrict__ y,
                                                        int y_stride, const double* __restrict__ x,
                                                        double* __restrict__ res) {
  pc_lambda_sweep_body(blockIdx.x, nz, nd, nn, mu, F, L, e, y, y_stride, x, res);
}

// one launch over several contexts: block b is context r's block b - off[r]
__global__ void __launch_bounds__(64) k_pc_lambda_sweep_grouped(const GPcSweep* __restrict__ A,
                                                                const int* __restrict__ off, int n) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  const GPcSweep& a = A[lo];
  pc_lambda_sweep_body(blockIdx.x - off[lo], a.nz, a.nd, a.nn, a.mu, a.F, a.L, a.e, a.y, a.y_stride, a.x, a.res);
}

int launch_pc_sweep_grouped(hipStream_t s, const GPcSweep* args, const int* off, int n, int blocks) {
  hipLaunchKernelGGL(k_pc_lambda_sweep_grouped, dim3(blocks), dim3(64), 0, s, args, off, n);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

int launch_formal_scalar(trap_ctx* ctx, int prec, const double* e, const double* y, int y_stride, const double* x,
                         double* res) {
  (void)prec;      // the tabulated step coefficients are FP64
  Problem& P = ctx->pb;
  hipLaunchKernelGGL(k_pc_lambda_sweep, dim3(ceil_div((long long)P.nd * P.nn, 64)), dim3(64), 0, ctx->stream, P.nz,
                     P.nd, P.nn, P.d_mu, ctx->pre.d_pcF, ctx->pre.d_pcL, e, y, y_stride, x, res);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

int formal_apply(trap_ctx* ctx, const void* eps, void* I, int with_boundary, int prec) {
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (!ctx->pre.d_K) return fail(TRAP_ESTATE, "precompute not run");
  if (!eps || !I) return fail(TRAP_EINVAL, "null vector");
  Problem& P = ctx->pb;
  const int rays = P.nd * P.nn;
  const int pr = prof_begin(ctx, TRAP_STAGE_FORMAL);
  const int sch = ctx->formal_scheme;
  // BESSER linearised about a reference emissivity (set by the mixed-precision
  // Anderson-Richardson solve for its inner corrections)
  const bool lin = sch == TRAP_FORMAL_BESSER && ctx->besser_ref && ctx->besser_ref_prec == prec;
  if (prec == TRAP_FP64) {
    auto kern = lin ? k_formal<double, 3>
                : (sch == TRAP_FORMAL_BESSER ? k_formal<double, 2>
                   : (sch == TRAP_FORMAL_DELOPAR ? k_formal<double, 1> : k_formal<double, 0>));
    hipLaunchKernelGGL(kern, dim3(ceil_div(rays, 64)), dim3(64), 0, ctx->stream, P.nz, P.nd, P.nn, P.d_mu,
                       P.d_tau, ctx->pre.d_K, P.d_WT, static_cast<const double*>(eps), static_cast<double*>(I),
                       with_boundary, lin ? static_cast<const double*>(ctx->besser_ref) : nullptr);
  } else if (prec == TRAP_FP32) {
    auto kern = lin ? k_formal<float, 3>
                : (sch == TRAP_FORMAL_BESSER ? k_formal<float, 2>
                   : (sch == TRAP_FORMAL_DELOPAR ? k_formal<float, 1> : k_formal<float, 0>));
    hipLaunchKernelGGL(kern, dim3(ceil_div(rays, 64)), dim3(64), 0, ctx->stream, P.nz, P.nd, P.nn, P.d_mu,
                       P.d_tau, ctx->pre.d_K, P.d_WT, static_cast<const float*>(eps), static_cast<float*>(I),
                       with_boundary, lin ? static_cast<const float*>(ctx->besser_ref) : nullptr);
  } else {
    return fail(TRAP_EINVAL, "unknown precision");
  }
  TRAP_HIP(hipGetLastError());
  prof_end(ctx, pr);
  return TRAP_OK;
}

}  // namespace trap
