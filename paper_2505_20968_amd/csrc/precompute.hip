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
// 1.5 Gaussian widths 2 sin(Theta/2) (GL-16 integrates the Gaussian factor
// over such a panel to rounding); the Gaussian factor is cut where
// it falls below e^-43.
#include <cmath>
#include <mutex>
#include <set>
#include <vector>

#include "faddeeva.h"

#include "trap_internal.h"

namespace trap {

__constant__ FaddeevaCoef c_fad;
__constant__ double c_gl_t[16];
__constant__ double c_gl_w[16];
__constant__ double c_gl8_t[8];      // Gauss-Legendre 8 on [0, 1]
__constant__ double c_gl8_w[8];

static constexpr double kSqrtPi = 1.7724538509055160273;
static constexpr double kInvSqrtPi = 0.56418958354775628695;
static constexpr double kPiD = 3.14159265358979323846;

__device__ inline double2 wz(double x, double y) { return faddeeva_w(x, y, c_fad); }

// F(Theta, up, u) in reduced units; pi_limit selects the Theta = pi form.
// The per-row divisors are kept as reciprocals (an FP64 division costs about
// ten vector instructions, a product one).
struct FParams {
  double sG, cG;     // sin(Theta/2), cos(Theta/2) (1, 0 at Theta = pi)
  double inv2sG;     // 1 / (2 sin(Theta/2))
  double inv2cG;     // 1 / (2 cos(Theta/2))
  double a_cG;       // a / cos(Theta/2)
  double inv_sinT;   // 1 / sin(Theta)
  double a;
  bool pi_limit;
};

__device__ inline FParams f_params(double Th, double a) {
  FParams p;
  p.pi_limit = (Th >= kPiD);
  double sG = 1.0, cG = 0.0;
  if (!p.pi_limit) sincos(0.5 * Th, &sG, &cG);
  p.sG = sG;
  p.cG = cG;
  p.inv2sG = 0.5 / sG;
  p.inv2cG = p.pi_limit ? 0.0 : 0.5 / cG;
  p.a_cG = p.pi_limit ? 0.0 : a / cG;
  p.inv_sinT = p.pi_limit ? 0.0 : 1.0 / (2.0 * sG * cG);      // sin(Theta) = 2 sin(Theta/2) cos(Theta/2)
  p.a = a;
  return p;
}

__device__ inline double2 Ffun(const FParams& p, double up, double u) {
  if (p.pi_limit) {
    const double g = exp(-0.25 * (u - up) * (u - up));
    // i / (2 sqrt(pi) (m + i a)) = i (m - i a) / (2 sqrt(pi) (m^2 + a^2))
    const double m = 0.5 * (u + up);
    const double r = g / (2.0 * kSqrtPi * (m * m + p.a * p.a));
    return make_double2(r * p.a, r * m);
  }
  const double q = (u - up) * p.inv2sG;
  const double g = exp(-q * q);
  if (g == 0.0) return make_double2(0.0, 0.0);
  const double2 w = wz((u + up) * p.inv2cG, p.a_cG);
  return make_double2(g * w.x * p.inv_sinT, g * w.y * p.inv_sinT);
}

// F(Theta, up_j, u) at K frequencies up_j of one row, their Faddeeva factors
// evaluated side by side (faddeeva_wk).
template <int K>
__device__ inline void Ffun_k(const FParams& p, const double (&up)[K], double u, double2 (&out)[K]) {
  if (p.pi_limit) {
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] = Ffun(p, up[j], u);
    return;
  }
  double xw[K], g[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double q = (u - up[j]) * p.inv2sG;
    g[j] = exp(-q * q) * p.inv_sinT;
    xw[j] = (u + up[j]) * p.inv2cG;
  }
  double2 w[K];
  faddeeva_wk<K>(xw, p.a_cG, c_fad, w);
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = make_double2(g[j] * w[j].x, g[j] * w[j].y);
}

// ------------------------------------------------------------------ profiles
__global__ void k_profiles(int nz, int nd, int nn, int nt, const double* __restrict__ x,
                           const double* __restrict__ lam, const double* __restrict__ a,
                           const double* __restrict__ ub, const double* __restrict__ st,
                           const double* __restrict__ g, const double* __restrict__ eta0,
                           const double* __restrict__ eps, const double* __restrict__ WT,
                           double c_abs, const double* __restrict__ kc, const double* __restrict__ scc,
                           double* __restrict__ K8, double* __restrict__ epsth) {
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
  // continuum opacity on the diagonal (App. A), relative to the line centre
  const double kz = kc ? kc[(long long)z * nn + n] * eta0[z] : 0.0;
  const double sz = scc ? scc[(long long)z * nn + n] * eta0[z] : 0.0;
  const double etot = eta[0] + kz + sz;
  const double inv = 1.0 / etot;
  double* k = K8 + id * 8;
  k[0] = eta[1] * inv;
  k[1] = eta[2] * inv;
  k[2] = eta[3] * inv;
  k[3] = rho[1] * inv;
  k[4] = rho[2] * inv;
  k[5] = rho[3] * inv;
  k[6] = inv;
  k[7] = etot / eta0[z];
  const double th = eps[z] * WT[z];
  for (int j = 0; j < 4; ++j) epsth[id * 4 + j] = th * eta[j];
  epsth[id * 4] += kz * WT[z];          // LTE continuum emission
}

// ------------------------------------------------------------------ panel integration helper
// Panels of the graded rule on [pa, pb]: swept away from the end nearest the
// core xc (from xc outwards on both sides when it lies inside), each of width
// min(Lg, max(wc, |x - xc|)); a remainder under a quarter of the next width
// joins the last panel.  fn(l, r) is called per panel, in sweep order.
template <typename Fn>
__device__ inline void graded_panels(double pa, double pb, double xc, double wc, double Lg, Fn fn) {
  auto sweep = [&](double start, double end) {
    const double dir = end > start ? 1.0 : -1.0;
    double pos = start;
    int guard = 0;
    while (dir * (end - pos) > 0.0 && guard < 4096) {
      const double dist = fabs(pos - xc);
      double w = fmin(Lg, fmax(wc, dist));
      double nxt = pos + dir * w;
      if (dir * (end - nxt) < 0.25 * w) nxt = end;
      fn(fmin(pos, nxt), fmax(pos, nxt));
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

// Integrate f(x) * t^q (q = 0..nq-1, t = (x - x0)/h) over [pa, pb] with
// Gauss-Legendre 16 on the graded panels.  Accumulates into acc[q] (complex).
template <typename Fn>
__device__ void graded_integrate(double pa, double pb, double xc, double wc, double Lg, double x0,
                                 double invh, int nq, Fn f, double2* acc) {
  graded_panels(pa, pb, xc, wc, Lg, [&](double l, double r) {
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
  });
}

// Orders this wave's LDS writes before its later reads (the other waves of
// the block are not waited for).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// ------------------------------------------------------------------ factor tables (uniform grids)
// On a uniform grid x_k = x_0 + k h with the same 16 Gauss-Legendre nodes t_i
// in every knot interval, the node x' = x_k + h t_i of interval k seen from row
// n has  x_n - x' = h (n - k - t_i)  and  x_n + x' = 2 x_0 + h (n + k + t_i).
// The Gaussian factor of F therefore depends on (d = n - k, i) only and the
// Faddeeva factor on (p = n + k, i) only; both are tabulated per (height,
// Theta[, transition]) so the row integration needs no transcendental calls.
//   G[d + nn - 1 + ntail][i] = exp(-(lam h (d - t_i) / (2 sin(Theta/2)))^2)
//   V[p + ntail][i]          = W(a/cos(Theta/2), (lam (2 x_0 + h (p + t_i)) + 2 s)/(2 cos(Theta/2)))
// (Theta = pi: exp(-(lam h (d - t_i)/2)^2) and i/(2 sqrt(pi)(m + i a)), m = half the sum.)
// The index ranges reach ntail intervals past either end of the grid, so the
// tails of a row's support (where the spline is extended flat) are integrated
// with the same rule over virtual intervals x_0 + k h, k < 0 or k >= nn - 1.
__global__ void k_kernel_tables(int z0, int nth, int nt, int nn, int ntail, double x0, double h,
                                const double* __restrict__ lam, const double* __restrict__ av,
                                const double* __restrict__ st, const double* __restrict__ theta,
                                double* __restrict__ Gt, double2* __restrict__ Vt) {
  const int t = blockIdx.x % nt;
  const int th = (blockIdx.x / nt) % nth;
  const int zl = blockIdx.x / (nt * nth);
  const int z = z0 + zl;
  const double L = lam[z], a = av[z], s = st[z * nt + t], Th = theta[th];
  if (Th == 0.0) return;
  const bool pil = Th >= kPiD;
  const double sG = pil ? 1.0 : sin(0.5 * Th), cG = pil ? 0.0 : cos(0.5 * Th);
  const int nd2 = 2 * nn - 1 + 2 * ntail;
  // this height's rows reach at most ntz intervals past the grid ends (support
  // half-width 13.2 / lam); entries beyond are never read and not computed
  const int ntz = min(ntail, (int)ceil(13.2 / (L * h)) + 2);
  const int e0 = (ntail - ntz) * 16, e1 = nd2 * 16 - e0;
  double2* V = Vt + ((size_t)(zl * nth + th) * nt + t) * nd2 * 16;
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int p = (e >> 4) - ntail, i = e & 15;
    const double xs = 2.0 * x0 + h * (p + c_gl_t[i]);
    if (pil) {
      const double m = 0.5 * (L * xs + 2.0 * s);
      const double d = 2.0 * kSqrtPi * (m * m + a * a);
      V[e] = make_double2(a / d, m / d);
    } else {
      V[e] = wz((L * xs + 2.0 * s) / (2.0 * cG), a / cG);
    }
  }
  if (t == 0) {
    double* G = Gt + (size_t)(zl * nth + th) * nd2 * 16;
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const int dd = (e >> 4) - (nn - 1) - ntail, i = e & 15;
      const double q = L * h * (dd - c_gl_t[i]) / (2.0 * sG);
      G[e] = exp(-q * q);
    }
  }
}

// ------------------------------------------------------------------ R_II kernel rows
// One wave (a 64-thread block) per complex row (z, theta, t, n) of a height
// chunk.  The integral of F against the spline piece on interval k is written
// with the piece's node values v_k, v_{k+1} and second derivatives s_k, s_{k+1}:
//   int F S = mu0 v_k + mu1 (v_{k+1} - v_k)
//           + h^2 (-mu1/3 + mu2/2 - mu3/6) s_k + h^2 (mu3 - mu1)/6 s_{k+1},
// mu_q = int_0^1 F t^q.  Collecting per node gives the row as
//   M[n][m] = L[m] + sum_j Gam[j] Sig[j][m]
// with Sig = d s / d v the spline's second-derivative map; L and Gam are
// accumulated per node in LDS and written here, the product with Sig is one
// batched GEMM (k_sig_gemm, k_sig_gemm_tiles).
constexpr int kPanelCap = 64;         // graded work units listed per window of one row
constexpr double kGl8Ratio = 0.15;    // panels up to this fraction of F's local scale take 8 nodes

// LDS of one row: node accumulators L[nacc], Gam[nacc] (complex) for the
// nodes from the first one the row's support reaches, then one window of the
// graded work-unit list: {left, width}, {t at left, t span} and the packed
// knot interval and node set of each unit.  nacc bounds the node span of
// every row (kernel_row_span); it is nn at most.
__host__ __device__ constexpr size_t kernel_row_lds(int nacc) {
  return ((size_t)nacc * 2 + 2 * kPanelCap) * sizeof(double2) + kPanelCap * sizeof(int);
}

// Largest node span (top - base + 1 in k_kernel_rows) of any kernel row of
// the problem: the rows of Theta = pi have the widest support, 6.6 sigma with
// sigma = 2 / lambda on either side of the row's frequency, and narrower
// supports reach a subset of its knot intervals.  The same interval search
// as the kernel's (upper_interval), on the host.
static int kernel_row_span(const Problem& P) {
  const int nn = P.nn;
  const double* x = P.x.data();
  auto upper = [&](double v) {
    if (v < x[0]) return -1;
    if (v >= x[nn - 1]) return nn - 1;
    int lo = 0, hi = nn - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (x[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
  };
  int span = 1;
  for (int z = 0; z < P.nz; ++z) {
    const double R = 6.6 * (2.0 / P.lam[z]);
    for (int n = 0; n < nn; ++n) {
      const int plo = upper(x[n] - R);
      int phi = upper(x[n] + R);
      if (phi >= 0 && phi < nn - 1 && x[phi] >= x[n] + R) phi -= 1;
      const int base = std::min(std::max(plo, 0), nn - 1), top = std::min(std::max(phi + 1, 0), nn - 1);
      span = std::max(span, top - base + 1);
    }
  }
  return std::min(nn, span + 2);    // two nodes of margin against rounding in the support's ends
}

// Mirror roles of the transitions' kernel rows (Problem::row_role), by value.
constexpr int kMaxRoles = 128;
struct RowRoles {
  int on;                 // 0: every row is computed
  int role[kMaxRoles];
};

// Rows that come from the mirror image of a computed row instead.
__device__ __forceinline__ bool row_mirrored(const RowRoles& R, int t, int n, int nn) {
  if (!R.on) return false;
  const int r = R.role[t];
  return r >= 0 && (r != t || n > nn - 1 - n);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Moments mu_q of knot interval k (or the zeroth moment of a tail, k = -1 or
// nn - 1) into the node accumulators, by the collection formula above.
// The accumulators hold nodes base, base + 1, ... of the row.
__device__ __forceinline__ void add_moments(double2* Lacc, double2* Gacc, const double* __restrict__ x, int nn,
                                            int base, int k, const double2* mu) {
  if (k < 0 || k >= nn - 1) {
    const int m = (k < 0 ? 0 : nn - 1) - base;
    atomicAdd(&Lacc[m].x, mu[0].x);
    atomicAdd(&Lacc[m].y, mu[0].y);
    return;
  }
  const double h = x[k + 1] - x[k], hh = h * h;
  const int m = k - base;
  atomicAdd(&Lacc[m].x, mu[0].x - mu[1].x);
  atomicAdd(&Lacc[m].y, mu[0].y - mu[1].y);
  atomicAdd(&Lacc[m + 1].x, mu[1].x);
  atomicAdd(&Lacc[m + 1].y, mu[1].y);
  atomicAdd(&Gacc[m].x, hh * (-mu[1].x * (1.0 / 3.0) + 0.5 * mu[2].x - mu[3].x * (1.0 / 6.0)));
  atomicAdd(&Gacc[m].y, hh * (-mu[1].y * (1.0 / 3.0) + 0.5 * mu[2].y - mu[3].y * (1.0 / 6.0)));
  atomicAdd(&Gacc[m + 1].x, hh * (mu[3].x - mu[1].x) * (1.0 / 6.0));
  atomicAdd(&Gacc[m + 1].y, hh * (mu[3].y - mu[1].y) * (1.0 / 6.0));
}

// Bound by vector issue (FP64 arithmetic of the Faddeeva and Gaussian
// factors) with the waves' dependency chains in between: occupancy counts.
// Four waves per SIMD fit 128 registers with a few spilled dwords (measured
// faster than three without spills, and than five with more spills); the LDS
// of one row covers only the nodes its support reaches.
__global__ void __launch_bounds__(64, 4) k_kernel_rows(
    long long nrows, int nth, int nt, int nn, int ldm, const double* __restrict__ x,
    const double* __restrict__ lam, const double* __restrict__ av, const double* __restrict__ st,
    const double* __restrict__ theta, double* __restrict__ Lout, double* __restrict__ Gout,
    long long row0, int z0, double h_uniform, const double* __restrict__ Gt,
    const double2* __restrict__ Vt, int ntail, RowRoles roles, int2* __restrict__ gspan, int nacc,
    int span_only) {
  extern __shared__ double2 smem[];    // kernel_row_lds(nacc) bytes
  const int lane = threadIdx.x;
  double2* Lacc = smem;
  double2* Gacc = smem + nacc;
  double2* plw = Gacc + nacc;                    // graded work units: {left, width}
  double2* pts = plw + kPanelCap;                // {t at left, t span} in the piece's knot interval
  int* pk = (int*)(pts + kPanelCap);             // knot interval of the panel
  const long long rl = blockIdx.x;               // row within this launch
  if (rl >= nrows) return;
  const long long row = row0 + rl;
  const int n = row % nn;
  const int t = (row / nn) % nt;
  const int th = (row / ((long long)nn * nt)) % nth;
  const int z = z0 + (int)(row / ((long long)nn * nt * nth));
  // gspan (optional): the node range [x, y] outside which the row's L and
  // Gam are zero (empty: x > y), for the product with Sig; with span_only
  // the row stores hold the row inside that range only (the product reads
  // nothing else), otherwise whole rows
  if (row_mirrored(roles, t, n, nn)) {                          // filled by k_mirror_rows
    if (gspan && lane == 0) gspan[row] = make_int2(nn, -1);
    return;
  }
  const double L = lam[z], a = av[z], s = st[z * nt + t], Th = theta[th];
  // chunk-local row index of the real plane; the imaginary plane follows nn rows later
  const size_t cbase = (size_t)((((size_t)(z - z0) * nth + th) * nt + t) * 2) * nn * ldm;
  const size_t rre = cbase + (size_t)n * ldm, rim = cbase + (size_t)nn * ldm + (size_t)n * ldm;
  if (Th == 0.0) {
    const double2 w = wz(L * x[n] + s, a);
    if (gspan && lane == 0) gspan[row] = make_int2(n, n);
    if (span_only) {
      if (lane == 0) {
        Lout[rre + n] = kSqrtPi * w.x;
        Lout[rim + n] = kSqrtPi * w.y;
        Gout[rre + n] = 0.0;
        Gout[rim + n] = 0.0;
      }
      return;
    }
    for (int m = lane; m < ldm; m += 64) {
      Lout[rre + m] = (m == n) ? kSqrtPi * w.x : 0.0;
      Lout[rim + m] = (m == n) ? kSqrtPi * w.y : 0.0;
      Gout[rre + m] = 0.0;
      Gout[rim + m] = 0.0;
    }
    return;
  }
  const FParams fp = f_params(Th, a);
  const double sigma = 2.0 * fp.sG / L;
  const double R = 6.6 * sigma;
  const double xn = x[n];
  const double lo = xn - R, hi = xn + R;
  const double xc = -xn - 2.0 * s / L;
  const double wc = 2.0 * fmax(fp.cG, a) / L;
  const double Lg = 1.5 * sigma;
  // pieces: -1 left tail, 0..nn-2 knot intervals, nn-1 right tail
  int plo = upper_interval(x, nn, lo);          // -1 if lo < x0
  int phi = upper_interval(x, nn, hi);
  if (phi >= 0 && phi < nn - 1 && x[phi] >= hi) phi -= 1;
  // every node the row's moments reach: knot intervals plo..phi and the
  // tails' end nodes (no more than nacc of them, kernel_row_span)
  const int base = min(max(plo, 0), nn - 1);
  const int top = min(max(phi + 1, 0), nn - 1);
  for (int i = lane; i <= top - base; i += 64) {
    Lacc[i] = make_double2(0.0, 0.0);
    Gacc[i] = make_double2(0.0, 0.0);
  }
  wave_sync();
  const double un = L * xn + s;
  // table fast path: uniform grid, Gaussian resolved by the interval nodes
  const bool fast = (Gt != nullptr) && (sigma >= 0.5 * h_uniform);
  const int nd2 = 2 * nn - 1 + 2 * ntail;
  const double* Grow = fast ? Gt + (size_t)((z - z0) * nth + th) * nd2 * 16 : nullptr;
  const double2* Vrow = fast ? Vt + ((size_t)((z - z0) * nth + th) * nt + t) * nd2 * 16 : nullptr;
  const int g_off = n + nn - 1 + ntail, v_off = n + ntail;     // table row = g_off - k, v_off + k
  const double fscale = L * h_uniform * (fp.pi_limit ? 1.0 : fp.inv_sinT);
  const bool sharp = wc < h_uniform;      // Voigt core narrower than an interval
  // Graded region: where the 16-node rule per interval does not resolve F --
  // the whole support when the Gaussian is narrower than half an interval or
  // the grid is not uniform, else the intervals next to a sharp Voigt core.
  // Its pieces (knot intervals, and the tails past the grid ends) are cut
  // into panels graded towards the core, each taking the 16-node rule or,
  // when it is short against the local scale of F, the 8-node rule; the
  // row's list of eight-node work units is built in LDS (a lane per piece,
  // offsets from a prefix sum over the wave) and the units are spread over
  // the lanes, four lanes per unit and two nodes per lane (their Faddeeva
  // factors evaluated side by side), so the work per lane follows the row's
  // node count and not the number of pieces a lane's share of the support
  // happens to cross.  (Four lanes per unit: with sixteen, rows whose
  // support crosses many short knot intervals reduce over sixteen lanes at
  // nearly every unit; with one, rows of few units leave most lanes idle.)
  // Every other interval of the support takes the table rule, one lane per
  // interval (virtual intervals of width h past the grid ends for the tails,
  // where the spline is extended flat).
  const double x0 = x[0];
  auto xk = [&](int k) { return (k >= 0 && k < nn) ? x[k] : x0 + h_uniform * k; };
  const int kmin = fast ? (int)floor((lo - x0) / h_uniform) : 0;
  const int kmax = fast ? (int)floor((hi - x0) / h_uniform) : 0;
  const bool tail_tab = fast && kmin >= -ntail && kmax <= nn - 2 + ntail;
  // near-core intervals k (real or virtual): x_k - h < xc < x_{k+1} + h
  auto near_core = [&](int k) { return sharp && xc > xk(k) - h_uniform && xc < xk(k + 1) + h_uniform; };
  bool graded = false;
  int kA = 1, kB = 0;                  // table-rule intervals skip [kA, kB]
  double ga = 0.0, gb = 0.0;
  if (!fast || !tail_tab) {
    graded = true;
    ga = lo;
    gb = hi;
    kA = -(1 << 30);
    kB = 1 << 30;
  } else if (sharp) {
    const int kc = (int)floor((xc - x0) / h_uniform);
    kA = 1 << 30;
    kB = -(1 << 30);
    for (int k = kc - 3; k <= kc + 2; ++k)
      if (k >= kmin && k <= kmax && near_core(k)) {
        kA = min(kA, k);
        kB = max(kB, k);
      }
    if (kA <= kB) {
      graded = true;
      ga = fmax(xk(kA), lo);
      gb = fmin(xk(kB + 1), hi);
    }
  }
  // table rule: knot intervals inside the support, one lane per interval
  const int ilo = max(plo, 0), ihi = min(phi, nn - 2);
  if (gspan && lane == 0) gspan[row] = make_int2(base, top);
  for (int p = ilo + lane; fast && p <= ihi; p += 64) {
    if (p >= kA && p <= kB) continue;
    double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const double* g = Grow + (size_t)(g_off - p) * 16;
    const double2* v = Vrow + (size_t)(v_off + p) * 16;
    for (int i = 0; i < 16; ++i) {
      const double f = fscale * c_gl_w[i] * g[i];
      const double2 vv = v[i];
      double tp = f;
      const double ti = c_gl_t[i];
      for (int q = 0; q < 4; ++q) {
        acc[q].x += tp * vv.x;
        acc[q].y += tp * vv.y;
        tp *= ti;
      }
    }
    add_moments(Lacc, Gacc, x, nn, base, p, acc);
  }
  // graded pieces (the region is per row, so every branch here is uniform
  // over the wave)
  if (graded && gb > ga) {
    const int gA = upper_interval(x, nn, ga);        // -1: left tail, nn - 1: right tail
    const int gB = upper_interval(x, nn, gb);
    const int npc = gB - gA + 1;
    // piece k: its clipped range and the map to t of its knot interval
    auto piece = [&](int k, double& pa, double& pb, double& xl, double& invh) {
      pa = (k < 0) ? ga : fmax(ga, x[k]);
      pb = (k >= nn - 1) ? gb : fmin(gb, x[k + 1]);
      const bool inner = k >= 0 && k < nn - 1;
      xl = inner ? x[k] : 0.0;
      invh = inner ? 1.0 / (x[k + 1] - x[k]) : 0.0;
    };
    // Work units of eight nodes: a panel takes the 16-node rule (two units)
    // unless it spans at most kGl8Ratio of the local scale of F, the
    // smaller of the Gaussian's panel cap Lg and the Voigt scale
    // max(wc, distance to the core); there the 8-node rule (one unit) is
    // as accurate.
    auto units_of = [&](double l, double r) -> int {
      const double d = (xc > l && xc < r) ? 0.0 : fmin(fabs(l - xc), fabs(r - xc));
      return (r - l) <= kGl8Ratio * fmin(Lg, fmax(wc, d)) ? 1 : 2;
    };
    int mine = 0;                                    // this lane's unit count
    for (int j = lane; j < npc; j += 64) {
      double pa, pb, xl, invh;
      piece(gA + j, pa, pb, xl, invh);
      graded_panels(pa, pb, xc, wc, Lg, [&](double l, double r) { mine += units_of(l, r); });
    }
    int off = mine;                                  // inclusive prefix over lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(off, d, 64);
      if (lane >= d) off += v;
    }
    const int total = __shfl(off, 63, 64);
    off -= mine;
    const int g = lane >> 2, i4 = lane & 3;        // unit group, first node
    for (int w0 = 0; w0 < total; w0 += kPanelCap) {
      const int w1 = min(total, w0 + kPanelCap);
      // this window's units into LDS: the panel, and its knot interval k and
      // node set (0, 1: the two halves of the 16-node rule, 2: the 8-node
      // rule) packed as (k + 1) << 2 | set
      int e = off;
      for (int j = lane; j < npc && e < w1; j += 64) {
        double pa, pb, xl, invh;
        piece(gA + j, pa, pb, xl, invh);
        graded_panels(pa, pb, xc, wc, Lg, [&](double l, double r) {
          const int nu = units_of(l, r);
          for (int h = 0; h < nu; ++h, ++e) {
            if (e >= w0 && e < w1) {
              plw[e - w0] = make_double2(l, r - l);
              pts[e - w0] = make_double2((l - xl) * invh, (r - l) * invh);
              pk[e - w0] = ((gA + j + 1) << 2) | (nu == 1 ? 2 : h);
            }
          }
        });
      }
      wave_sync();
      // nodes i4 and i4 + 4 of each unit's node set (of the 16-node rule:
      // i4 + 8 and i4 + 12 in its second half) of units g, g + 16, ...:
      // moments summed in registers while the interval stays the same, then
      // over the four lanes of the unit and into the node accumulators
      double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      int cur = -2;
      const int np = w1 - w0;
      auto flush = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int d = 2; d >= 1; d >>= 1) {
            acc[q].x += __shfl_xor(acc[q].x, d, 4);
            acc[q].y += __shfl_xor(acc[q].y, d, 4);
          }
        if (i4 == 0) add_moments(Lacc, Gacc, x, nn, base, cur, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
      };
      for (int pb0 = 0; pb0 < np; pb0 += 16) {
        const int pi = pb0 + g;
        const int code = pi < np ? pk[pi] : 0;
        const int k = pi < np ? (code >> 2) - 1 : -2;
        if (cur != -2 && k != cur) flush();         // uniform over the four lanes of group g
        cur = k;
        if (pi < np) {
          const double2 lw = plw[pi], tt = pts[pi];
          // the lane's nodes, read per unit (registers are what limits occupancy)
          const int set = code & 3;
          const double* nt_ = set == 2 ? c_gl8_t : c_gl_t;
          const double* nw_ = set == 2 ? c_gl8_w : c_gl_w;
          const int i0 = i4 + (set == 1 ? 8 : 0);
          const double tn[2] = {nt_[i0], nt_[i0 + 4]};
          const double wn[2] = {nw_[i0], nw_[i0 + 4]};
          double upn[2];
          double2 Fn[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) upn[u] = L * (lw.x + lw.y * tn[u]) + s;
          Ffun_k<2>(fp, upn, un, Fn);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const double2 v = make_double2(L * Fn[u].x, L * Fn[u].y);
            double tp = lw.y * wn[u];
            const double tq = tt.x + tt.y * tn[u];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              acc[q].x += tp * v.x;
              acc[q].y += tp * v.y;
              tp *= tq;
            }
          }
        }
      }
      if (cur != -2) flush();
      wave_sync();                                   // the list is rewritten by the next window
    }
  }
  // table rule on the tails: virtual intervals past the ends, summed over the wave
  for (int side = 0; side < 2; ++side) {
    const bool present = tail_tab && (side == 0 ? (plo < 0) : (phi >= nn - 1));
    if (!present) continue;
    double2 acc = make_double2(0.0, 0.0);
    const int ka = side == 0 ? kmin : nn - 1, kb = side == 0 ? -1 : kmax;
    for (int k = ka + lane; k <= kb; k += 64) {
      if (k >= kA && k <= kB) continue;
      const double* gg = Grow + (size_t)(g_off - k) * 16;
      const double2* v = Vrow + (size_t)(v_off + k) * 16;
      for (int i = 0; i < 16; ++i) {
        const double f = fscale * c_gl_w[i] * gg[i];
        const double2 vv = v[i];
        acc.x += f * vv.x;
        acc.y += f * vv.y;
      }
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) add_moments(Lacc, Gacc, x, nn, base, side == 0 ? -1 : nn - 1, &acc);
  }
  wave_sync();
  if (span_only) {
    for (int m = base + lane; m <= top; m += 64) {
      const double2 lv = Lacc[m - base], gv = Gacc[m - base];
      Lout[rre + m] = lv.x;
      Lout[rim + m] = lv.y;
      Gout[rre + m] = gv.x;
      Gout[rim + m] = gv.y;
    }
    return;
  }
  for (int m = lane; m < ldm; m += 64) {
    const bool in = m >= base && m <= top;
    const double2 lv = in ? Lacc[m - base] : make_double2(0.0, 0.0);
    const double2 gv = in ? Gacc[m - base] : make_double2(0.0, 0.0);
    Lout[rre + m] = lv.x;
    Lout[rim + m] = lv.y;
    Gout[rre + m] = gv.x;
    Gout[rim + m] = gv.y;
  }
}

// ------------------------------------------------------------------ M = L + Gam Sig on matrix cores
// rows = every (theta, t, plane, n) of a height chunk; K = columns = nn.
// v_mfma_f64_16x16x4: A_in = Gam tile, B_in = Sig tile; lane l holds
// D[(l/16) + 4 r][l % 16].  Block: 4 waves x 16 rows = 64 rows, 8 column tiles.
constexpr int kSigColTiles = 8;
typedef double doublex4_g __attribute__((ext_vector_type(4)));

// Banded output of the kernel rows: chunk-local real row gr = [zl][th][t][c][n]
// of heights z0 + zl goes to its 16-row tile of the store (KStore), which
// keeps the columns of the tile's range; each value is split into an FP32
// value and its FP32 remainder (hi + lo carries the FP64 row to 2^-48).
struct BandOut {
  float* hi = nullptr;
  float* lo = nullptr;
  const TileDesc* td = nullptr;
  int z0 = 0, nth = 0, nt = 0, nn = 0, nq = 0, pad = 0;
};

// store index of (plane p, row n, column col) of (z, theta), or -1 outside its tile's range
__device__ __forceinline__ long long band_at(const BandOut& B, size_t zt, int p, int n, int col) {
  int q, lr;
  row_tile(B.pad, 2 * B.nt, B.nn, p, n, &q, &lr);
  const TileDesc d = B.td[zt * B.nq + q];
  if (col < d.lo || col >= d.hi) return -1;
  return d.off + (long long)lr * (d.hi - d.lo) + (col - d.lo);
}

__device__ __forceinline__ long long band_index(const BandOut& B, long long gr, int col) {
  const int n = (int)(gr % B.nn);
  long long q = gr / B.nn;
  const int p = (int)(q % (2 * B.nt));
  q /= 2 * B.nt;
  const int th = (int)(q % B.nth), zl = (int)(q / B.nth);
  return band_at(B, (size_t)(B.z0 + zl) * B.nth + th, p, n, col);
}

// The stored columns [lo, hi) of chunk-local row gr (< 2^31) and the store
// index of its column 0.
struct BandRow {
  long long base;
  int lo, hi;
};
__device__ __forceinline__ BandRow band_row(const BandOut& B, int gr) {
  const int n = gr % B.nn;
  int q = gr / B.nn;
  const int p = q % (2 * B.nt);
  q /= 2 * B.nt;
  const int th = q % B.nth, zl = q / B.nth;
  const size_t zt = (size_t)(B.z0 + zl) * B.nth + th;
  int tq, lr;
  row_tile(B.pad, 2 * B.nt, B.nn, p, n, &tq, &lr);
  const TileDesc d = B.td[zt * B.nq + tq];
  BandRow r;
  r.lo = d.lo;
  r.hi = d.hi;
  r.base = d.off + (long long)lr * (r.hi - r.lo) - r.lo;
  return r;
}

__device__ __forceinline__ void band_put(const BandOut& B, long long i, double v) {
  const float h = (float)v;
  B.hi[i] = h;
  B.lo[i] = (float)(v - (double)h);
}

__global__ void k_fill_zero(float* __restrict__ a, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = 0.0f;
}

// Rows of a mirrored transition from their mirror images (Problem::row_role):
// M[t][c][n][m] = (c ? -1 : 1) M[src][c][nn-1-n][nn-1-m] for m < nn, zero in
// the padding, over the tile range of each mirrored row, heights [z0, z0 + zc).
// A source entry outside its tile's range is below the band's cut and taken
// as zero.  One wave per row.
__global__ void __launch_bounds__(256) k_mirror_rows(int nth, int nt, int nn, RowRoles roles, BandOut B) {
  // grid z: height in the chunk; y: (angle, transition, plane); x: rows, four per block
  const int plane = blockIdx.y;
  const int c = plane & 1, t = (plane >> 1) % nt, th = (plane >> 1) / nt;
  const int r = roles.role[t];
  if (r < 0) return;
  const int nfirst = r == t ? nn / 2 + (nn & 1) : 0;     // first mirrored row: n > nn-1-n
  const int n = nfirst + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= nn) return;
  const size_t zt = (size_t)(B.z0 + blockIdx.z) * nth + th;
  int q, lr;
  row_tile(B.pad, 2 * nt, nn, 2 * t + c, n, &q, &lr);
  const TileDesc d = B.td[zt * B.nq + q];
  const int lo = d.lo, hi = d.hi;
  const long long dst = d.off + (long long)lr * (hi - lo) - lo;
  for (int m = lo + (threadIdx.x & 63); m < hi; m += 64) {
    float h = 0.0f, l = 0.0f;
    if (m < nn) {
      const long long i = band_at(B, zt, 2 * r + c, nn - 1 - n, nn - 1 - m);
      if (i >= 0) {
        h = B.hi[i];
        l = B.lo[i];
      }
    }
    B.hi[dst + m] = c ? -h : h;
    B.lo[dst + m] = c ? -l : l;
  }
}

__global__ void __launch_bounds__(256) k_sig_gemm(long long nrows, int nn, int ldm,
                                                  const double* __restrict__ Gam,
                                                  const double* __restrict__ Lrow,
                                                  const double* __restrict__ Sig,
                                                  double* __restrict__ M64, float* __restrict__ M32,
                                                  long long out_row0, BandOut bo) {
  constexpr int KC = 16;
  __shared__ double As[64][KC + 1];
  __shared__ double Bs[KC][kSigColTiles * 16 + 4];
  const long long row0 = (long long)blockIdx.x * 64;
  const int col_base = blockIdx.y * kSigColTiles * 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  doublex4_g acc[kSigColTiles];
  for (int j = 0; j < kSigColTiles; ++j)
    for (int r = 0; r < 4; ++r) acc[j][r] = 0.0;
  for (int k0 = 0; k0 < nn; k0 += KC) {
    for (int e = tid; e < 64 * KC; e += 256) {
      const int r = e / KC, kk = e % KC;
      const long long gr = row0 + r;
      const int gk = k0 + kk;
      As[r][kk] = (gr < nrows && gk < nn) ? Gam[gr * ldm + gk] : 0.0;
    }
    for (int e = tid; e < KC * kSigColTiles * 16; e += 256) {
      const int kk = e / (kSigColTiles * 16), c = e % (kSigColTiles * 16);
      const int gk = k0 + kk, gc = col_base + c;
      Bs[kk][c] = (gk < nn && gc < nn) ? Sig[(size_t)gk * nn + gc] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < KC; kk += 4) {
      const double af = As[wave * 16 + lr][kk + lk];
#pragma unroll
      for (int j = 0; j < kSigColTiles; ++j) {
        const double bf = Bs[kk + lk][j * 16 + lr];
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kSigColTiles; ++j) {
    const int col = col_base + j * 16 + lr;
    if (col >= ldm) continue;
    for (int r = 0; r < 4; ++r) {
      const long long gr = row0 + wave * 16 + lk + 4 * r;
      if (gr >= nrows) continue;
      const double v = (col < nn) ? acc[j][r] + Lrow[gr * ldm + col] : 0.0;
      if (bo.hi) {
        const long long i = band_index(bo, gr, col);
        if (i >= 0) band_put(bo, i, v);
        continue;
      }
      const size_t o = (size_t)(out_row0 + gr) * ldm + col;
      if (M64) M64[o] = v;
      if (M32) M32[o] = (float)v;
    }
  }
}

// Persistent form for grids whose Sig fits in LDS: each block stages Sig once
// (rows k padded with zeros to 8 NH, columns to whole 16-column tiles) and its
// 8 waves then stream 16-row tiles of Gam independently (no barrier in the
// loop, so the waves drift apart and one's loads overlap another's products):
// the kernel-row fragments are loaded straight into registers in the permuted
// K order k = 2 (4 h + lk) + jj (two-element vector loads).
template <int NH, int NCT>
__global__ void __launch_bounds__(512, 1) k_sig_gemm_lds(long long nrows, int nn, int ldm,
                                                         const double* __restrict__ Gam,
                                                         const double* __restrict__ Lrow,
                                                         const double* __restrict__ Sig,
                                                         double* __restrict__ M64, float* __restrict__ M32,
                                                         long long out_row0, RowRoles roles, int nt,
                                                         BandOut bo) {
  constexpr int KP = 8 * NH, CP = 16 * NCT, BST = CP + 4;
  extern __shared__ double sgs[];      // [KP][BST]
  for (int e = threadIdx.x; e < KP * CP; e += blockDim.x) {
    const int k = e / CP, c = e - k * CP;
    sgs[k * BST + c] = (k < nn && c < nn) ? Sig[(size_t)k * nn + c] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const long long ntile = (nrows + 15) / 16;
  const long long step = (long long)gridDim.x * 8;
  auto load = [&](long long tile, double2 (&f)[NH]) {
    const long long row = min(tile * 16 + lr, nrows - 1);
    const double* g = Gam + row * ldm;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int k = 2 * (4 * h + lk);
      f[h] = *reinterpret_cast<const double2*>(g + min(k, ldm - 2));
      if (k >= ldm) f[h] = make_double2(0.0, 0.0);
    }
  };
  double2 fa[NH];
  const double* bcol = sgs + 2 * lk * BST + lr;
  for (long long tile = (long long)blockIdx.x * 8 + wave; tile < ntile; tile += step) {
    // tiles of mirrored rows only are left to k_mirror_rows (rows [..][t][c][n])
    if (roles.on) {
      bool all = true;
      for (int i = 0; i < 16 && all; ++i) {
        const long long gr = tile * 16 + i;
        all = gr >= nrows || row_mirrored(roles, (int)((gr / (2LL * nn)) % nt), (int)(gr % nn), nn);
      }
      if (all) continue;
    }
    load(tile, fa);
    doublex4_g acc[NCT];
#pragma unroll
    for (int j = 0; j < NCT; ++j)
      for (int r = 0; r < 4; ++r) acc[j][r] = 0.0;
    // the B values of step h + 1 are read before step h's products are
    // issued; the scheduling barriers keep that order and stop the compiler
    // from hoisting every read of the unrolled loop
    double bc[2][NCT], bx[2][NCT];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int j = 0; j < NCT; ++j) bc[jj][j] = bcol[jj * BST + j * 16];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      if (h + 1 < NH) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int j = 0; j < NCT; ++j) bx[jj][j] = bcol[(8 * (h + 1) + jj) * BST + j * 16];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const double af = jj ? fa[h].y : fa[h].x;
#pragma unroll
        for (int j = 0; j < NCT; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bc[jj][j], acc[j], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (h + 1 < NH) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int j = 0; j < NCT; ++j) bc[jj][j] = bx[jj][j];
      }
    }
    // lane holds D[row lk + 4 r][column 16 j + lr]
    if (bo.hi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long gr = tile * 16 + lk + 4 * r;
        if (gr >= nrows) continue;
        const BandRow br = band_row(bo, (int)gr);
#pragma unroll
        for (int j = 0; j < NCT; ++j) {
          const int col = j * 16 + lr;
          if (col < br.lo || col >= br.hi) continue;
          const double v = (col < nn) ? acc[j][r] + Lrow[gr * ldm + col] : 0.0;
          band_put(bo, br.base + col, v);
        }
      }
      continue;
    }
#pragma unroll
    for (int j = 0; j < NCT; ++j) {
      const int col = j * 16 + lr;
      if (col >= ldm) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long gr = tile * 16 + lk + 4 * r;
        if (gr >= nrows) continue;
        const double v = (col < nn) ? acc[j][r] + Lrow[gr * ldm + col] : 0.0;
        const size_t o = (size_t)(out_row0 + gr) * ldm + col;
        if (M64) M64[o] = v;
        if (M32) M32[o] = (float)v;
      }
    }
  }
}

// Banded M = L + Gam Sig straight into the store, one wave per (height, angle,
// store tile, group of 64 columns): the tile's 16 rows over its column range
// only, with the sum over j restricted to that range too (Gam vanishes outside
// a row's band, which the tile's range contains).  v_mfma_f64_16x16x4 with
// A = Gam fragment (lane l: row l % 16, k l / 16), B = Sig read from global
// memory (the map is shared by every tile and stays in the caches), lane l
// holding D[l / 16 + 4 r][l % 16].  Tiles made only of mirrored rows are left
// to k_mirror_rows.
constexpr int kTileGemmWaves = 4;
__global__ void __launch_bounds__(64 * kTileGemmWaves) k_sig_gemm_tiles(
    int zc, int nth, int nt, int nn, int ldm, int nnp, int nq, const double* __restrict__ Gam,
    const double* __restrict__ Lrow, const double* __restrict__ Sig, BandOut B, RowRoles roles,
    const int2* __restrict__ gspan) {
  // one wave per tile, looping over its 64-column groups (the rows' setup
  // and their Gam, cached after the first group, serve every group)
  const long long tq = (long long)blockIdx.x * kTileGemmWaves + (threadIdx.x >> 6);
  if (tq >= (long long)zc * nth * nq) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int q = (int)(tq % nq);
  const int th = (int)((tq / nq) % nth), zl = (int)(tq / ((long long)nq * nth));
  const int np = 2 * nt;
  const size_t zt = (size_t)(B.z0 + zl) * nth + th;
  const TileDesc d = B.td[zt * nq + q];
  if (d.hi <= d.lo) return;
  const int r0 = tile_row0(B.pad, np, nnp, q);
  // chunk row of tile row i (or -1 past the grid), and whether every row is mirrored
  auto crow = [&](int i) -> long long {
    const int r = r0 + i, p = r / nnp, n = r - p * nnp;
    if (p >= np || n >= nn) return -1;
    return (((long long)zl * nth + th) * np + p) * nn + n;
  };
  if (roles.on) {
    bool all = true;
    for (int i = 0; i < 16 && all; ++i) {
      const int r = r0 + i, p = r / nnp, n = r - p * nnp;
      all = p >= np || n >= nn || row_mirrored(roles, p >> 1, n, nn);
    }
    if (all) return;
  }
  const long long ra = crow(lr);
  const double* grow = Gam + (ra < 0 ? 0 : ra) * ldm;
  // K range: the tile's column range, cut to the union of its rows' Gam
  // spans (Gam is zero outside them, so the sum is the same)
  int klo = d.lo, khi = min(d.hi, nn);
  // complex row of real row r = [zl][th][t][c][n]: [zl][th][t][n]
  auto span_of = [&](long long r) {
    return r < 0 ? make_int2(nn, -1) : gspan[(r / (2LL * nn)) * nn + r % nn];
  };
  // the lane's own row span: the row stores hold nothing valid outside it
  const int2 sp = gspan ? span_of(ra) : make_int2(0, nn - 1);
  if (gspan) {
    int a0 = sp.x, a1 = sp.y;
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
      a0 = min(a0, __shfl_xor(a0, m, 64));
      a1 = max(a1, __shfl_xor(a1, m, 64));
    }
    klo = max(klo, a0);
    khi = min(khi, a1 + 1);
  }
  // the stored rows' spans of this lane's output rows (epilogue)
  int2 si[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) si[r] = gspan ? span_of(crow(lk + 4 * r)) : make_int2(0, nn - 1);
  const int w = d.hi - d.lo;
  for (int c0 = d.lo; c0 < d.hi; c0 += 64) {
    doublex4_g acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int r = 0; r < 4; ++r) acc[j][r] = 0.0;
    // Four K steps per iteration, their loads issued together ahead of the
    // products.  The loads are unconditional (indices clamped into the valid
    // range): a bounds test around each load becomes a branch with a wait in
    // front of its product.  Steps outside the range or the row's span are
    // cancelled through the Gam operand (selected to 0); columns past the
    // grid are not stored.
    const int kmax = max(khi - 1, 0);
    constexpr int KU = 4;
    for (int k0 = klo; k0 < khi; k0 += 4 * KU) {
      double af[KU], bf[KU][4];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + 4 * u + lk;
        const int kc = min(k, kmax);
        // (a select, not a product: outside the span the stores hold stale values)
        const double g = grow[kc];
        af[u] = (ra >= 0 && k < khi && k >= sp.x && k <= sp.y) ? g : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[u][j] = Sig[(size_t)kc * nn + min(c0 + 16 * j + lr, nn - 1)];
      }
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[u], bf[u][j], acc[j], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lk + 4 * r;
      const long long rc = crow(i);
      if (rc < 0) {
        // a row past the grid (padding): zeros, so the store holds no stale values
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = c0 + 16 * j + lr;
          if (col < d.hi) band_put(B, d.off + (long long)i * w + (col - d.lo), 0.0);
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + 16 * j + lr;
        if (col >= d.hi) continue;
        const double lv = Lrow[rc * ldm + min(col, nn - 1)];
        const double v = col < nn ? acc[j][r] + ((col >= si[r].x && col <= si[r].y) ? lv : 0.0) : 0.0;
        band_put(B, d.off + (long long)i * w + (col - d.lo), v);
      }
    }
  }
}

// M = L + Gam Sig for `rrows` real rows; the persistent form when Sig fits
// `roles` (optional): mirror roles of rows laid out [..][t][c][n]; tiles made
// only of mirrored rows are skipped (the persistent form), k_mirror_rows fills them
// whether the persistent LDS form of the product applies (Sig resident in LDS)
static bool sig_gemm_fits_lds(const trap_ctx* ctx) {
  const int nn = ctx->pb.nn, ldm = ctx->pb.ldm;
  const int nh = ldm / 8, nct = (nn + 15) / 16;
  const size_t lds = (size_t)8 * nh * (16 * nct + 4) * sizeof(double);
  return lds <= (size_t)ctx->max_lds && nh >= 1 && nh <= 16 && nct <= 8;
}

int launch_sig_gemm(trap_ctx* ctx, long long rrows, const double* Gam, const double* Lrow, double* M64,
                    float* M32, long long out_row0, const RowRoles* roles = nullptr, const BandOut* band = nullptr) {
  const BandOut bo = band ? *band : BandOut{};
  Problem& P = ctx->pb;
  const int nn = P.nn, ldm = P.ldm;
  const int nh = ldm / 8, nct = (nn + 15) / 16;
  const size_t lds = (size_t)8 * nh * (16 * nct + 4) * sizeof(double);
  auto fallback = [&]() -> int {
    dim3 gg(ceil_div(rrows, 64), ceil_div(ldm, kSigColTiles * 16));
    hipLaunchKernelGGL(k_sig_gemm, gg, dim3(256), 0, ctx->stream, rrows, nn, ldm, Gam, Lrow, P.d_Sig, M64, M32,
                       out_row0, bo);
    TRAP_HIP(hipGetLastError());
    return TRAP_OK;
  };
  if (lds > (size_t)ctx->max_lds || nh < 1 || nh > 16 || nct > 8) return fallback();
  const int grid = (int)std::min<long long>(ctx->n_cu, ceil_div((rrows + 15) / 16, 8));
  const RowRoles rr = roles ? *roles : RowRoles{};
  auto launch = [&](auto kern) -> int {
    if (lds > 64 * 1024)
      TRAP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(512), lds, ctx->stream, rrows, nn, ldm, Gam, Lrow, P.d_Sig, M64, M32,
                       out_row0, rr, P.nt, bo);
    TRAP_HIP(hipGetLastError());
    return TRAP_OK;
  };
#define TRAP_SIG_NCT(NHV)                                              \
  switch (nct) {                                                       \
    case 1: return launch(k_sig_gemm_lds<NHV, 1>);                     \
    case 2: return launch(k_sig_gemm_lds<NHV, 2>);                     \
    case 3: return launch(k_sig_gemm_lds<NHV, 3>);                     \
    case 4: return launch(k_sig_gemm_lds<NHV, 4>);                     \
    case 5: return launch(k_sig_gemm_lds<NHV, 5>);                     \
    case 6: return launch(k_sig_gemm_lds<NHV, 6>);                     \
    case 7: return launch(k_sig_gemm_lds<NHV, 7>);                     \
    default: return launch(k_sig_gemm_lds<NHV, 8>);                    \
  }
  switch (nh) {
    case 1: TRAP_SIG_NCT(1)
    case 2: TRAP_SIG_NCT(2)
    case 3: TRAP_SIG_NCT(3)
    case 4: TRAP_SIG_NCT(4)
    case 5: TRAP_SIG_NCT(5)
    case 6: TRAP_SIG_NCT(6)
    case 7: TRAP_SIG_NCT(7)
    case 8: TRAP_SIG_NCT(8)
    case 9: TRAP_SIG_NCT(9)
    case 10: TRAP_SIG_NCT(10)
    case 11: TRAP_SIG_NCT(11)
    case 12: TRAP_SIG_NCT(12)
    case 13: TRAP_SIG_NCT(13)
    case 14: TRAP_SIG_NCT(14)
    case 15: TRAP_SIG_NCT(15)
    default: TRAP_SIG_NCT(16)
  }
#undef TRAP_SIG_NCT
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
  // tails in u units: int [w(u'+s+ia) - i/(sqrt(pi) u')] du' over (-inf, u0]
  // (lanes 0-31) and [u1, inf) (lanes 32-63), u' = u_edge +- |u_edge| tau/(1 - tau),
  // 32 panels of 16 Gauss-Legendre nodes in tau, one panel per lane
  {
    const int side = lane >> 5, pnl = lane & 31;
    const double uedge = side == 0 ? L * x[0] : L * x[nn - 1];
    const double sgn = side == 0 ? -1.0 : 1.0;
    const double sc = fabs(uedge);
    double2 acc = make_double2(0.0, 0.0);
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
    for (int off = 16; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (pnl == 0) mom[(side == 0 ? 0 : nn) * 4] = acc;
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

// f = (1 - eps) W_T eta_I / num with the line's own eta_I (the continuum takes
// no part in the App. E factor); 1 where the line scatters nothing (eps = 1)
__global__ void k_norm_factor(long long total, int nd, int nn, const double* __restrict__ eps,
                              const double* __restrict__ WT, const double* __restrict__ K8,
                              const double* __restrict__ num, const double* __restrict__ kc,
                              const double* __restrict__ scc, const double* __restrict__ eta0,
                              double* __restrict__ f) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int z = id / ((long long)nd * nn);
  const long long zn = (long long)z * nn + id % nn;
  const double cont = ((kc ? kc[zn] : 0.0) + (scc ? scc[zn] : 0.0)) * eta0[z];
  const double etaI = 1.0 / K8[id * 8 + 6] - cont;
  const double d = num[id * 4];
  f[id] = d != 0.0 ? (1.0 - eps[z]) * WT[z] * etaI / d : 1.0;
}

// ------------------------------------------------------------------ driver
// Angular coefficients of the R_II sum for every pair (o, o') (App. D, Eq.
// eps_sc_II_exp written with explicit dipole vectors):
//   C^{u' l, l'}_ij(o, o') = (c_sc w_o' / pi) sum_u alpha_{u u'} E_i(o; u', u, l') A_j(o'; u, u', l)
// stored per pair in slot-major order as cf[z][p][t = (u', l)][c][l'][i][j] with
// c = 0 holding Re C (multiplies Re W) and c = 1 holding -Im C (multiplies Im W).
// One block per (z, pair); threads over (t, l', i, j).
__global__ void k_coef_table(int nd, int nu, int nl, double c_sc, const double* __restrict__ w,
                             const int* __restrict__ pair_o, const int* __restrict__ pair_slot_dir,
                             const double2* __restrict__ E, const double2* __restrict__ A,
                             const double2* __restrict__ alpha, double* __restrict__ cf64,
                             float* __restrict__ cf32) {
  const int np = nd * nd;
  const int z = blockIdx.x / np, p = blockIdx.x % np;
  const int o = pair_o[p], op = pair_slot_dir[p];
  const int nt = nu * nl;
  const int nitem = nt * nl * 16;
  const double sc = c_sc * w[op] / kPiD;
  for (int e = threadIdx.x; e < nitem; e += blockDim.x) {
    const int j = e & 3, i = (e >> 2) & 3;
    const int lp = (e >> 4) % nl, t = (e >> 4) / nl;
    const int upr = t / nl, l = t % nl;
    const double2* Ez = E + ((size_t)z * nd + o) * 4 * nu * nu * nl;
    const double2* Az = A + ((size_t)z * nd + op) * 4 * nu * nu * nl;
    double re = 0.0, im = 0.0;
    for (int u = 0; u < nu; ++u) {
      const double2 al = alpha[((size_t)z * nu + u) * nu + upr];
      const double2 ee = Ez[((size_t)(i * nu + upr) * nu + u) * nl + lp];
      const double2 aa = Az[((size_t)(j * nu + u) * nu + upr) * nl + l];
      const double2 v = cmul(al, cmul(ee, aa));
      re += v.x;
      im += v.y;
    }
    const size_t base = ((((size_t)z * np + p) * nt + t) * 2) * nl * 16 + lp * 16 + i * 4 + j;
    const size_t off_im = (size_t)nl * 16;
    if (cf64) {
      cf64[base] = sc * re;
      cf64[base + off_im] = -sc * im;
    }
    if (cf32) {
      cf32[base] = (float)(sc * re);
      cf32[base + off_im] = (float)(-sc * im);
    }
  }
}

// Angle-averaged kernels (Sect. 5.2, Eq. R_AA): M[z][0][t][c][n][m] =
// sum_g w_g Mg[z][g][t][c][n][m] over the Theta nodes of one height chunk.
// The angle-averaged class kernels of the preconditioner, dense [zl][t][c][n][ldm].
__global__ void k_theta_average_dense(long long per_z_out, int ng, int zc, const double* __restrict__ w,
                                      const double* __restrict__ Mg, double* __restrict__ M64,
                                      long long out_offset) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= per_z_out * zc) return;
  const long long zl = id / per_z_out, r = id % per_z_out;
  double v = 0.0;
  for (int g = 0; g < ng; ++g) v += w[g] * Mg[(zl * ng + g) * per_z_out + r];
  M64[out_offset + id] = v;
}

// The angle-averaged kernel of heights [z0, z0 + zc) from the rows at the
// Gauss-Legendre angles (scratch [zl][g][t][c][n][ldm]) into the banded store
// (one stored angle).
__global__ void k_theta_average(long long per_z_out, int ng, int zc, int ldm, const double* __restrict__ w,
                                const double* __restrict__ Mg, BandOut B) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= per_z_out * zc) return;
  const long long zl = id / per_z_out, r = id % per_z_out;
  const int col = (int)(r % ldm);
  const long long i = band_index(B, zl * (per_z_out / ldm) + r / ldm, col);
  if (i < 0) return;
  double v = 0.0;
  for (int g = 0; g < ng; ++g) v += w[g] * Mg[(zl * ng + g) * per_z_out + r];
  band_put(B, i, v);
}

// Gauss-Legendre rule of n nodes on [0, 1], nodes ascending: the roots of
// P_n by Newton's method from the usual cosine guesses, weights
// 1 / ((1 - z^2) P_n'(z)^2) (halved with the map from [-1, 1]).
static void gauss_legendre01(int n, double* t, double* w) {
  auto legendre = [n](double z, double* dp) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    *dp = n * (z * p1 - p0) / (z * z - 1.0);
    return p1;
  };
  for (int i = 0; i < n; ++i) {
    double z = cos(kPiD * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      const double dz = legendre(z, &dp) / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    legendre(z, &dp);
    t[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

// The Faddeeva and quadrature constants: computed once per process, copied to
// each device's constant memory once (the copy waits for the device).
static int load_constants(int device) {
  static std::mutex mu;
  static bool coef_ready = false;
  static FaddeevaCoef hc;
  static double gt[16], gw[16], gt8[8], gw8[8];
  static std::set<int> devices_loaded;
  std::lock_guard<std::mutex> lk(mu);
  if (!coef_ready) {
    faddeeva_coefficients(&hc);
    gauss_legendre01(16, gt, gw);
    gauss_legendre01(8, gt8, gw8);
    coef_ready = true;
  }
  if (!devices_loaded.count(device)) {
    TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_fad), &hc, sizeof(hc)));
    TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_t), gt, sizeof(gt)));
    TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), gw, sizeof(gw)));
    TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_t), gt8, sizeof(gt8)));
    TRAP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_w), gw8, sizeof(gw8)));
    devices_loaded.insert(device);
  }
  return TRAP_OK;
}

__global__ void k_faddeeva_eval(int n, const double* __restrict__ v, const double* __restrict__ a,
                                double2* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = wz(v[i], a[i]);
}

int faddeeva_eval(int device, const double* v, const double* a, int n, double* out) {
  TRAP_TRY(load_constants(device));
  double *dv = nullptr, *da = nullptr;
  double2* dout = nullptr;
  const size_t b = (size_t)n * sizeof(double);
  TRAP_HIP(hipMalloc(&dv, b));
  int rc = TRAP_OK;
  if (hipMalloc(&da, b) != hipSuccess || hipMalloc(&dout, 2 * b) != hipSuccess) {
    rc = fail(TRAP_ENOMEM, "faddeeva scratch");
  } else if (hipMemcpy(dv, v, b, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(da, a, b, hipMemcpyHostToDevice) != hipSuccess) {
    rc = fail(TRAP_EDEVICE, "faddeeva upload");
  } else {
    hipLaunchKernelGGL(k_faddeeva_eval, dim3(ceil_div(n, 256)), dim3(256), 0, nullptr, n, dv, da, dout);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = fail(TRAP_EDEVICE, std::string("k_faddeeva_eval: ") + hipGetErrorString(e));
    else if (hipMemcpy(out, dout, 2 * b, hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(TRAP_EDEVICE, "faddeeva download");
  }
  if (dout) TRAP_NOTE(hipFree(dout));
  if (da) TRAP_NOTE(hipFree(da));
  TRAP_NOTE(hipFree(dv));
  return rc;
}

int run_precompute(trap_ctx* ctx, int store_mask) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  hipStream_t s = ctx->stream;
  TRAP_TRY(load_constants(ctx->device));
  const int nz = P.nz, nd = P.nd, nn = P.nn, nt = P.nt, nth = P.nth;
  const int nthr = P.nth_rows;                    // angles at which rows are computed
  const bool aa = P.prd_mode == TRAP_PRD_AA;
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
                     P.d_lam, P.d_a, P.d_ub, P.d_st, P.d_g, P.d_eta0, P.d_eps, P.d_WT, P.c_abs, P.d_kc, P.d_sc,
                     C.d_K, C.d_epsth);
  TRAP_HIP(hipGetLastError());
  // everything the preconditioner tables read exists from here on
  if (!ctx->ev_fork) TRAP_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  TRAP_HIP(hipEventRecord(ctx->ev_fork, s));
  ctx->fork_recorded = true;
  // the banded store holds both precisions at once: FP32 values and their
  // FP32 remainders (the FP64 kernel is their sum); store_mask bit 1 decides
  // only whether the FP32 applies' coefficient tables are built
  const int mask = store_mask | 1;     // FP64 applies always exist (residual, f, b)
  // mirror roles of the transitions' rows: mirrored rows come from their
  // mirror images (the mirror pass takes one grid row per angle, transition
  // and plane)
  RowRoles roles{};
  if (!P.row_role.empty() && nt <= kMaxRoles && (long long)nth * nt * 2 <= 65535) {
    roles.on = 1;
    for (int t = 0; t < nt; ++t) roles.role[t] = P.row_role[t];
  }
  // the tile product writes every row of every tile, the rows past the grid
  // (padding) as zeros, unless mirror roles let it skip tiles
  const bool tile_path = !aa && !sig_gemm_fits_lds(ctx);
  if (!C.d_Mhi) {
    const size_t ne = std::max<size_t>(P.kentries, 2);
    TRAP_TRY(dalloc_t(ctx, &C.d_Mhi, ne));
    TRAP_TRY(dalloc_t(ctx, &C.d_Mlo, ne));
    if (!tile_path || roles.on) {
      // rows of a tile past the grid (padding) are never written otherwise: zero
      const int fg = (int)std::min<long long>(4096, ceil_div((long long)ne, 256));
      hipLaunchKernelGGL(k_fill_zero, dim3(fg), dim3(256), 0, s, C.d_Mhi, (long long)ne);
      hipLaunchKernelGGL(k_fill_zero, dim3(fg), dim3(256), 0, s, C.d_Mlo, (long long)ne);
      TRAP_HIP(hipGetLastError());
    }
  }
  C.store_mask = mask;
  BandOut bo;
  bo.hi = C.d_Mhi;
  bo.lo = C.d_Mlo;
  bo.td = P.d_td;
  bo.nth = nth;
  bo.nt = nt;
  bo.nn = nn;
  bo.nq = P.nq;
  bo.pad = P.qpad;
  const int nacc = kernel_row_span(P);
  const size_t lds = kernel_row_lds(nacc);
  if (lds > 64 * 1024) return fail(TRAP_EINVAL, "frequency grid too large for the kernel precompute");
  // uniform grid -> factor tables, heights in chunks so the tables stay cache sized
  const PrecompLayout lay = precomp_layout(nz, nn, P.ldm, nt, nthr, aa, P.x.data(), P.lam.data());
  const bool uniform = lay.uniform;
  const double h = lay.h;
  const int ntail = lay.ntail, nd2 = lay.nd2, zc_tab = lay.zc_tab;
  const size_t rows_per_z = (size_t)nthr * nt * 2 * nn;
  if (uniform && !C.d_Gt) {
    TRAP_TRY(dalloc_t(ctx, &C.d_Gt, (size_t)zc_tab * nthr * nd2 * 16));
    TRAP_TRY(dalloc_t(ctx, &C.d_Vt, (size_t)zc_tab * nthr * nt * nd2 * 16));
  }
  if (!C.d_Lrow || C.zc_rows < zc_tab) {
    TRAP_TRY(dalloc_t(ctx, &C.d_Lrow, (size_t)zc_tab * rows_per_z * P.ldm));
    TRAP_TRY(dalloc_t(ctx, &C.d_Grow, (size_t)zc_tab * rows_per_z * P.ldm));
    TRAP_TRY(dalloc_t(ctx, &C.d_gspan, (size_t)zc_tab * rows_per_z / 2));
    if (aa) TRAP_TRY(dalloc_t(ctx, &C.d_Mtmp, (size_t)zc_tab * rows_per_z * P.ldm));
    C.zc_rows = zc_tab;
  }
  // the tile product reads each row inside its span only: the kernel rows
  // then write just that part (the other products read whole rows)
  const int span_only = tile_path ? 1 : 0;
  const int pr = prof_begin(ctx, TRAP_STAGE_KERNEL_ROWS);
  for (int z0 = 0; z0 < nz; z0 += zc_tab) {
    const int zc = std::min(zc_tab, nz - z0);
    if (uniform) {
      hipLaunchKernelGGL(k_kernel_tables, dim3(zc * nthr * nt), dim3(256), 0, s, z0, nthr, nt, nn, ntail, P.x[0], h,
                         P.d_lam, P.d_a, P.d_st, P.d_theta_rows, C.d_Gt, C.d_Vt);
      TRAP_HIP(hipGetLastError());
    }
    const long long nrows = (long long)zc * nthr * nt * nn;     // complex rows of this chunk
    const long long chunk = 1 << 22;
    for (long long r0 = 0; r0 < nrows; r0 += chunk) {
      const long long nr = std::min(chunk, nrows - r0);
      hipLaunchKernelGGL(k_kernel_rows, dim3((unsigned)nr), dim3(64), lds, s, nr, nthr, nt,
                         nn, P.ldm, P.d_x,
                         P.d_lam, P.d_a, P.d_st, P.d_theta_rows, C.d_Lrow, C.d_Grow, r0, z0, h,
                         uniform ? C.d_Gt : nullptr, uniform ? C.d_Vt : nullptr, ntail, roles, C.d_gspan, nacc,
                         span_only);
      TRAP_HIP(hipGetLastError());
    }
    const long long rrows = 2 * nrows;                           // real rows (both planes)
    bo.z0 = z0;
    if (tile_path) {
      const long long units = (long long)zc * nth * P.nq;          // tiles
      hipLaunchKernelGGL(k_sig_gemm_tiles, dim3((unsigned)ceil_div(units, kTileGemmWaves)),
                         dim3(64 * kTileGemmWaves), 0, s, zc, nth, nt, nn, P.ldm, P.nnp, P.nq, C.d_Grow,
                         C.d_Lrow, P.d_Sig, bo, roles, C.d_gspan);
      TRAP_HIP(hipGetLastError());
    } else if (!aa) {
      TRAP_TRY(launch_sig_gemm(ctx, rrows, C.d_Grow, C.d_Lrow, nullptr, nullptr, 0LL, &roles, &bo));
    } else {
      // rows at the Gauss-Legendre angles into the scratch store, then their weighted sum
      TRAP_TRY(launch_sig_gemm(ctx, rrows, C.d_Grow, C.d_Lrow, C.d_Mtmp, (float*)nullptr, 0LL));
      const long long per_z_out = (long long)nt * 2 * nn * P.ldm;
      hipLaunchKernelGGL(k_theta_average, dim3(ceil_div(per_z_out * zc, 256)), dim3(256), 0, s, per_z_out, nthr,
                         zc, P.ldm, P.d_theta_rw, C.d_Mtmp, bo);
      TRAP_HIP(hipGetLastError());
    }
    if (roles.on) {
      const dim3 mg((unsigned)ceil_div(nn, 4), (unsigned)(nth * nt * 2), (unsigned)zc);
      hipLaunchKernelGGL(k_mirror_rows, mg, dim3(256), 0, s, nth, nt, nn, roles, bo);
      TRAP_HIP(hipGetLastError());
    }
  }
  prof_end(ctx, pr);
  hipLaunchKernelGGL(k_r3_rows, dim3(nz * nt), dim3(64), (size_t)(nn + 1) * 4 * sizeof(double2), s, nt, nn, P.d_x,
                     P.d_P, P.d_lam, P.d_a,
                     P.d_st, C.d_r3, C.d_prof);
  TRAP_HIP(hipGetLastError());
  {
    const size_t ncf = (size_t)nz * nd * nd * nt * 2 * P.nl * 16;
    if ((mask & 1) && !C.d_cf64) TRAP_TRY(dalloc_t(ctx, &C.d_cf64, ncf));
    if ((mask & 2) && !C.d_cf32) TRAP_TRY(dalloc_t(ctx, &C.d_cf32, ncf));
    hipLaunchKernelGGL(k_coef_table, dim3(nz * nd * nd), dim3(64), 0, s, nd, P.nu, P.nl, P.c_sc, P.d_w,
                       P.d_pair_o, P.d_pair_dir, P.d_E, P.d_A, P.d_alpha, (mask & 1) ? C.d_cf64 : nullptr,
                       (mask & 2) ? C.d_cf32 : nullptr);
    TRAP_HIP(hipGetLastError());
  }
  C.done = true;
  // normalisation factor f: one unnormalised FP64 Sigma apply on (W_T, 0, 0, 0)
  TRAP_TRY(ensure_work(ctx, TRAP_FP64));
  double* flat = ctx->wk.tmp64;
  double* num = ctx->wk.r;
  hipLaunchKernelGGL(k_flat_field, dim3(ceil_div(npt, 256)), dim3(256), 0, s, npt, nd, nn, P.d_WT, flat);
  TRAP_HIP(hipGetLastError());
  // (its contraction reduces to the stored rows' sums: k_flat_contract)
  ctx->flat_field = 1;
  const int rcn = sigma_apply(ctx, flat, num, TRAP_FP64, 0, 0);
  ctx->flat_field = 0;
  TRAP_TRY(rcn);
  hipLaunchKernelGGL(k_norm_factor, dim3(ceil_div(npt, 256)), dim3(256), 0, s, npt, nd, nn, P.d_eps,
                     P.d_WT, C.d_K, num, P.d_kc, P.d_sc, P.d_eta0, C.d_f);
  TRAP_HIP(hipGetLastError());
  // right-hand side b = Lambda eps_th + t
  TRAP_TRY(formal_apply(ctx, C.d_epsth, C.d_b, 1, TRAP_FP64));
  return TRAP_OK;
}

// ------------------------------------------------------------------ preconditioner tables
// Comoving coupling of the preconditioner (Sect. 5.2): for height z and row n,
//   Phi[z][n][m] = sum_k (cr_k M_k^re[n][m] + ci_k M_k^im[n][m])
//                + sum_{a,b} Re[X1_ab P_a(n) R_b(m) + X2_ab conj(P_a(n)) R_b(m)
//                               + X3_ab P_a(n) conj(R_b(m)) + X4_ab conj(P_a(n)) conj(R_b(m))]
// with the angle-averaged kernels M_k, R_III rows R_k and profiles P_k of the
// zero-field transition classes.
__global__ void __launch_bounds__(128) k_pc_phi(int nk, int nn, int ldm, const double* __restrict__ M,
                                                const double* __restrict__ cr, const double* __restrict__ ci,
                                                const double2* __restrict__ X, const double2* __restrict__ R3,
                                                const double2* __restrict__ prof, double* __restrict__ Phi) {
  const int z = blockIdx.x / nn, n = blockIdx.x % nn;
  for (int m = threadIdx.x; m < nn; m += blockDim.x) {
    double v = 0.0;
    for (int k = 0; k < nk; ++k) {
      const size_t base = ((size_t)(z * nk + k) * 2) * nn * ldm + (size_t)n * ldm + m;
      v += cr[z * nk + k] * M[base] + ci[z * nk + k] * M[base + (size_t)nn * ldm];
    }
    const double2* Xz = X + (size_t)z * 4 * nk * nk;
    for (int a = 0; a < nk; ++a) {
      const double2 pa = prof[((size_t)z * nk + a) * nn + n];
      for (int b = 0; b < nk; ++b) {
        const double2 rb = R3[((size_t)z * nk + b) * nn + m];
        const int ab = a * nk + b;
        v += cmul(Xz[ab], cmul(pa, rb)).x + cmul(Xz[nk * nk + ab], cmul(cconj(pa), rb)).x +
             cmul(Xz[2 * nk * nk + ab], cmul(pa, cconj(rb))).x +
             cmul(Xz[3 * nk * nk + ab], cmul(cconj(pa), cconj(rb))).x;
      }
    }
    Phi[((size_t)z * nn + n) * nn + m] = v;
  }
}

// Column m of A_z = sum_Omega w_Omega U_Omega Lambda_zz(Omega) V_Omega Phi_z,
// directions of equal Doppler shift taken together: the column of Phi is
// interpolated to the class's observer grid (x_n + u_b/lam), weighted by the
// summed w Lambda_zz of the class, interpolated back to the comoving grid
// (x_m - u_b/lam) and accumulated.  One block per (z, m).
__global__ void __launch_bounds__(128) k_pc_A(int nd, int nn, const double* __restrict__ x,
                                              const double* __restrict__ SigT, const double* __restrict__ lam,
                                              const double* __restrict__ w, const int* __restrict__ mem,
                                              const int* __restrict__ moff, const int* __restrict__ ncls,
                                              const double* __restrict__ cub,
                                              const double* __restrict__ L, const double* __restrict__ Phi,
                                              double* __restrict__ A) {
  extern __shared__ double sh[];
  double* ph = sh;
  double* sp = sh + nn;
  double* g = sh + 2 * nn;
  double* sg = sh + 3 * nn;
  double* acc = sh + 4 * nn;
  const int z = blockIdx.x / nn, m = blockIdx.x % nn;
  const double* Pz = Phi + (size_t)z * nn * nn;
  for (int j = threadIdx.x; j < nn; j += blockDim.x) {
    ph[j] = Pz[(size_t)j * nn + m];
    acc[j] = 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    double a = 0.0;
    for (int j = 0; j < nn; ++j) a += SigT[(size_t)j * nn + i] * ph[j];
    sp[i] = a;
  }
  __syncthreads();
  const double Lz = lam[z];
  for (int c = 0; c < ncls[z]; ++c) {
    const double shf = cub[(size_t)z * nd + c] / Lz;
    const int k0 = moff[(size_t)z * (nd + 1) + c], k1 = moff[(size_t)z * (nd + 1) + c + 1];
    for (int n = threadIdx.x; n < nn; n += blockDim.x) {
      double d = 0.0;
      for (int k = k0; k < k1; ++k) {
        const int o = mem[(size_t)z * nd + k];
        d += w[o] * L[((size_t)z * nd + o) * nn + n];
      }
      g[n] = d * spline_at(x, nn, ph, sp, x[n] + shf);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
      double a = 0.0;
      for (int j = 0; j < nn; ++j) a += SigT[(size_t)j * nn + i] * g[j];
      sg[i] = a;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nn; i += blockDim.x) acc[i] += spline_at(x, nn, g, sg, x[i] - shf);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nn; i += blockDim.x) A[((size_t)z * nn + i) * nn + m] = acc[i];
}

// C_z = Phi_z (Id - A_z)^-1 from (Id - A_z)^T C_z^T = Phi_z^T: Gauss-Jordan
// elimination with partial pivoting on [ (Id - A_z)^T | Phi_z^T ] (rows of
// 2 nn entries in global scratch), one block per height.
constexpr int kInvThreads = 1024;

__global__ void __launch_bounds__(kInvThreads) k_pc_invert(int nn, const double* __restrict__ A,
                                                           const double* __restrict__ Phi, double* __restrict__ aug,
                                                           double* __restrict__ C) {
  __shared__ double rv[kInvThreads / 64];
  __shared__ int ri[kInvThreads / 64];
  __shared__ double fac[1024];
  const int z = blockIdx.x, tid = threadIdx.x;
  const int w2 = 2 * nn;
  double* G = aug + (size_t)z * nn * w2;
  const double* Az = A + (size_t)z * nn * nn;
  const double* Pz = Phi + (size_t)z * nn * nn;
  for (int e = tid; e < nn * w2; e += blockDim.x) {
    const int i = e / w2, j = e % w2;
    G[e] = j < nn ? (i == j ? 1.0 : 0.0) - Az[(size_t)j * nn + i] : Pz[(size_t)(j - nn) * nn + i];
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  for (int k = 0; k < nn; ++k) {
    // pivot: the largest |G[i][k]|, i >= k (smallest i on ties): within each
    // wave by shuffles, then across the waves
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < nn; i += blockDim.x) {
      const double v = fabs(G[(size_t)i * w2 + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wv] = best;
      ri[wv] = bi;
    }
    __syncthreads();
    int p = ri[0];
    double pb = rv[0];
    for (int r = 1; r < nwv; ++r)
      if (rv[r] > pb || (rv[r] == pb && ri[r] < p)) {
        pb = rv[r];
        p = ri[r];
      }
    if (p != k)
      for (int j = k + tid; j < w2; j += blockDim.x) {
        const double t = G[(size_t)k * w2 + j];
        G[(size_t)k * w2 + j] = G[(size_t)p * w2 + j];
        G[(size_t)p * w2 + j] = t;
      }
    __syncthreads();
    const double inv = 1.0 / G[(size_t)k * w2 + k];
    __syncthreads();
    for (int j = k + tid; j < w2; j += blockDim.x) G[(size_t)k * w2 + j] *= inv;
    for (int i = tid; i < nn; i += blockDim.x) fac[i] = (i == k) ? 0.0 : G[(size_t)i * w2 + k];
    __syncthreads();
    const int wk = w2 - k - 1;
    for (long long e = tid; e < (long long)nn * wk; e += blockDim.x) {
      const int i = (int)(e / wk), j = k + 1 + (int)(e % wk);
      if (i != k) G[(size_t)i * w2 + j] -= fac[i] * G[(size_t)k * w2 + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nn * nn; e += blockDim.x) {
    const int n = e / nn, m = e % nn;
    C[(size_t)z * nn * nn + e] = G[(size_t)m * w2 + nn + n];
  }
}

static int precompute_precond_body(trap_ctx* ctx) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  hipStream_t s = ctx->stream;
  if (!ctx->has_problem || !C.done) return fail(TRAP_ESTATE, "precompute not run");
  const int nz = P.nz, nd = P.nd, nn = P.nn, ldm = P.ldm, nk = P.pc_nk, ng = 25;
  if (nn > 1024) return fail(TRAP_EINVAL, "frequency grid too large for the preconditioner (n_nu > 1024)");
  if (nk < 1) return fail(TRAP_ESTATE, "no zero-field transitions");
  TRAP_TRY(load_constants(ctx->device));
  const size_t lds_row = (size_t)(nn + 1) * 4 * sizeof(double2);
  if (lds_row > 64 * 1024) return fail(TRAP_EINVAL, "frequency grid too large for the kernel precompute");
  const PrecompLayout lay = precomp_layout(nz, nn, ldm, nk, ng, true, P.x.data(), P.lam.data());
  const size_t rows_per_z = (size_t)ng * nk * 2 * nn;
  // row scratch in height chunks of at most 32 MB per buffer
  const int zc_max = (int)std::max<size_t>(1, std::min<size_t>(nz, (size_t(32) << 20) / (rows_per_z * ldm * 8)));
  if (!C.d_pcPhi) {
    std::vector<double> st((size_t)nz * nk), gt, gw, th(ng), rw(ng);
    for (int z = 0; z < nz; ++z)
      for (int k = 0; k < nk; ++k) st[(size_t)z * nk + k] = P.pc_dE[k] / P.dnuD[z];
    gauss_legendre_unit(ng, gt, gw);
    for (int g = 0; g < ng; ++g) {
      th[g] = kPiD * gt[g];
      rw[g] = kPiD * gw[g] * 0.5 * std::sin(th[g]);
    }
    UploadBatch up;
    up.add(&C.d_pcSt, st);
    up.add(&C.d_pcCr, P.pc_cr);
    up.add(&C.d_pcCi, P.pc_ci);
    up.add(&C.d_pcX, P.pc_X);
    up.add(&C.d_pcMem, P.pc_mem);
    up.add(&C.d_pcMoff, P.pc_moff);
    up.add(&C.d_pcNcls, P.pc_ncls);
    up.add(&C.d_pcCub, P.pc_cub);
    up.add(&C.d_pcTheta, th);
    up.add(&C.d_pcRw, rw);
    TRAP_TRY(up.commit(ctx));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcPhi, (size_t)nz * nn * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcC, (size_t)nz * nn * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcL, (size_t)nz * nd * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcF, (size_t)nz * nd * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcA, (size_t)nz * nn * nn * 3));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcM, (size_t)nz * nk * 2 * nn * ldm));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcR3, (size_t)nz * nk * nn));
    TRAP_TRY(dalloc_t(ctx, &C.d_pcProf, (size_t)nz * nk * nn));
  }
  // angle-averaged kernels of the zero-field classes: rows at the
  // Gauss-Legendre angles, then their weighted sum (as the AA precompute)
  double *Gt = nullptr, *Lrow = nullptr, *Grow = nullptr, *Mtmp = nullptr;
  double2* Vt = nullptr;
  if (lay.uniform) {
    TRAP_TRY(dalloc_t(ctx, &Gt, (size_t)zc_max * ng * lay.nd2 * 16));
    TRAP_TRY(dalloc_t(ctx, &Vt, (size_t)zc_max * ng * nk * lay.nd2 * 16));
  }
  TRAP_TRY(dalloc_t(ctx, &Lrow, (size_t)zc_max * rows_per_z * ldm));
  TRAP_TRY(dalloc_t(ctx, &Grow, (size_t)zc_max * rows_per_z * ldm));
  TRAP_TRY(dalloc_t(ctx, &Mtmp, (size_t)zc_max * rows_per_z * ldm));
  const int nacc = kernel_row_span(P);
  const size_t lds_kr = kernel_row_lds(nacc);
  if (lds_kr > 64 * 1024) return fail(TRAP_EINVAL, "frequency grid too large for the kernel precompute");
  const long long per_z_out = (long long)nk * 2 * nn * ldm;
  for (int z0 = 0; z0 < nz; z0 += zc_max) {
    const int zc = std::min(zc_max, nz - z0);
    if (lay.uniform) {
      hipLaunchKernelGGL(k_kernel_tables, dim3(zc * ng * nk), dim3(256), 0, s, z0, ng, nk, nn, lay.ntail, P.x[0],
                         lay.h, P.d_lam, P.d_a, C.d_pcSt, C.d_pcTheta, Gt, Vt);
      TRAP_HIP(hipGetLastError());
    }
    const long long nrows = (long long)zc * ng * nk * nn;
    hipLaunchKernelGGL(k_kernel_rows, dim3((unsigned)nrows), dim3(64), lds_kr, s, nrows, ng,
                       nk, nn, ldm, P.d_x, P.d_lam, P.d_a, C.d_pcSt, C.d_pcTheta, Lrow, Grow, 0LL, z0, lay.h,
                       lay.uniform ? Gt : nullptr, lay.uniform ? Vt : nullptr, lay.ntail, RowRoles{}, nullptr, nacc, 0);
    TRAP_HIP(hipGetLastError());
    TRAP_TRY(launch_sig_gemm(ctx, 2 * nrows, Grow, Lrow, Mtmp, (float*)nullptr, 0LL));
    hipLaunchKernelGGL(k_theta_average_dense, dim3(ceil_div(per_z_out * zc, 256)), dim3(256), 0, s, per_z_out, ng,
                       zc, C.d_pcRw, Mtmp, C.d_pcM, (long long)z0 * per_z_out);
    TRAP_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_r3_rows, dim3(nz * nk), dim3(64), lds_row, s, nk, nn, P.d_x, P.d_P, P.d_lam, P.d_a, C.d_pcSt,
                     C.d_pcR3, C.d_pcProf);
  TRAP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pc_phi, dim3(nz * nn), dim3(128), 0, s, nk, nn, ldm, C.d_pcM, C.d_pcCr, C.d_pcCi, C.d_pcX,
                     C.d_pcR3, C.d_pcProf, C.d_pcPhi);
  TRAP_HIP(hipGetLastError());
  TRAP_TRY(launch_pc_local_lambda(ctx));
  hipLaunchKernelGGL(k_pc_A, dim3(nz * nn), dim3(128), 5 * nn * sizeof(double), s, nd, nn, P.d_x, P.d_SigT, P.d_lam,
                     P.d_w, C.d_pcMem, C.d_pcMoff, C.d_pcNcls, C.d_pcCub, C.d_pcL, C.d_pcPhi, C.d_pcA);
  TRAP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pc_invert, dim3(nz), dim3(kInvThreads), 0, s, nn, C.d_pcA, C.d_pcPhi,
                     C.d_pcA + (size_t)nz * nn * nn, C.d_pcC);
  TRAP_HIP(hipGetLastError());
  C.pc_ncmax = 1;
  for (int z = 0; z < nz; ++z) C.pc_ncmax = std::max(C.pc_ncmax, P.pc_ncls[z]);
  C.pc_done = true;
  return TRAP_OK;
}

// The tables need the problem tables and the propagation matrix only, so
// they are built on the context's side stream from the fork event of the
// precompute on, overlapping its kernel rows and normalisation; the
// context's stream waits for them before anything enqueued later.
int run_precompute_precond(trap_ctx* ctx) {
  if (!ctx->has_problem || !ctx->pre.done || !ctx->fork_recorded) return fail(TRAP_ESTATE, "precompute not run");
  if (!ctx->side) {
    TRAP_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    TRAP_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  TRAP_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
  hipStream_t main = ctx->stream;
  ctx->stream = ctx->side;
  const int rc = precompute_precond_body(ctx);
  ctx->stream = main;
  TRAP_HIP(hipEventRecord(ctx->ev_join, ctx->side));
  TRAP_HIP(hipStreamWaitEvent(main, ctx->ev_join, 0));
  return rc;
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
