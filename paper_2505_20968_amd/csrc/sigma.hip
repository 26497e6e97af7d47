// Sigma apply (paper Sect. 4.1-4.3, App. D, App. E), per precision T:
//   1. comoving field Ibar(u_m) = S[I](u_m - u_b(Omega'))          k_spline_shift
//   2. W_{t,j}(slot, n) = sum_m M[z][theta(slot)][t][n][m] Ibar_j(dir(slot), m)
//                                                               k_contract
//   3. R_III incoming factors Y and their angular sums X           k_r3_Y, k_r3_X
//   4. eps_bar_i(o, n; l, l') = Re sum_{o', u'} sum_j C_ij W_{u' l, j}
//        + R_III outer product                                     k_angular
//      with C^{u' l, l'}_ij(o, o') = (c_sc w_o'/pi) sum_u alpha_{u u'}
//        E_i(o; u', u, l') A_j(o'; u, u', l)  (the [G(u') + G(u)*] pairing of
//      Eq. RQIIKKp folded into a real part)
//   5. eps = sum_{l,l'} S[eps_bar(.; l, l')](u_n + u_b(Omega) + u_{l l'}),
//      times f on Stokes I, plus eps_th if asked                  k_spline_shift
// Heights are processed in chunks so the W intermediate of a chunk stays
// bounded (and cache resident on the 256 MB Infinity Cache for small chunks).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "trap_internal.h"

namespace trap {

static constexpr double kInvPi = 0.31830988618379067154;

// Non-oscillatory value at xs in [x_lo, x_lo+1] of the four Stokes columns of
// v [nn][4] (the blend of the two three-node quadratics documented with
// trap_set_interpolation): both quadratics pass through the interval's end
// values, q_k = v_lo + d (xs - x_lo) + D_k (xs - x_lo)(xs - x_lo+1), and
// their second differences are blended with weights that follow the smoother
// stencil.  The first and last intervals take their one quadratic.
__device__ inline void weno4_point(const double* __restrict__ x, int nn, const double* v, int lo, double xs,
                                   double* val) {
  const double x0 = x[lo], x1 = x[lo + 1];
  const double h = x1 - x0;
  const double bub = (xs - x0) * (xs - x1);
  const bool left = lo == 0, right = lo == nn - 2;
  const double xm = left ? 0.0 : x[lo - 1], xp = right ? 0.0 : x[lo + 2];
  const double g1 = (left || right) ? 0.0 : (xp - xs) / (xp - xm);
  for (int q = 0; q < 4; ++q) {
    const double v0 = v[4 * lo + q], v1 = v[4 * (lo + 1) + q];
    const double d = (v1 - v0) / h;
    const double lin = v0 + d * (xs - x0);
    if (left || right) {
      // the stencil that stays on the grid: {0, 1, 2} or {nn-3, nn-2, nn-1}
      const int a = left ? 0 : nn - 3;
      const double fa = v[4 * a + q], fb = v[4 * (a + 1) + q], fc = v[4 * (a + 2) + q];
      const double D = ((fc - fb) / (x[a + 2] - x[a + 1]) - (fb - fa) / (x[a + 1] - x[a])) / (x[a + 2] - x[a]);
      val[q] = lin + D * bub;
      continue;
    }
    const double vm = v[4 * (lo - 1) + q], vp = v[4 * (lo + 2) + q];
    const double D1 = (d - (v0 - vm) / (x0 - xm)) / (x1 - xm);
    const double D2 = ((vp - v1) / (xp - x1) - d) / (xp - x0);
    const double b1 = (h * h * D1) * (h * h * D1), b2 = (h * h * D2) * (h * h * D2);
    const double e = 1e-12 * (vm * vm + v0 * v0 + v1 * v1 + vp * vp) * 0.25 + 1e-150;
    const double a1 = g1 / ((e + b1) * (e + b1)), a2 = (1.0 - g1) / ((e + b2) * (e + b2));
    const double w1 = a1 / (a1 + a2);
    val[q] = lin + (w1 * D1 + (1.0 - w1) * D2) * bub;
  }
}


// ------------------------------------------------------------------ spline evaluation
// out[z][o][n][s] (+)= S[in[z][o][:][s]](x_n + shift) for one (l, l') class,
// flat extension outside [x_0, x_{nn-1}];  shift (x units) =
// (ub_sign * ub[z][o] + sll[z][cls]) / lam[z].  One block per (z, o): the
// column goes to LDS, the spline's second derivatives s = Sig v (Sig^T stored,
// so the reads are coalesced) are formed once, then every frequency evaluates
//   S(x) = (1-t) v_k + t v_{k+1} + h^2 [((1-t)^3 - (1-t)) s_k + (t^3 - t) s_{k+1}] / 6.
// Optionally multiplies Stokes I by f and adds eps_th.
template <typename T>
__device__ __forceinline__ void spline_shift_body(
    int bx, double* spl, int nz0, int nd, int nn, const double* __restrict__ x, const double* __restrict__ SigT,
    const double* __restrict__ lam, const double* __restrict__ ub, double ub_sign,
    const double* __restrict__ sll, int ncls, int cls, const T* __restrict__ in, long long in_z_stride,
    long long in_o_stride, T* __restrict__ out, int accumulate, const double* __restrict__ f,
    const double* __restrict__ epsth, int weno) {
  double* v = spl;               // [nn][4]
  double* sd = spl + 4 * nn;     // [nn][4]
  const int zl = bx / nd, o = bx % nd;
  const int z = nz0 + zl;
  const double L = lam[z];
  double sh = ub_sign * ub[(long long)z * nd + o];
  if (sll) sh += sll[(long long)z * ncls + cls];
  const T* src = in + zl * in_z_stride + o * in_o_stride;
  const bool shifted = sh != 0.0;
  if (shifted) {
    for (int e = threadIdx.x; e < 4 * nn; e += blockDim.x) v[e] = (double)src[e];
    __syncthreads();
    // the spline's second derivatives (the non-oscillatory blend needs none)
    for (int m = threadIdx.x; m < nn && !weno; m += blockDim.x) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int j = 0; j < nn; ++j) {
        const double g = SigT[(size_t)j * nn + m];
        a0 += g * v[4 * j];
        a1 += g * v[4 * j + 1];
        a2 += g * v[4 * j + 2];
        a3 += g * v[4 * j + 3];
      }
      sd[4 * m] = a0;
      sd[4 * m + 1] = a1;
      sd[4 * m + 2] = a2;
      sd[4 * m + 3] = a3;
    }
    __syncthreads();
  }
  const double dx = sh / L;
  for (int n = threadIdx.x; n < nn; n += blockDim.x) {
    double val[4];
    if (!shifted) {
      for (int q = 0; q < 4; ++q) val[q] = (double)src[n * 4 + q];
    } else {
      const double xs = x[n] + dx;
      if (xs <= x[0]) {
        for (int q = 0; q < 4; ++q) val[q] = v[q];
      } else if (xs >= x[nn - 1]) {
        for (int q = 0; q < 4; ++q) val[q] = v[4 * (nn - 1) + q];
      } else {
        int lo = 0, hi = nn - 1;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (x[mid] <= xs) lo = mid; else hi = mid;
        }
        if (weno) {
          weno4_point(x, nn, v, lo, xs, val);
        } else {
          const double h = x[lo + 1] - x[lo];
          const double t = (xs - x[lo]) / h, u = 1.0 - t;
          const double cs = h * h / 6.0;
          const double wk = cs * (u * u * u - u), wk1 = cs * (t * t * t - t);
          for (int q = 0; q < 4; ++q)
            val[q] = u * v[4 * lo + q] + t * v[4 * lo + 4 + q] + wk * sd[4 * lo + q] + wk1 * sd[4 * lo + 4 + q];
        }
      }
    }
    const long long pidx = ((long long)z * nd + o) * nn + n;
    if (f) val[0] *= f[pidx];
    if (epsth) {
      const double* e = epsth + pidx * 4;
      for (int q = 0; q < 4; ++q) val[q] += e[q];
    }
    T* dst = out + (((long long)zl * nd + o) * nn + n) * 4;
    if (accumulate) {
      for (int q = 0; q < 4; ++q) dst[q] = (T)((double)dst[q] + val[q]);
    } else {
      for (int q = 0; q < 4; ++q) dst[q] = (T)val[q];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(128) k_spline_shift(
    int nz0, int nzc, int nd, int nn, const double* __restrict__ x, const double* __restrict__ SigT,
    const double* __restrict__ lam, const double* __restrict__ ub, double ub_sign,
    const double* __restrict__ sll, int ncls, int cls, const T* __restrict__ in, long long in_z_stride,
    long long in_o_stride, T* __restrict__ out, int accumulate, const double* __restrict__ f,
    const double* __restrict__ epsth, int weno) {
  extern __shared__ double spl[];
  (void)nzc;
  spline_shift_body<T>(blockIdx.x, spl, nz0, nd, nn, x, SigT, lam, ub, ub_sign, sll, ncls, cls, in, in_z_stride,
                       in_o_stride, out, accumulate, f, epsth, weno);
}

// ------------------------------------------------------------------ R_II contraction
// One GEMM per (z, theta) over every transition at once:
//   C[(t, c, n), (sl, s)] = sum_m M[z][theta][(t, c, n)][m] * Ibar[z][dir(sl)][m][s]
// rows R = 2 nt nn (transition, real/imaginary plane, frequency), columns
// 4 nslots(theta) (incoming-direction slot, Stokes), K = nn.  Matrix cores:
// v_mfma_{f32,f64}_16x16x4 with the operands swapped (A_in = B^T, B_in = M^T)
// so that each lane's four accumulators are the four Stokes components of one
// (row, slot) entry of W -- one contiguous 16/32-byte store.
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaOp;
// Output layouts differ: for the f32 16x16x4 instruction lane l holds rows
// 4 (l/16) + r of the 16x16 result, for the f64 one rows (l/16) + 4 r.  The f64
// path stores the B tile with its 16 columns transposed as a 4x4 grid so that
// both end up with one slot's four Stokes values per lane.
template <> struct MfmaOp<float> {
  typedef floatx4_t acc_t;
  static constexpr bool kInterleavedRows = false;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaOp<double> {
  typedef doublex4_t acc_t;
  static constexpr bool kInterleavedRows = true;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};


template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };
template <typename T> struct T2of;
template <> struct T2of<float> { typedef float2 type; };
template <> struct T2of<double> { typedef double2 type; };

// Block: 8 waves, each one 16-row wave tile of the banded store (the block's
// eight tiles in block order, KStore), x one column group (up to 4 NCT slots of
// one Theta, 16 NCT columns).  K runs over the block's column range [klo, khi)
// (the union of its rows' bands) in chunks of 8 NH: each lane loads its
// kernel-row fragment straight into registers with two-element vector loads,
// using the permuted K order k = k0 + 2 (4 h + lk) + jj for step (h, jj) of
// the matrix-core chain, zero outside its row's band; the column group's
// comoving field for the chunk is staged once in LDS and read with the same k.
// A wave issues only the steps that meet its own tile's column range.
// LDS row strides are padded so that the four k rows read by one matrix-core
// step (rows 2 apart) fall in different bank groups.
template <typename T> struct ContractCfg;
template <> struct ContractCfg<float> { static constexpr int BST = 136; };   // 128 columns + pad
template <> struct ContractCfg<double> { static constexpr int BST = 72; };   // 64 columns + pad

// Two consecutive kernel-row entries at index i of the store: the FP32 values,
// or (FP64) the sums of values and remainders.
template <typename T> struct KLoad;
template <> struct KLoad<float> {
  __device__ static inline float2 at(const KStore& ks, long long i) {
    return *reinterpret_cast<const float2*>(ks.hi + i);
  }
};
template <> struct KLoad<double> {
  __device__ static inline double2 at(const KStore& ks, long long i) {
    const float2 h = *reinterpret_cast<const float2*>(ks.hi + i);
    const float2 l = *reinterpret_cast<const float2*>(ks.lo + i);
    return make_double2((double)h.x + (double)l.x, (double)h.y + (double)l.y);
  }
};

// The row a lane multiplies in wave tile q of (z, theta): plane p = 2 t + c,
// frequency n and whether it is a grid row; the wave's stored column range
// [wlo, whi) (wave-uniform) and the store index of the lane's column 0 in
// the tile (`base`, so column k in range is at base + k).
struct KRow {
  long long base;
  int p, n, wlo, whi;
  bool live;
};

__device__ __forceinline__ KRow krow(const KStore& ks, long long zt, int q, int lr, int nt, int nn) {
  KRow r;
  q = __builtin_amdgcn_readfirstlane(q);
  const bool qv = q < ks.nq;
  const int grow = tile_row0(ks.pad, ks.np, ks.nnp, q) + lr;
  r.p = grow / ks.nnp;
  r.n = grow - r.p * ks.nnp;
  r.live = qv && r.p < 2 * nt && r.n < nn;
  TileDesc d{0, 0, 0};
  if (qv) d = ks.td[zt * ks.nq + q];
  r.wlo = __builtin_amdgcn_readfirstlane(d.lo);
  r.whi = __builtin_amdgcn_readfirstlane(d.hi);
  r.base = d.off + (long long)lr * (r.whi - r.wlo) - r.wlo;
  if (qv && ks.t32) {
    // the products step through the narrower window only (same addresses)
    const unsigned v = __builtin_amdgcn_readfirstlane(ks.t32[zt * ks.nq + q]);
    r.wlo = (int)(v & 0xffffu);
    r.whi = (int)(v >> 16);
  }
  return r;
}

// The products of one K chunk starting at column k0: for step (h, jj) every
// column tile jt takes its B value from LDS (row 8 h + jj of the lane's k
// group) and the lane's kernel-row fragment.  The B values of step h + 1 are
// read into registers before the products of step h are issued, so LDS
// latency overlaps the matrix cores.  Steps outside [hlo, hhi) (wave-uniform)
// are skipped.
template <typename T, int NH, int NCT>
__device__ __forceinline__ void mfma_chunk(const T* bcol, int bst, const typename T2of<T>::type (&mf)[NH],
                                           typename MfmaOp<T>::acc_t (&acc)[NCT], int hlo, int hhi) {
  using Op = MfmaOp<T>;
  T bc[2][NCT], bx[2][NCT];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int jt = 0; jt < NCT; ++jt) bc[jj][jt] = bcol[jj * bst + jt * 16];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    if (h + 1 < NH) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int jt = 0; jt < NCT; ++jt) bx[jj][jt] = bcol[(8 * (h + 1) + jj) * bst + jt * 16];
    }
    // keep the reads of step h + 1 ahead of the products of step h (the
    // scheduler would otherwise sink each read next to its use)
    __builtin_amdgcn_sched_barrier(0);
    if (h >= hlo && h < hhi) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const T bf = jj ? mf[h].y : mf[h].x;
#pragma unroll
        for (int jt = 0; jt < NCT; ++jt) acc[jt] = Op::run(bc[jj][jt], bf, acc[jt]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (h + 1 < NH) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int jt = 0; jt < NCT; ++jt) bc[jj][jt] = bx[jj][jt];
    }
  }
}

// step range of a wave whose columns are [wlo, whi) in the chunk at k0
template <int NH>
__device__ __forceinline__ void wave_steps(int wlo, int whi, int k0, int* hlo, int* hhi) {
  const int a = max(0, (wlo - k0) >> 3), b = min(NH, (whi - k0 + 7) >> 3);
  *hlo = __builtin_amdgcn_readfirstlane(a);
  *hhi = __builtin_amdgcn_readfirstlane(b);
}

// lane holds C[row][slot s0 + 4 jt + lk][Stokes]: W[zl][t][slot][c][n][s]
template <typename T, int NCT>
__device__ __forceinline__ void store_w(const KRow& r, int zl, int nt, int nn, int nslot, int s0, int cnt, int lk,
                                        const typename MfmaOp<T>::acc_t (&acc)[NCT], T* __restrict__ W) {
  if (!r.live) return;
  const int rt = r.p >> 1, rc = r.p & 1;
#pragma unroll
  for (int jt = 0; jt < NCT; ++jt) {
    const int sl = 4 * jt + lk;
    if (sl < cnt) {
      // non-temporal: W is read back once by the angular sum, after the
      // kernel rows and fields of the whole launch have streamed through L2
      typedef T NV __attribute__((ext_vector_type(4)));
      const NV o = {acc[jt][0], acc[jt][1], acc[jt][2], acc[jt][3]};
      __builtin_nontemporal_store(
          o, reinterpret_cast<NV*>(W + (((((size_t)zl * nt + rt) * nslot + s0 + sl) * 2 + rc) * w_stride(nn) + r.n) * 4));
    }
  }
}

template <typename T, int NH, int NCT>
__device__ __forceinline__ void contract_block(int rb, int g, int zl, int z0, int nth, int nt, int nn, int nd,
                                               const KStore& ks, const T* __restrict__ Ibar,
                                               const int* __restrict__ cgrp, const int* __restrict__ slot_dir,
                                               T* __restrict__ W, int nslot, T* Bs) {
  using Op = MfmaOp<T>;
  using acc_t = typename Op::acc_t;
  using V4 = typename Vec4<T>::type;
  using T2 = typename T2of<T>::type;
  constexpr int KCH = 8 * NH;
  constexpr int BST = ContractCfg<T>::BST;
  constexpr int CG = 4 * NCT;                       // slots per column group
  const int th = cgrp[3 * g], s0 = cgrp[3 * g + 1], cnt = cgrp[3 * g + 2];
  const long long zt = (long long)(z0 + zl) * nth + th;
  const unsigned bw = (ks.qb32 ? ks.qb32 : ks.qb)[zt * ks.nqb + rb];
  const int klo = (int)(bw & 0xffffu), khi = (int)(bw >> 16);
  const int nkc = max(1, (khi - klo + KCH - 1) / KCH);
  const T* Ib = Ibar + (size_t)zl * nd * nn * 4;
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const KRow r = krow(ks, zt, rb * 8 + wave, lr, nt, nn);
  acc_t acc[NCT];
#pragma unroll
  for (int j = 0; j < NCT; ++j)
    for (int q = 0; q < 4; ++q) acc[j][q] = T(0);
  for (int kc = 0; kc < nkc; ++kc) {
    const int k0 = klo + kc * KCH;
    int hlo, hhi;
    wave_steps<NH>(r.wlo, r.whi, k0, &hlo, &hhi);
    T2 mf[NH];
    const long long i0 = r.base + k0 + 2 * lk;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      if (h >= hlo && h < hhi) {       // wave-uniform: the wave tile's stored columns
        mf[h] = KLoad<T>::at(ks, i0 + 8 * h);
      } else {
        mf[h].x = T(0);
        mf[h].y = T(0);
      }
    }
    if (kc > 0) __syncthreads();
    for (int e = tid; e < KCH * CG; e += 512) {
      const int sl = e / KCH, kk = e - sl * KCH, k = k0 + kk;
      V4 v;
      if (sl < cnt && k < nn) {
        v = *reinterpret_cast<const V4*>(Ib + ((size_t)slot_dir[s0 + sl] * nn + k) * 4);
      } else {
        v.x = T(0); v.y = T(0); v.z = T(0); v.w = T(0);
      }
      T* dst = Bs + (size_t)kk * BST;
      if (Op::kInterleavedRows) {
        const int base = (sl >> 2) * 16 + (sl & 3);
        dst[base] = v.x;
        dst[base + 4] = v.y;
        dst[base + 8] = v.z;
        dst[base + 12] = v.w;
      } else {
        *reinterpret_cast<V4*>(dst + 4 * sl) = v;
      }
    }
    __syncthreads();
    mfma_chunk<T, NH, NCT>(Bs + 2 * lk * BST + lr, BST, mf, acc, hlo, hhi);
  }
  store_w<T, NCT>(r, zl, nt, nn, nslot, s0, cnt, lk, acc, W);
}


// One launch covers both column classes: groups [0, n8) have up to 32 slots
// (8 column tiles, FP32 only), groups [n8, ngrp) up to 16 (4 tiles); the wider
// groups come first in the dispatch order (the group index is the slowest grid
// dimension).
template <typename T, int NH>
__global__ void __launch_bounds__(512, 2) k_contract(int z0, int nth, int nt, int nn, int nd, KStore ks,
                                                     const T* __restrict__ Ibar, const int* __restrict__ cgrp, int n8,
                                                     const int* __restrict__ slot_dir, T* __restrict__ W,
                                                     int nslot) {
  extern __shared__ __align__(16) unsigned char csh[];
  T* Bs = reinterpret_cast<T*>(csh);
  const int g = blockIdx.z, zl = blockIdx.y;
  if constexpr (sizeof(T) == sizeof(float)) {
    if (g < n8) {
      contract_block<T, NH, 8>(blockIdx.x, g, zl, z0, nth, nt, nn, nd, ks, Ibar, cgrp, slot_dir, W, nslot, Bs);
      return;
    }
  }
  contract_block<T, NH, 4>(blockIdx.x, g, zl, z0, nth, nt, nn, nd, ks, Ibar, cgrp, slot_dir, W, nslot, Bs);
}

// The contraction of a flat incoming field, W_T in Stokes I at every
// direction and frequency (Q, U, V zero), as the normalisation factor of
// App. E asks for: every slot of angle Theta receives W_T times the sum of
// its stored kernel row in Stokes I and zero in Q, U, V, the same for every
// incoming direction.  So the intermediate is kept per Theta instead of per
// slot, Wf[zl][t][theta][c][n][s] (the angular sum then reads it through the
// pairs' Theta index), and one pass over the store (FP32 values plus
// remainders, in FP64) replaces the products.  One wave per 16-row tile of
// (height, Theta): the sixteen row sums, then one coalesced write of the
// tile's 16 x 4 values.
__global__ void __launch_bounds__(64) k_flat_contract(int z0, int nth, int nt, int nn, KStore ks,
                                                      const double* __restrict__ WT, double* __restrict__ Wf) {
  const int lane = threadIdx.x;
  const long long u = blockIdx.x;                  // (zl, theta, tile)
  const int q = (int)(u % ks.nq);
  const int th = (int)((u / ks.nq) % nth), zl = (int)(u / ((long long)ks.nq * nth));
  const long long zt = (long long)(z0 + zl) * nth + th;
  const TileDesc d = ks.td[zt * ks.nq + q];
  const int w = d.hi - d.lo;
  // four lanes per row, float4 loads (every tile row starts at a multiple of
  // 8 entries), sixteen columns per step of the four lanes
  const int i = lane >> 2, sk = lane & 3;
  const long long base = d.off + (long long)i * w;
  double acc = 0.0;
#pragma unroll 4
  for (int c = 4 * sk; c < w; c += 16) {
    const float4 h = *reinterpret_cast<const float4*>(ks.hi + base + c);
    const float4 l = *reinterpret_cast<const float4*>(ks.lo + base + c);
    acc += ((double)h.x + (double)l.x) + ((double)h.y + (double)l.y) + ((double)h.z + (double)l.z) +
           ((double)h.w + (double)l.w);
  }
  acc += __shfl_xor(acc, 1, 4);
  acc += __shfl_xor(acc, 2, 4);
  const double v = acc;
  // lane: row i = lane / 4, Stokes lane % 4
  const int gr = tile_row0(ks.pad, ks.np, ks.nnp, q) + i, p = gr / ks.nnp, n = gr - p * ks.nnp;
  if (p >= ks.np || n >= nn) return;
  const int t = p >> 1, c = p & 1;
  Wf[((((size_t)zl * nt + t) * nth + th) * 2 + c) * w_stride(nn) * 4 + (size_t)n * 4 + sk] = sk == 0 ? WT[z0 + zl] * v : 0.0;
}

// chunking of K: the fewest chunks of at most 128 columns, NH = chunk / 8
static void contract_chunks(int ldm, int* nkc, int* nh) {
  *nkc = (ldm + 127) / 128;
  *nh = (ldm + 8 * *nkc - 1) / (8 * *nkc);
}

// ---- persistent, software-pipelined FP32 contraction
// The same products as k_contract, with one block per compute unit looping
// over the tiles (block of wave tiles, height, column group), each in as many
// K chunks as its column range needs.  While the matrix cores work on one
// stage (kernel-row fragments in registers, comoving tile in LDS buffer b),
// the block already has the loads of the next stage in flight: its kernel-row
// fragments into a second register set and its comoving tile into registers,
// written to the other LDS buffer once the products are issued.  One barrier
// per stage.  The slot -> direction table is copied to LDS at the start so
// the comoving gather has no dependent global load.  Groups with up to 32
// slots (8 column tiles) are processed first, then those with up to 16.
template <int NH, int NCT>
__device__ __forceinline__ void contract_pipe_class(
    int first, int count, int step, int gbase, int zc, int z0, int nth, int nt, int nn, int nd, const KStore& ks,
    const float* __restrict__ Ibar, const int* __restrict__ cgrp, const int* sdir, float* __restrict__ W, int nslot,
    float* Bs0, float* Bs1) {
  using acc_t = floatx4_t;
  constexpr int KCH = 8 * NH;
  constexpr int BST = ContractCfg<float>::BST;
  constexpr int CG = 4 * NCT;
  constexpr int NB = (KCH * CG + 511) / 512;
  if (first >= count) {
    return;
  }
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int rb_n = ks.nqb;
  const int per_g = zc * rb_n;
  struct St {
    int t, kc, nkc, klo, g, zl;
    long long zt;
  };
  auto decode = [&](int t, St& d) {
    d.t = t;
    d.kc = 0;
    d.g = gbase + t / per_g;
    const int r = t % per_g;
    d.zl = r / rb_n;
    const int rb = r % rb_n;
    d.zt = (long long)(z0 + d.zl) * nth + cgrp[3 * d.g];
    const unsigned bw = (ks.qb32 ? ks.qb32 : ks.qb)[d.zt * ks.nqb + rb];
    d.klo = (int)(bw & 0xffffu);
    d.nkc = max(1, ((int)(bw >> 16) - d.klo + KCH - 1) / KCH);
    return rb;
  };
  // Loads read a valid address and keep the raw values; the masks (zero
  // outside the wave tile's column range, past the last slot or frequency of
  // the tile) are applied when the values are consumed, after the products of
  // the current stage are issued, so no load of the next stage is waited for
  // early.
  // the steps of a stage that meet the wave tile's stored columns (uniform)
  auto load_a = [&](const St& d, const KRow& r, float2 (&dst)[NH], int* hlo, int* hhi) {
    const int k0 = d.klo + d.kc * KCH;
    wave_steps<NH>(r.wlo, r.whi, k0, hlo, hhi);
    const float* ptr = ks.hi + (r.base + k0 + 2 * lk);
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      if (h >= *hlo && h < *hhi) {
        dst[h] = *reinterpret_cast<const float2*>(ptr + 8 * h);
      } else {
        dst[h] = make_float2(0.0f, 0.0f);
      }
    }
  };
  float4 bn[NB];
  unsigned bmask = 0;
  auto load_b = [&](const St& d) {
    const int s0 = cgrp[3 * d.g + 1], cnt = cgrp[3 * d.g + 2];
    const float* Ib = Ibar + (size_t)d.zl * nd * nn * 4;
    const int k0 = d.klo + d.kc * KCH;
    int dir[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int sl = (tid + 512 * q) / KCH;
      dir[q] = sdir[s0 + min(sl, cnt - 1)];
    }
    bmask = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 512 * q;
      const int sl = e / KCH, kk = e - sl * KCH, k = k0 + kk;
      bn[q] = *reinterpret_cast<const float4*>(Ib + ((size_t)dir[q] * nn + min(k, nn - 1)) * 4);
      bmask |= (e < KCH * CG && sl < cnt && k < nn ? 1u : 0u) << q;
    }
  };
  auto store_b = [&](float* Bs) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 512 * q;
      if (e < KCH * CG) {
        const int sl = e / KCH, kk = e - sl * KCH;
        const bool ok = (bmask >> q) & 1u;
        const float4 v = ok ? bn[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        *reinterpret_cast<float4*>(Bs + (size_t)kk * BST + 4 * sl) = v;
      }
    }
  };
  auto take_a = [&](float2 (&dst)[NH], const float2 (&src)[NH]) {
#pragma unroll
    for (int h = 0; h < NH; ++h) dst[h] = src[h];
  };
  float2 mf[NH], mfn[NH];
  acc_t acc[NCT];
#pragma unroll
  for (int j = 0; j < NCT; ++j)
    for (int q = 0; q < 4; ++q) acc[j][q] = 0.0f;
  St cur;
  int rb = decode(first, cur);
  KRow rc = krow(ks, cur.zt, rb * 8 + wave, lr, nt, nn);
  int hlo, hhi, hlo_n = 0, hhi_n = 0;
  load_a(cur, rc, mfn, &hlo, &hhi);
  load_b(cur);
  store_b(Bs0);
  take_a(mf, mfn);
  __syncthreads();
  int buf = 0;
  while (true) {
    St nx = cur;
    KRow rn = rc;
    bool more = true;
    if (cur.kc + 1 < cur.nkc) {
      nx.kc = cur.kc + 1;
    } else if (cur.t + step < count) {
      const int rbn = decode(cur.t + step, nx);
      rn = krow(ks, nx.zt, rbn * 8 + wave, lr, nt, nn);
    } else {
      more = false;
    }
    if (more) {
      load_a(nx, rn, mfn, &hlo_n, &hhi_n);
      load_b(nx);
    }
    mfma_chunk<float, NH, NCT>((buf ? Bs1 : Bs0) + 2 * lk * BST + lr, BST, mf, acc, hlo, hhi);
    if (cur.kc == cur.nkc - 1) {
      store_w<float, NCT>(rc, cur.zl, nt, nn, nslot, cgrp[3 * cur.g + 1], cgrp[3 * cur.g + 2], lk, acc, W);
#pragma unroll
      for (int j = 0; j < NCT; ++j)
        for (int q = 0; q < 4; ++q) acc[j][q] = 0.0f;
    }
    if (!more) break;
    store_b(buf ? Bs0 : Bs1);
    take_a(mf, mfn);
    __syncthreads();
    buf ^= 1;
    cur = nx;
    rc = rn;
    hlo = hlo_n;
    hhi = hhi_n;
  }
  // the next class starts by writing LDS buffer 0: every wave is done reading
  __syncthreads();
}

template <int NH>
__global__ void __launch_bounds__(512, 1) k_contract_pipe(int z0, int zc, int nth, int nt, int nn, int nd, KStore ks,
                                                          const float* __restrict__ Ibar,
                                                          const int* __restrict__ cgrp, int ngrp, int n8,
                                                          const int* __restrict__ slot_dir, float* __restrict__ W,
                                                          int nslot) {
  extern __shared__ __align__(16) unsigned char psh[];
  constexpr int KCH = 8 * NH;
  float* Bs0 = reinterpret_cast<float*>(psh);
  float* Bs1 = Bs0 + KCH * ContractCfg<float>::BST;
  int* sdir = reinterpret_cast<int*>(Bs1 + KCH * ContractCfg<float>::BST);
  for (int i = threadIdx.x; i < nslot; i += blockDim.x) sdir[i] = slot_dir[i];
  __syncthreads();
  const int per_g = zc * ks.nqb;
  contract_pipe_class<NH, 8>(blockIdx.x, n8 * per_g, gridDim.x, 0, zc, z0, nth, nt, nn, nd, ks, Ibar, cgrp, sdir, W,
                             nslot, Bs0, Bs1);
  contract_pipe_class<NH, 4>(blockIdx.x, (ngrp - n8) * per_g, gridDim.x, n8, zc, z0, nth, nt, nn, nd, ks, Ibar, cgrp,
                             sdir, W, nslot, Bs0, Bs1);
}

static size_t contract_pipe_lds(int nh, int nslot) {
  return (size_t)2 * 8 * nh * ContractCfg<float>::BST * sizeof(float) + (size_t)nslot * sizeof(int);
}

template <int NH>
static int launch_contract_pipe_nh(trap_ctx* ctx, hipStream_t stream, int zc, int z0, const KStore& ks,
                                   const float* Ibar, float* W, size_t lds) {
  Problem& P = ctx->pb;
  const int ngrp = (int)P.cgrp[1].size() / 3;
  const long long ntiles = (long long)ngrp * zc * ks.nqb;
  const int grid = (int)std::min<long long>(ntiles, ctx->n_cu);
  auto kern = k_contract_pipe<NH>;
  if (lds > 64 * 1024)
    TRAP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(512), lds, stream, z0, zc, P.nth, P.nt, P.nn, P.nd, ks, Ibar,
                     P.d_cgrp[1], ngrp, P.cgrp_n8[1], P.d_slot_dir, W, P.nslot);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

// ---- resident-field FP32 contraction
// One work unit is (column group, slice of the (height, theta) plane's wave
// tiles, height): the group's comoving field over every frequency is staged in
// LDS once, and the block's eight waves then take the slice's tiles one at a
// time from a counter in LDS, each wave stepping through its own tile's column
// window with no barrier between waves.  A wave keeps the kernel-row
// fragments of its next D steps in flight while the matrix cores work on the
// current D, across tile boundaries (the next tile's descriptor is read one
// tile ahead).  Blocks take units from a global ticket in order of decreasing
// work (the groups sorted on the host), the next ticket fetched while the
// current unit runs; the last block to finish resets the ticket and its own
// count to zero for the next launch.  LDS layout: frequency pairs (k, k + 1)
// interleaved per column, [k / 2][column][k & 1]; column c of pair row kp
// sits at c ^ 16 (kp & 3), so the four pair rows one matrix-core step reads
// fall in different bank halves.
constexpr int kResD = 8;
constexpr int kResStage = 10;    // staging items per thread: (320 / 2) x 32 slots / 512 threads

__device__ __forceinline__ int res_grab(int* ctr, int lane) {
  int v = 0;
  if (lane == 0) v = atomicAdd(ctr, 1);
  return __builtin_amdgcn_readfirstlane(__shfl(v, 0));
}

// The loads take no branch (a step past the window re-reads its last step;
// its products are skipped), so the wait counts stay exact and the next
// group's loads are never waited for by the current group's products.
template <int D>
__device__ __forceinline__ void res_load(const float* __restrict__ hi, const KRow& r, int s, int e, int lk,
                                         float2 (&a)[D]) {
  // an empty window reads the store's first entries instead
  const bool any = e > s;
  const int last = max(e - 1, s);
  const float* ptr = any ? hi + (r.base + 2 * lk) : hi;
#pragma unroll
  for (int h = 0; h < D; ++h) a[h] = *reinterpret_cast<const float2*>(ptr + (any ? 8LL * min(s + h, last) : 0LL));
}

// the products of steps s .. min(s + D, e) - 1; bl: the lane's pair row lk
// and column lr; the B values of step h + 1 are read (unconditionally, a step
// past the window re-reading the last one) before the products of h
template <int NCT, int D>
__device__ __forceinline__ void res_mfma(const float* bl, const int (&co)[NCT], int s, int e, const float2 (&a)[D],
                                         floatx4_t (&acc)[NCT]) {
  constexpr int CW = 16 * NCT;
  const int n = e - s;
  if (n <= 0) return;
  const float* b0 = bl + (size_t)s * 8 * CW;
  float2 b[2][NCT];
#pragma unroll
  for (int jt = 0; jt < NCT; ++jt) b[0][jt] = *reinterpret_cast<const float2*>(b0 + co[jt]);
#pragma unroll
  for (int h = 0; h < D; ++h) {
    if (h + 1 < D) {
      const float* bh = b0 + min(h + 1, n - 1) * 8 * CW;
#pragma unroll
      for (int jt = 0; jt < NCT; ++jt) b[(h + 1) & 1][jt] = *reinterpret_cast<const float2*>(bh + co[jt]);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (h < n) {
#pragma unroll
      for (int jt = 0; jt < NCT; ++jt)
        acc[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[h & 1][jt].x, a[h].x, acc[jt], 0, 0, 0);
#pragma unroll
      for (int jt = 0; jt < NCT; ++jt)
        acc[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[h & 1][jt].y, a[h].y, acc[jt], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// krow with the tile descriptor read through the constant address space:
// scalar loads, counted apart from the vector loads of the kernel rows
__device__ __forceinline__ KRow krow_s(const KStore& ks, long long zt, int q, int lr, int nn) {
  typedef const __attribute__((address_space(4))) TileDesc* CTile;
  typedef const __attribute__((address_space(4))) unsigned* CWin;
  KRow r;
  q = __builtin_amdgcn_readfirstlane(q);
  const long long i = zt * ks.nq + q;
  const CTile d = (CTile)ks.td + i;
  const long long off = d->off;
  const int lo = d->lo, hi = d->hi;
  const int grow = tile_row0(ks.pad, ks.np, ks.nnp, q) + lr;
  r.p = grow / ks.nnp;
  r.n = grow - r.p * ks.nnp;
  r.live = r.p < ks.np && r.n < nn;
  r.wlo = lo;
  r.whi = hi;
  r.base = off + (long long)lr * (hi - lo) - lo;
  if (ks.t32) {
    const unsigned v = ((CWin)ks.t32)[i];
    r.wlo = (int)(v & 0xffffu);
    r.whi = (int)(v >> 16);
  }
  return r;
}

// one stage of a wave's stream: D steps of one tile (s .. e the tile's
// steps from s on); ok = 0 past the wave's last tile
struct RStage {
  KRow r;
  int s, e, ok;
};

// the wave's share of tiles [.., t1) of one unit (the LDS counter starts at
// the slice's first).  Kernel-row loads run two stages ahead through three
// register buffers; every stage issues its D loads so the wait counts stay
// exact.
template <int NCT>
__device__ __forceinline__ void res_tiles(const KStore& ks, long long zt, int t1, int zl, int nt, int nn, int nslot,
                                          int s0, int cnt, const float* Bs, int* ctr, float* __restrict__ W,
                                          int lane) {
  constexpr int D = kResD;
  constexpr int CW = 16 * NCT;
  const int lr = lane & 15, lk = lane >> 4;
  const float* bl = Bs + (size_t)lk * 2 * CW + 2 * lr;
  int co[NCT];
#pragma unroll
  for (int jt = 0; jt < NCT; ++jt) co[jt] = 32 * (jt ^ lk);
  // the stage after st: the tile's next D steps, else the next tile's first
  auto advance = [&](const RStage& st) {
    RStage n = st;
    if (!st.ok) return n;
    if (st.s + D < st.e) {
      n.s = st.s + D;
      return n;
    }
    const int q = res_grab(ctr, lane);
    if (q >= t1) {
      n.ok = 0;
      return n;
    }
    n.r = krow_s(ks, zt, q, lr, nn);
    n.s = n.r.wlo >> 3;
    n.e = n.r.whi >> 3;
    return n;
  };
  // a stage past the wave's end keeps the last stage's addresses; an empty
  // window reads D distinct steps at the start of the store (never a branch,
  // never one address for several loads)
  auto load = [&](const RStage& st, float2 (&a)[D]) {
    const bool any = st.e > st.s;
    const long long base = any ? st.r.base + 2 * lk : 2LL * lk;
    const int s = any ? st.s : 0, last = any ? st.e - 1 : D - 1;
#pragma unroll
    for (int h = 0; h < D; ++h) a[h] = *reinterpret_cast<const float2*>(ks.hi + base + 8LL * min(s + h, last));
  };
  floatx4_t acc[NCT];
#pragma unroll
  for (int j = 0; j < NCT; ++j)
    for (int c = 0; c < 4; ++c) acc[j][c] = 0.0f;
  RStage s0st;
  s0st.ok = 1;
  s0st.s = 0;
  s0st.e = 0;     // "tile finished": advance takes the first tile
  s0st.r = KRow{0, 0, 0, 0, 0, false};
  RStage st0 = advance(s0st);
  if (!st0.ok) return;
  RStage st1 = advance(st0);
  float2 a0[D], a1[D], a2[D];
  load(st0, a0);
  load(st1, a1);
  // compute stage st0 from buffer c while the stage two ahead loads into l;
  // false once the wave's last stage is done
  auto body = [&](float2 (&l)[D], const float2 (&c)[D]) {
    const RStage st2 = advance(st1);
    load(st2, l);
    // the buffer's loads (issued two stages ago) are complete here on every
    // path, whether or not the products below use all of it, so no later
    // reuse of its registers waits on the loads in flight (an empty asm that
    // only reads the registers: no instruction is emitted)
#pragma unroll
    for (int h = 0; h < D; ++h) asm volatile("" ::"v"(c[h].x), "v"(c[h].y));
    res_mfma<NCT, D>(bl, co, st0.s, st0.e, c, acc);
    if (st0.s + D >= st0.e) {
      store_w<float, NCT>(st0.r, zl, nt, nn, nslot, s0, cnt, lk, acc, W);
#pragma unroll
      for (int j = 0; j < NCT; ++j)
        for (int c4 = 0; c4 < 4; ++c4) acc[j][c4] = 0.0f;
    }
    st0 = st1;
    st1 = st2;
    return st0.ok != 0;
  };
  while (body(a2, a0) && body(a0, a1) && body(a1, a2)) {
  }
}

// unit ui -> (group cord[j], slice, height): ui = (j nsl + slice) zc + zl
__global__ void __launch_bounds__(512, 1) k_contract_res(int z0, int zc, int nth, int nt, int nn, int nd, int ldm,
                                                         KStore ks, const float* __restrict__ Ibar,
                                                         const int* __restrict__ cgrp, const int* __restrict__ cord,
                                                         int ngrp, int n8, int nsl, int* __restrict__ uctr,
                                                         const int* __restrict__ slot_dir, float* __restrict__ W,
                                                         int nslot) {
  extern __shared__ __align__(16) unsigned char rsh[];
  float* Bs = reinterpret_cast<float*>(rsh);
  // [0] tile counter, [2 + (i & 1)] the ticket of unit iteration i
  int* ctr = reinterpret_cast<int*>(Bs + (size_t)ldm * 128);
  const int tid = threadIdx.x, lane = tid & 63;
  const int nunit = zc * ngrp * nsl;
  const int np2 = ldm >> 1;
  if (tid == 0) ctr[2] = atomicAdd(&uctr[0], 1);
  __syncthreads();
  for (int it = 0;; ++it) {
    const int ui = ctr[2 + (it & 1)];
    if (ui >= nunit) break;
    const int zl = ui % zc, js = ui / zc, j = js / nsl, slice = js - j * nsl;
    const int g = cord[j];
    const int th = cgrp[3 * g], s0 = cgrp[3 * g + 1], cnt = cgrp[3 * g + 2];
    const bool wide = g < n8;
    const int cgs = wide ? 32 : 16, cw = 4 * cgs;
    const int t0 = (int)((long long)slice * ks.nq / nsl), t1 = (int)((long long)(slice + 1) * ks.nq / nsl);
    // stage the field: all loads first, then the LDS writes
    const float* Ib = Ibar + (size_t)zl * nd * nn * 4;
    // item e = tid + 512 q is (pair row e / cgs, slot e % cgs): the slot is
    // the same for all of a thread's items (512 is a multiple of cgs)
    const int nit = np2 * cgs;
    const int sl = tid % cgs, kpb = tid / cgs, kps = 512 / cgs;
    const float* src = Ib + (size_t)slot_dir[s0 + min(sl, cnt - 1)] * nn * 4;
    float4 v0[kResStage], v1[kResStage];
#pragma unroll
    for (int q = 0; q < kResStage; ++q) {
      const int kp = kpb + q * kps;
      const int k0 = min(2 * kp, nn - 1), k1 = min(2 * kp + 1, nn - 1);
      v0[q] = *reinterpret_cast<const float4*>(src + (size_t)k0 * 4);
      v1[q] = *reinterpret_cast<const float4*>(src + (size_t)k1 * 4);
    }
#pragma unroll
    for (int q = 0; q < kResStage; ++q) {
      const int e = tid + 512 * q;
      if (e < nit) {
        const int kp = kpb + q * kps;
        const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 a0 = (sl < cnt && 2 * kp < nn) ? v0[q] : z4;
        const float4 a1 = (sl < cnt && 2 * kp + 1 < nn) ? v1[q] : z4;
        const int pc = (4 * sl) ^ (16 * (kp & 3));
        float* dst = Bs + ((size_t)kp * cw + pc) * 2;
        *reinterpret_cast<float4*>(dst) = make_float4(a0.x, a1.x, a0.y, a1.y);
        *reinterpret_cast<float4*>(dst + 4) = make_float4(a0.z, a1.z, a0.w, a1.w);
      }
    }
    if (tid == 0) {
      ctr[0] = t0;
      ctr[2 + ((it + 1) & 1)] = atomicAdd(&uctr[0], 1);
    }
    __syncthreads();
    const long long zt = (long long)(z0 + zl) * nth + th;
    if (wide) {
      res_tiles<8>(ks, zt, t1, zl, nt, nn, nslot, s0, cnt, Bs, ctr, W, lane);
    } else {
      res_tiles<4>(ks, zt, t1, zl, nt, nn, nslot, s0, cnt, Bs, ctr, W, lane);
    }
    __syncthreads();    // every wave is done with the field and the tile counter
  }
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&uctr[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&uctr[0], 0);
      atomicExch(&uctr[1], 0);
    }
  }
}

static size_t contract_res_lds(int ldm) { return (size_t)ldm * 128 * sizeof(float) + 16; }

// 1 when launched, 0 when one group's field over all frequencies does not fit LDS
static int launch_contract_res(trap_ctx* ctx, hipStream_t stream, int zc, int z0, const float* Ibar, float* W) {
  Problem& P = ctx->pb;
  const int ngrp = (int)P.cgrp[1].size() / 3;
  if (ngrp == 0) return 1;
  const size_t lds = contract_res_lds(P.ldm);
  if (lds > (size_t)ctx->max_lds || P.ldm > 320) return 0;
  const KStore ks = kernel_store(ctx, true);
  // slices per plane: about four units per compute unit
  const long long base = (long long)zc * ngrp;
  const int nsl = (int)std::max<long long>(1, std::min<long long>({8, ks.nq, (4LL * ctx->n_cu + base - 1) / base}));
  const int nunit = (int)(base * nsl);
  const int grid = std::min(nunit, ctx->n_cu);
  if (lds > 64 * 1024)
    TRAP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_contract_res),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_contract_res, dim3(grid), dim3(512), lds, stream, z0, zc, P.nth, P.nt, P.nn, P.nd, P.ldm, ks,
                     Ibar, P.d_cgrp[1], P.d_cord, ngrp, P.cgrp_n8[1], nsl, P.d_unit_ctr, P.d_slot_dir, W, P.nslot);
  TRAP_HIP(hipGetLastError());
  return 1;
}

// ---- resident-field FP64 contraction
// The FP32 kernel's scheme for the FP64 operator: groups of at most 16 slots
// (four column tiles), the comoving field in LDS as doubles with frequency
// pairs interleaved per column and each 16-column tile's columns transposed
// as a 4 x 4 grid (the f64 matrix-core output then holds one slot's four
// Stokes values per lane), kernel rows as value + remainder read two stages
// ahead through three register buffers, products over the full bands.
constexpr int kRes64D = 8;
constexpr int kRes64Stage = 5;   // staging items per thread: (320 / 2) x 16 slots / 512 threads

template <int D>
__device__ __forceinline__ void res64_load(const KStore& ks, const RStage& st, int lk, double2 (&a)[D]) {
  const bool any = st.e > st.s;
  const long long base = any ? st.r.base + 2 * lk : 2LL * lk;
  const int s = any ? st.s : 0, last = any ? st.e - 1 : D - 1;
#pragma unroll
  for (int h = 0; h < D; ++h) {
    const long long i = base + 8LL * min(s + h, last);
    const float2 vh = *reinterpret_cast<const float2*>(ks.hi + i);
    const float2 vl = *reinterpret_cast<const float2*>(ks.lo + i);
    a[h] = make_double2((double)vh.x + (double)vl.x, (double)vh.y + (double)vl.y);
  }
}

template <int D>
__device__ __forceinline__ void res64_mfma(const double* bl, int s, int e, const double2 (&a)[D],
                                           doublex4_t (&acc)[4]) {
  constexpr int CW = 64;
  const int n = e - s;
  if (n <= 0) return;
  const double* b0 = bl + (size_t)s * 8 * CW;
  double2 b[2][4];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) b[0][jt] = *reinterpret_cast<const double2*>(b0 + 32 * jt);
#pragma unroll
  for (int h = 0; h < D; ++h) {
    if (h + 1 < D) {
      const double* bh = b0 + min(h + 1, n - 1) * 8 * CW;
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) b[(h + 1) & 1][jt] = *reinterpret_cast<const double2*>(bh + 32 * jt);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (h < n) {
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
        acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[h & 1][jt].x, a[h].x, acc[jt], 0, 0, 0);
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
        acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[h & 1][jt].y, a[h].y, acc[jt], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ void res64_tiles(const KStore& ks, long long zt, int t1, int zl, int nt, int nn, int nslot,
                                            int s0, int cnt, const double* Bs, int* ctr, double* __restrict__ W,
                                            int lane) {
  constexpr int D = kRes64D;
  constexpr int CW = 64;
  const int lr = lane & 15, lk = lane >> 4;
  const double* bl = Bs + (size_t)lk * 2 * CW + 2 * lr;
  auto advance = [&](const RStage& st) {
    RStage n = st;
    if (!st.ok) return n;
    if (st.s + D < st.e) {
      n.s = st.s + D;
      return n;
    }
    const int q = res_grab(ctr, lane);
    if (q >= t1) {
      n.ok = 0;
      return n;
    }
    n.r = krow_s(ks, zt, q, lr, nn);
    n.s = n.r.wlo >> 3;
    n.e = n.r.whi >> 3;
    return n;
  };
  doublex4_t acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    for (int c = 0; c < 4; ++c) acc[j][c] = 0.0;
  RStage s0st;
  s0st.ok = 1;
  s0st.s = 0;
  s0st.e = 0;
  s0st.r = KRow{0, 0, 0, 0, 0, false};
  RStage st0 = advance(s0st);
  if (!st0.ok) return;
  RStage st1 = advance(st0);
  double2 a0[D], a1[D], a2[D];
  res64_load<D>(ks, st0, lk, a0);
  res64_load<D>(ks, st1, lk, a1);
  auto body = [&](double2 (&l)[D], const double2 (&c)[D]) {
    const RStage st2 = advance(st1);
    res64_load<D>(ks, st2, lk, l);
    // the buffer's loads are complete here on every path (an empty asm that
    // only reads the registers: no instruction is emitted)
#pragma unroll
    for (int h = 0; h < D; ++h) asm volatile("" ::"v"(c[h].x), "v"(c[h].y));
    res64_mfma<D>(bl, st0.s, st0.e, c, acc);
    if (st0.s + D >= st0.e) {
      store_w<double, 4>(st0.r, zl, nt, nn, nslot, s0, cnt, lk, acc, W);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        for (int c4 = 0; c4 < 4; ++c4) acc[j][c4] = 0.0;
    }
    st0 = st1;
    st1 = st2;
    return st0.ok != 0;
  };
  while (body(a2, a0) && body(a0, a1) && body(a1, a2)) {
  }
}

// unit ui -> (group cord0[j], slice, height): ui = (j nsl + slice) zc + zl;
// the ticket and count are the FP32 kernel's (one contraction at a time per context)
__global__ void __launch_bounds__(512, 1) k_contract_res64(int z0, int zc, int nth, int nt, int nn, int nd, int ldm,
                                                           KStore ks, const double* __restrict__ Ibar,
                                                           const int* __restrict__ cgrp, const int* __restrict__ cord,
                                                           int ngrp, int nsl, int* __restrict__ uctr,
                                                           const int* __restrict__ slot_dir, double* __restrict__ W,
                                                           int nslot) {
  extern __shared__ __align__(16) unsigned char rsh64[];
  double* Bs = reinterpret_cast<double*>(rsh64);
  int* ctr = reinterpret_cast<int*>(Bs + (size_t)ldm * 64);
  const int tid = threadIdx.x, lane = tid & 63;
  const int nunit = zc * ngrp * nsl;
  const int np2 = ldm >> 1;
  if (tid == 0) ctr[2] = atomicAdd(&uctr[0], 1);
  __syncthreads();
  for (int it = 0;; ++it) {
    const int ui = ctr[2 + (it & 1)];
    if (ui >= nunit) break;
    const int zl = ui % zc, js = ui / zc, j = js / nsl, slice = js - j * nsl;
    const int g = cord[j];
    const int th = cgrp[3 * g], s0 = cgrp[3 * g + 1], cnt = cgrp[3 * g + 2];
    const int t0 = (int)((long long)slice * ks.nq / nsl), t1 = (int)((long long)(slice + 1) * ks.nq / nsl);
    // item e = tid + 512 q is (pair row e / 16, slot e % 16): one slot per thread
    const double* Ib = Ibar + (size_t)zl * nd * nn * 4;
    const int nit = np2 * 16;
    const int sl = tid & 15, kpb = tid >> 4;
    const double* src = Ib + (size_t)slot_dir[s0 + min(sl, cnt - 1)] * nn * 4;
    double4 v0[kRes64Stage], v1[kRes64Stage];
#pragma unroll
    for (int q = 0; q < kRes64Stage; ++q) {
      const int kp = kpb + 32 * q;
      const int k0 = min(2 * kp, nn - 1), k1 = min(2 * kp + 1, nn - 1);
      v0[q] = *reinterpret_cast<const double4*>(src + (size_t)k0 * 4);
      v1[q] = *reinterpret_cast<const double4*>(src + (size_t)k1 * 4);
    }
    // column of (slot sl, Stokes st) inside its 16-column tile: st * 4 + sl % 4
    const int cb = 16 * (sl >> 2) + (sl & 3);
#pragma unroll
    for (int q = 0; q < kRes64Stage; ++q) {
      const int e = tid + 512 * q;
      if (e < nit) {
        const int kp = kpb + 32 * q;
        const double4 z4 = make_double4(0.0, 0.0, 0.0, 0.0);
        const double4 a0 = (sl < cnt && 2 * kp < nn) ? v0[q] : z4;
        const double4 a1 = (sl < cnt && 2 * kp + 1 < nn) ? v1[q] : z4;
        double* dst = Bs + ((size_t)kp * 64 + cb) * 2;
        *reinterpret_cast<double2*>(dst) = make_double2(a0.x, a1.x);
        *reinterpret_cast<double2*>(dst + 8) = make_double2(a0.y, a1.y);
        *reinterpret_cast<double2*>(dst + 16) = make_double2(a0.z, a1.z);
        *reinterpret_cast<double2*>(dst + 24) = make_double2(a0.w, a1.w);
      }
    }
    if (tid == 0) {
      ctr[0] = t0;
      ctr[2 + ((it + 1) & 1)] = atomicAdd(&uctr[0], 1);
    }
    __syncthreads();
    res64_tiles(ks, (long long)(z0 + zl) * nth + th, t1, zl, nt, nn, nslot, s0, cnt, Bs, ctr, W, lane);
    __syncthreads();
  }
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&uctr[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&uctr[0], 0);
      atomicExch(&uctr[1], 0);
    }
  }
}

// 1 when launched, 0 when one group's field over all frequencies does not fit LDS
static int launch_contract_res64(trap_ctx* ctx, hipStream_t stream, int zc, int z0, const double* Ibar, double* W) {
  Problem& P = ctx->pb;
  const int ngrp = (int)P.cgrp[0].size() / 3;
  if (ngrp == 0) return 1;
  const size_t lds = contract_res_lds(P.ldm);
  if (lds > (size_t)ctx->max_lds || P.ldm > 320) return 0;
  const KStore ks = kernel_store(ctx, false);
  const long long base = (long long)zc * ngrp;
  const int nsl = (int)std::max<long long>(1, std::min<long long>({8, ks.nq, (4LL * ctx->n_cu + base - 1) / base}));
  const int nunit = (int)(base * nsl);
  const int grid = std::min(nunit, ctx->n_cu);
  if (lds > 64 * 1024)
    TRAP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_contract_res64),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_contract_res64, dim3(grid), dim3(512), lds, stream, z0, zc, P.nth, P.nt, P.nn, P.nd, P.ldm,
                     ks, Ibar, P.d_cgrp[0], P.d_cord0, ngrp, nsl, P.d_unit_ctr, P.d_slot_dir, W, P.nslot);
  TRAP_HIP(hipGetLastError());
  return 1;
}

// 1 when launched, 0 when the problem does not fit the pipelined kernel's LDS
static int launch_contract_pipe(trap_ctx* ctx, hipStream_t stream, int zc, int z0, const float* Ibar, float* W) {
  Problem& P = ctx->pb;
  if ((int)P.cgrp[1].size() / 3 == 0) return 1;
  int nkc, nh;
  contract_chunks(P.ldm, &nkc, &nh);
  const size_t lds = contract_pipe_lds(nh, P.nslot);
  if (lds > (size_t)ctx->max_lds) return 0;
  const KStore ks = kernel_store(ctx, true);
  switch (nh) {
#define TRAP_PIPE_CASE(NHV) \
  case NHV:                 \
    TRAP_TRY(launch_contract_pipe_nh<NHV>(ctx, stream, zc, z0, ks, Ibar, W, lds)); \
    return 1;
    TRAP_PIPE_CASE(1) TRAP_PIPE_CASE(2) TRAP_PIPE_CASE(3) TRAP_PIPE_CASE(4)
    TRAP_PIPE_CASE(5) TRAP_PIPE_CASE(6) TRAP_PIPE_CASE(7) TRAP_PIPE_CASE(8)
    TRAP_PIPE_CASE(9) TRAP_PIPE_CASE(10) TRAP_PIPE_CASE(11) TRAP_PIPE_CASE(12)
    TRAP_PIPE_CASE(13) TRAP_PIPE_CASE(14) TRAP_PIPE_CASE(15) TRAP_PIPE_CASE(16)
#undef TRAP_PIPE_CASE
    default:
      return fail(TRAP_EINVAL, "internal: bad contraction chunk");
  }
}

template <typename T>
static int launch_contract(trap_ctx* ctx, int zc, int z0, const T* Ibar, T* W) {
  Problem& P = ctx->pb;
  const int pi = sizeof(T) == 8 ? 0 : 1;
  const int ngrp = (int)P.cgrp[pi].size() / 3;
  if (ngrp == 0) return TRAP_OK;
  int nkc, nh;
  contract_chunks(P.ldm, &nkc, &nh);
  const size_t lds = (size_t)8 * nh * ContractCfg<T>::BST * sizeof(T);
  const KStore ks = kernel_store(ctx, sizeof(T) == sizeof(float));
  dim3 grid(ks.nqb, zc, ngrp);
  const int n8 = P.cgrp_n8[pi];
  switch (nh) {
#define TRAP_CONTRACT_CASE(NHV)                                                                               \
  case NHV:                                                                                                   \
    hipLaunchKernelGGL((k_contract<T, NHV>), grid, dim3(512), lds, ctx->stream, z0, P.nth, P.nt, P.nn, P.nd, ks, \
                       Ibar, P.d_cgrp[pi], n8, P.d_slot_dir, W, P.nslot);                                     \
    break;
    TRAP_CONTRACT_CASE(1) TRAP_CONTRACT_CASE(2) TRAP_CONTRACT_CASE(3) TRAP_CONTRACT_CASE(4)
    TRAP_CONTRACT_CASE(5) TRAP_CONTRACT_CASE(6) TRAP_CONTRACT_CASE(7) TRAP_CONTRACT_CASE(8)
    TRAP_CONTRACT_CASE(9) TRAP_CONTRACT_CASE(10) TRAP_CONTRACT_CASE(11) TRAP_CONTRACT_CASE(12)
    TRAP_CONTRACT_CASE(13) TRAP_CONTRACT_CASE(14) TRAP_CONTRACT_CASE(15) TRAP_CONTRACT_CASE(16)
#undef TRAP_CONTRACT_CASE
    default:
      return fail(TRAP_EINVAL, "internal: bad contraction chunk");
  }
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

// ------------------------------------------------------------------ R_III factors
// Y[z][t][o][s] = sum_m r3[z][t][m] Ibar[z][o][m][s]
template <typename T>
__device__ __forceinline__ void r3_Y_body(int bx, int z0, int nzc, int nt, int nd, int nn,
                                          const double2* __restrict__ r3, const T* __restrict__ Ibar,
                                          double2* __restrict__ Y) {
  const long long id = bx * (long long)blockDim.x + threadIdx.x;
  const long long total = (long long)nzc * nt * nd * 4;
  if (id >= total) return;
  const int s = id & 3;
  const int o = (id >> 2) % nd;
  const int t = (id / (4LL * nd)) % nt;
  const int zl = id / (4LL * nd * nt);
  const int z = z0 + zl;
  const double2* r = r3 + ((size_t)z * nt + t) * nn;
  const T* I = Ibar + ((size_t)zl * nd + o) * nn * 4 + s;
  double re = 0.0, im = 0.0;
  for (int m = 0; m < nn; ++m) {
    const double v = (double)I[(size_t)m * 4];
    re += r[m].x * v;
    im += r[m].y * v;
  }
  Y[(((size_t)z * nt + t) * nd + o) * 4 + s] = make_double2(re, im);
}

template <typename T>
__global__ void k_r3_Y(int z0, int nzc, int nt, int nd, int nn, const double2* __restrict__ r3,
                       const T* __restrict__ Ibar, double2* __restrict__ Y) {
  r3_Y_body<T>(blockIdx.x, z0, nzc, nt, nd, nn, r3, Ibar, Y);
}

// X[z][u][u'][l] = sum_o' w_o' sum_j A[z][o'][j][u][u'][l] (Y[(u',l)][o'][j] + conj Y[(u,l)][o'][j])
__device__ __forceinline__ void r3_X_body(int bx, int z0, int nu, int nl, int nd, const double* __restrict__ w,
                                          const double2* __restrict__ A, const double2* __restrict__ Y,
                                          double2* __restrict__ X) {
  const int e = bx;   // (zl, u, up, l)
  const int l = e % nl;
  const int up = (e / nl) % nu;
  const int u = (e / (nl * nu)) % nu;
  const int zl = e / (nl * nu * nu);
  const int z = z0 + zl;
  const int nt = nu * nl;
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < nd * 4; k += blockDim.x) {
    const int o = k >> 2, j = k & 3;
    const double2 a = A[((((size_t)z * nd + o) * 4 + j) * nu + u) * nu * nl + (size_t)up * nl + l];
    const double2 y1 = Y[(((size_t)z * nt + up * nl + l) * nd + o) * 4 + j];
    const double2 y2 = Y[(((size_t)z * nt + u * nl + l) * nd + o) * 4 + j];
    const double2 yy = make_double2(y1.x + y2.x, y1.y - y2.y);
    re += w[o] * (a.x * yy.x - a.y * yy.y);
    im += w[o] * (a.x * yy.y + a.y * yy.x);
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sr[threadIdx.x] += sr[threadIdx.x + st];
      si[threadIdx.x] += si[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) X[((((size_t)z * nu + u) * nu + up) * nl) + l] = make_double2(sr[0], si[0]);
}

__global__ void k_r3_X(int z0, int nu, int nl, int nd, const double* __restrict__ w,
                       const double2* __restrict__ A, const double2* __restrict__ Y,
                       double2* __restrict__ X) {
  r3_X_body(blockIdx.x, z0, nu, nl, nd, w, A, Y, X);
}

// ------------------------------------------------------------------ angular / sublevel sum
// eps_bar[z][l][l'][o][n][i] = sum_{o'} sum_{u'} sum_c sum_j cf[z][p(o,o')][(u',l)][c][l'][i][j]
//                                  W[z][(u',l)][slot(o,o')][c][n][j]  +  R_III term
// with the angular coefficients precomputed per pair (c = 0 multiplies Re W,
// c = 1 multiplies Im W).  A block covers one outgoing direction o and 64
// frequencies (one per lane); its KQ waves split the incoming directions
// into contiguous ranges, so within a wave the slot, the pair and hence the
// coefficients are uniform (scalar loads) and each W load is 64 consecutive
// frequencies.  The waves also share the R_III outer product (its
// transition pairs dealt round-robin); the partial sums meet in LDS.  The
// kernel streams W once and waits on memory: more waves per block keep
// more loads in flight (KQ = 8 for the single-problem launch at 64 or more
// directions, 4 otherwise).
constexpr int kAngQ = 4;

template <typename T, int kAngMaxNl, int KQ>
__device__ __forceinline__ void angular_body(
    int bx, int by, T (&red)[KQ][64][kAngMaxNl][4], int z0, int nd, int nn, int nu, int nl, int nslot,
    const int* __restrict__ pair_slot, const int* __restrict__ pair_index, const T* __restrict__ cf,
    const T* __restrict__ W, double c_sc, const double2* __restrict__ E, const double2* __restrict__ bma,
    const double2* __restrict__ X, const double2* __restrict__ prof, T* __restrict__ Eb) {
  using V4 = typename Vec4<T>::type;
  const int zl = bx / nd, o = bx % nd;
  const int z = z0 + zl;
  const int nt = nu * nl;
  const int np = nd * nd;
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = by * 64 + lane;
  const bool live = n < nn;
  const int nc = min(n, nn - 1);
  const size_t pstride = (size_t)nt * 2 * nl * 16;
  const T* cfz = cf + (size_t)z * np * pstride;
  const double sc3 = c_sc * 0.25 * kInvPi;
  const double2* Ez = E + ((size_t)z * nd + o) * 4 * nu * nu * nl;
  for (int l = 0; l < nl; ++l) {
    T acc[kAngMaxNl][4];
#pragma unroll
    for (int a = 0; a < kAngMaxNl; ++a)
      for (int i = 0; i < 4; ++i) acc[a][i] = T(0);
    const int chunk = (nd + KQ - 1) / KQ;
    const int op1 = min(nd, (q + 1) * chunk);
#pragma unroll 4
    for (int op = q * chunk; op < op1; ++op) {
      const int slot = pair_slot[o * nd + op];
      const T* cp = cfz + (size_t)pair_index[o * nd + op] * pstride;
      for (int upr = 0; upr < nu; ++upr) {
        const int t = upr * nl + l;
        const T* Wp = W + (((size_t)zl * nt + t) * nslot + slot) * 2 * (size_t)w_stride(nn) * 4 + (size_t)nc * 4;
        const V4 wr = *reinterpret_cast<const V4*>(Wp);
        const V4 wi = *reinterpret_cast<const V4*>(Wp + (size_t)w_stride(nn) * 4);
        const T* c0 = cp + (size_t)t * 2 * nl * 16;
        const T* c1 = c0 + (size_t)nl * 16;
#pragma unroll
        for (int lp = 0; lp < kAngMaxNl; ++lp) {
          if (lp < nl) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const T* a = c0 + lp * 16 + i * 4;
              const T* b = c1 + lp * 16 + i * 4;
              acc[lp][i] += a[0] * wr.x + a[1] * wr.y + a[2] * wr.z + a[3] * wr.w +
                            b[0] * wi.x + b[1] * wi.y + b[2] * wi.z + b[3] * wi.w;
            }
          }
        }
      }
    }
    // R_III:  D_i(o, l', u, u') = c_sc/(4 pi) (beta - alpha)_{u u'} E_i(o; u', u, l') X[u][u'][l],
    // this wave's share of the (u, u') pairs
#pragma unroll
    for (int lp = 0; lp < kAngMaxNl; ++lp) {
      if (lp < nl) {
        double r3[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = q; k < nu * nu; k += KQ) {
          const int u = k / nu, upr = k - u * nu;
          const double2 bx = cmul(bma[((size_t)z * nu + u) * nu + upr], X[(((size_t)z * nu + u) * nu + upr) * nl + l]);
          const double2 pa = prof[((size_t)z * nt + upr * nl + l) * nn + nc];
          const double2 pb = prof[((size_t)z * nt + u * nl + l) * nn + nc];
          for (int i = 0; i < 4; ++i) {
            const double2 d = cmul(Ez[((size_t)(i * nu + upr) * nu + u) * nl + lp], bx);
            r3[i] += d.x * (pa.x + pb.x) - d.y * (pa.y - pb.y);
          }
        }
        for (int i = 0; i < 4; ++i) acc[lp][i] += (T)(sc3 * r3[i]);
      }
    }
    if (l > 0) __syncthreads();                        // previous class's partial sums consumed
#pragma unroll
    for (int lp = 0; lp < kAngMaxNl; ++lp)
      if (lp < nl)
        for (int i = 0; i < 4; ++i) red[q][lane][lp][i] = acc[lp][i];
    __syncthreads();
    if (q != 0 || !live) continue;
#pragma unroll
    for (int lp = 0; lp < kAngMaxNl; ++lp) {
      if (lp < nl) {
        T* dst = Eb + ((((size_t)zl * nl + l) * nl + lp) * nd + o) * (size_t)nn * 4 + (size_t)n * 4;
        for (int i = 0; i < 4; ++i) {
          T sum = T(0);
          for (int qq = 0; qq < KQ; ++qq) sum += red[qq][lane][lp][i];
          dst[i] = sum;
        }
      }
    }
  }
}

template <typename T, int kAngMaxNl, int KQ>
__global__ void __launch_bounds__(64 * KQ) k_angular(
    int z0, int nd, int nn, int nu, int nl, int nslot, const int* __restrict__ pair_slot,
    const int* __restrict__ pair_index, const T* __restrict__ cf, const T* __restrict__ W, double c_sc,
    const double2* __restrict__ E, const double2* __restrict__ bma, const double2* __restrict__ X,
    const double2* __restrict__ prof, T* __restrict__ Eb) {
  __shared__ T red[KQ][64][kAngMaxNl][4];
  angular_body<T, kAngMaxNl, KQ>(blockIdx.x, blockIdx.y, red, z0, nd, nn, nu, nl, nslot, pair_slot, pair_index,
                                 cf, W, c_sc, E, bma, X, prof, Eb);
}

// ------------------------------------------------------------------ fused R_II contraction + angular sum
// One block per (height z, tile of 16 comoving frequencies, lower sublevel l).
// The slots of each Theta are taken in groups of up to SG incoming directions.
// Per group the block stages in LDS the comoving field of those slots (the B
// tile), the angular coefficients of their pairs (o, o') and the pair lists;
// each wave multiplies the B tile on matrix cores by its kernel rows
// M[z][Theta][t][c][n0..n0+15][:] (held in registers, reloaded only when Theta
// changes) and the resulting W tile never leaves the CU: each lane forms
//   sum_j cf[pair][t][c][l'][i][j] W_j
// for every pair of its slot and adds it into an LDS accumulator
// eps_bar[l'][o][n][i].  The next group's B tile, coefficients and, at a Theta
// change, kernel rows are loaded into registers while the current group is
// multiplied.  The R_III term is added when the tile is written out.
// Waves own row tiles r = (u', c) (transition t = (u', l), real/imaginary
// plane c), TPW each.  The kernel-row fragments use a permuted K order: step
// (h, jj) takes k = 2 (4 h + lk) + jj in lane group lk, so each lane loads its
// fragment with two-element vector loads; the B tile is read with the same k.
template <typename T> struct FusedCfg;
template <> struct FusedCfg<float> { static constexpr int SG = 16, BST = 72; };
template <> struct FusedCfg<double> { static constexpr int SG = 8, BST = 40; };
// staged vectors per thread: B tile (RB) and coefficients (RC); the launcher
// picks (6, 4) for up to four upper sublevels and (6, 8) above
template <int TPW> struct FusedStage { static constexpr int RB = 6, RC = TPW == 1 ? 4 : 8; };

struct FusedLayout {
  size_t bs, el, cf, po;      // byte offsets of the LDS regions
  size_t total;
};

__host__ __device__ inline FusedLayout fused_layout(int ldm, int nd, int nu, int nl, int es, int sg, int bst) {
  FusedLayout L;
  L.bs = 0;
  L.el = L.bs + (size_t)ldm * bst * es;
  L.cf = L.el + (size_t)nl * nd * 64 * es;
  L.po = L.cf + ((size_t)2 * sg * nu * 2 * nl * 16 + 4) * es;   // + one vector that absorbs idle stores
  L.total = L.po + (size_t)(3 * sg + 2) * sizeof(int);
  return L;
}

template <typename T, int TPW, int NH>
__global__ void __launch_bounds__(512, TPW == 1 ? 3 : 2) k_fused(
    int nn, int ldm, int nd, int nth, int nt, int nu, int nl, int ntile, int nblk,
    const KStore ks, const T* __restrict__ Ibar, const int* __restrict__ grp, int ngrp,
    const int* __restrict__ slot_dir, const int* __restrict__ pair_off, const int* __restrict__ pair_o,
    const T* __restrict__ cf, double c_sc, const double2* __restrict__ E, const double2* __restrict__ bma,
    const double2* __restrict__ X, const double2* __restrict__ prof, T* __restrict__ Eb) {
  using Op = MfmaOp<T>;
  using acc_t = typename Op::acc_t;
  using V4 = typename Vec4<T>::type;
  using T2 = typename T2of<T>::type;
  constexpr int SG = FusedCfg<T>::SG, BST = FusedCfg<T>::BST, NCT = SG / 4;
  extern __shared__ __align__(16) unsigned char fsh[];
  const FusedLayout LY = fused_layout(ldm, nd, nu, nl, sizeof(T), SG, BST);
  T* Bs = reinterpret_cast<T*>(fsh + LY.bs);
  T* El = reinterpret_cast<T*>(fsh + LY.el);
  T* CFs = reinterpret_cast<T*>(fsh + LY.cf);
  int* Poff = reinterpret_cast<int*>(fsh + LY.po);     // [SG + 1] pair offsets of the group's slots
  int* Po = Poff + SG + 2;                             // [2 SG] outgoing direction of each pair
  // blocks are dealt round-robin to the 8 XCDs; renumber so that the frequency
  // tiles of one height (which read the same coefficients) share an XCD's L2
  const int b = blockIdx.x;
  const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, kx = b / 8;
  const int L = xcd < rem ? xcd * (per + 1) + kx : rem * (per + 1) + (xcd - rem) * per + kx;
  const int tile = L % ntile;
  const int l = (L / ntile) % nl;
  const int z = L / (ntile * nl);
  const int n0 = tile * 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int nthr = blockDim.x;
  const int np = nd * nd;
  const int n = n0 + lr;
  const int ncfv = nu * 2 * nl * 4;                    // coefficient vectors per pair (this l)
  for (int e = tid; e < nl * nd * 64; e += nthr) El[e] = T(0);
  int uq[TPW], cq[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int r = wave * TPW + q;
    uq[q] = r >> 1;
    cq[q] = r & 1;
  }
  const T* Ib = Ibar + (size_t)z * nd * nn * 4;
  const T* cfz = cf + (size_t)z * np * nt * 2 * nl * 16;

  // ---- staging of one group into registers, then LDS.  The (slot, k) of each
  //      B-tile item and the (pair, offset) of each coefficient item depend
  //      only on the thread, so they are decoded once.
  constexpr int RB = FusedStage<TPW>::RB, RC = FusedStage<TPW>::RC;
  int bsk[RB], cpo[RC];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int e = tid + i * nthr;
    const int sl = e / ldm;
    bsk[i] = (sl << 16) | (e - sl * ldm);
  }
#pragma unroll
  for (int i = 0; i < RC; ++i) {
    // e -> (pair pl, u', c, l', quarter); offset of the vector within the pair's block
    const int e = tid + i * nthr;
    const int qv = e & 3;
    int r = e >> 2;
    const int lp = r % nl; r /= nl;
    const int c = r & 1; r >>= 1;
    const int upr = r % nu;
    const int pl = r / nu;
    cpo[i] = (pl << 16) | ((((upr * nl + l) * 2 + c) * nl + lp) * 16 + qv * 4);
  }
  V4 rb[RB], rc[RC];
  int rpo0 = 0, rpo1 = 0;
  auto stage_load = [&](int g) {
    const int s0 = grp[3 * g + 1], cnt = grp[3 * g + 2];
    const int pb0 = pair_off[s0], npg = pair_off[s0 + cnt] - pb0;
    int dir[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int sl = bsk[i] >> 16;
      dir[i] = slot_dir[s0 + min(sl, cnt - 1)];
    }
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int pl = min(cpo[i] >> 16, npg - 1);
      rc[i] = *reinterpret_cast<const V4*>(cfz + (size_t)(pb0 + pl) * nt * 2 * nl * 16 + (cpo[i] & 0xffff));
    }
    if (tid <= cnt) rpo0 = pair_off[s0 + tid] - pb0;
    if (tid < npg) rpo1 = pair_o[pb0 + tid];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int sl = bsk[i] >> 16, k = bsk[i] & 0xffff;
      const V4 v = *reinterpret_cast<const V4*>(Ib + ((size_t)dir[i] * nn + min(k, nn - 1)) * 4);
      const bool ok = sl < cnt && k < nn;
      rb[i].x = ok ? v.x : T(0);
      rb[i].y = ok ? v.y : T(0);
      rb[i].z = ok ? v.z : T(0);
      rb[i].w = ok ? v.w : T(0);
    }
  };
  auto stage_store = [&](int g) {
    const int s0 = grp[3 * g + 1], cnt = grp[3 * g + 2];
    const int npg = pair_off[s0 + cnt] - pair_off[s0];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int sl = bsk[i] >> 16, k = bsk[i] & 0xffff;
      if (sl < SG) {
        T* dst = Bs + (size_t)k * BST;
        if (Op::kInterleavedRows) {
          const int base = (sl >> 2) * 16 + (sl & 3);
          dst[base] = rb[i].x;
          dst[base + 4] = rb[i].y;
          dst[base + 8] = rb[i].z;
          dst[base + 12] = rb[i].w;
        } else {
          *reinterpret_cast<V4*>(dst + 4 * sl) = rb[i];
        }
      }
    }
    const int lim = npg * ncfv, junk = 2 * SG * ncfv;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int e = tid + i * nthr;
      *reinterpret_cast<V4*>(CFs + (size_t)(e < lim ? e : junk) * 4) = rc[i];
    }
    if (tid <= cnt) Poff[tid] = rpo0;
    if (tid < npg) Po[tid] = rpo1;
  };
  // ---- kernel-row fragments (reloaded at a Theta change once the previous
  //      group's products are done, so the loads overlap its epilogue)
  T2 mf[TPW][NH];
  auto load_rows = [&](int th, T2 (&dst)[TPW][NH]) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = uq[q] * nl + l;
      const long long zt = (long long)z * nth + th;
      int tq = 0, tr = 0, lo = 0, hi = 0;
      long long base = 0;
      if (n < nn) {
        row_tile(ks.pad, ks.np, nn, 2 * t + cq[q], n, &tq, &tr);
        const TileDesc d = ks.td[zt * ks.nq + tq];
        lo = d.lo;
        hi = d.hi;
        base = d.off + (long long)tr * (hi - lo) - lo;
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int k = 2 * (4 * h + lk);
        if (k >= lo && k < hi) {
          dst[q][h] = KLoad<T>::at(ks, base + k);
        } else {
          dst[q][h].x = T(0);
          dst[q][h].y = T(0);
        }
      }
    }
  };

  stage_load(0);
  load_rows(grp[0], mf);
  __syncthreads();                       // El zeroed
  stage_store(0);
  __syncthreads();
  for (int g = 0; g < ngrp; ++g) {
    const int th = grp[3 * g], s0 = grp[3 * g + 1], cnt = grp[3 * g + 2];
    const bool more = g + 1 < ngrp;
    const bool newth = more && grp[3 * g + 3] != th;
    if (more) stage_load(g + 1);
    acc_t acc[TPW][NCT];
#pragma unroll
    for (int q = 0; q < TPW; ++q)
#pragma unroll
      for (int jt = 0; jt < NCT; ++jt)
        for (int r = 0; r < 4; ++r) acc[q][jt][r] = T(0);
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int k = 2 * (4 * h + lk) + jj;
#pragma unroll
        for (int jt = 0; jt < NCT; ++jt) {
          const T af = Bs[k * BST + jt * 16 + lr];
#pragma unroll
          for (int q = 0; q < TPW; ++q) acc[q][jt] = Op::run(af, jj ? mf[q][h].y : mf[q][h].x, acc[q][jt]);
        }
      }
    }
    if (newth) load_rows(grp[3 * g + 3], mf);
    // lane holds W_{t,c}(slot s0 + 4 jt + lk, n, Stokes 0..3)
    if (n < nn) {
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
#pragma unroll
        for (int jt = 0; jt < NCT; ++jt) {
          const int sl = 4 * jt + lk;
          if (sl < cnt) {
            const T w0 = acc[q][jt][0], w1 = acc[q][jt][1], w2 = acc[q][jt][2], w3 = acc[q][jt][3];
            const int p1 = Poff[sl + 1];
            for (int pl = Poff[sl]; pl < p1; ++pl) {
              const int o = Po[pl];
              const T* cp = CFs + (((size_t)pl * nu + uq[q]) * 2 + cq[q]) * nl * 16;
              for (int lp = 0; lp < nl; ++lp) {
                T* dst = El + ((lp * nd + o) * 16 + lr) * 4;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const V4 c4 = *reinterpret_cast<const V4*>(cp + lp * 16 + i * 4);
                  atomicAdd(dst + i, c4.x * w0 + c4.y * w1 + c4.z * w2 + c4.w * w3);
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
    if (more) stage_store(g + 1);
    __syncthreads();
  }
  // write eps_bar[z][l][l'][o][n][s], adding the R_III term
  //   D_i(o, l', u, u') = c_sc/(4 pi) (beta - alpha)_{u u'} E_i(o; u', u, l') X[u][u'][l]
  const double sc3 = c_sc * 0.25 * kInvPi;
  for (int e = tid; e < nl * nd * 16; e += nthr) {
    const int le = e & 15, o = (e >> 4) % nd, lp = (e >> 4) / nd;
    const int ne = n0 + le;
    if (ne >= nn) continue;
    double r3[4] = {0.0, 0.0, 0.0, 0.0};
    const double2* Ez = E + ((size_t)z * nd + o) * 4 * nu * nu * nl;
    for (int u = 0; u < nu; ++u)
      for (int upr = 0; upr < nu; ++upr) {
        const double2 bx = cmul(bma[((size_t)z * nu + u) * nu + upr], X[(((size_t)z * nu + u) * nu + upr) * nl + l]);
        const double2 pa = prof[((size_t)z * nt + upr * nl + l) * nn + ne];
        const double2 pb = prof[((size_t)z * nt + u * nl + l) * nn + ne];
        for (int i = 0; i < 4; ++i) {
          const double2 d = cmul(Ez[((size_t)(i * nu + upr) * nu + u) * nl + lp], bx);
          r3[i] += d.x * (pa.x + pb.x) - d.y * (pa.y - pb.y);
        }
      }
    T* dst = Eb + ((((size_t)z * nl + l) * nl + lp) * nd + o) * (size_t)nn * 4 + (size_t)ne * 4;
    for (int i = 0; i < 4; ++i) dst[i] = (T)((double)El[e * 4 + i] + sc3 * r3[i]);
  }
}

// LDS bytes of the fused kernel, or 0 when the problem does not fit its limits
// (padded frequency count <= 128, 2..8 upper sublevels, staging within the
// per-thread register budget, LDS within the device's per-block limit).
static size_t fused_lds(const trap_ctx* ctx, int prec) {
  const Problem& P = ctx->pb;
  // the FP64 operator (residuals, normalisation) keeps the height-chunked path
  if (prec == TRAP_FP64) return 0;
  const bool f64 = prec == TRAP_FP64;
  const int es = f64 ? 8 : 4;
  const int sg = f64 ? FusedCfg<double>::SG : FusedCfg<float>::SG;
  const int bst = f64 ? FusedCfg<double>::BST : FusedCfg<float>::BST;
  if (P.ldm > 128 || P.nu < 2 || P.nu > 8 || P.grp_maxpairs[f64 ? 0 : 1] > 2 * sg) return 0;
  const bool tpw1 = 2 * P.nu <= 8;
  const int nthr = 64 * (tpw1 ? 2 * P.nu : P.nu);
  const int rb = tpw1 ? FusedStage<1>::RB : FusedStage<2>::RB, rc = tpw1 ? FusedStage<1>::RC : FusedStage<2>::RC;
  if ((long long)nthr * rb < (long long)P.ldm * sg) return 0;
  if ((long long)nthr * rc < 2LL * sg * P.nu * 2 * P.nl * 4) return 0;
  if (nthr < 3 * sg + 2) return 0;
  const FusedLayout L = fused_layout(P.ldm, P.nd, P.nu, P.nl, es, sg, bst);
  if (L.total > (size_t)ctx->max_lds) return 0;
  return L.total;
}

template <typename T, int TPW, int NH>
static int launch_fused_t(trap_ctx* ctx, size_t lds, int nw, const T* Ibar, const T* cf, T* Eb) {
  Problem& P = ctx->pb;
  const int pi = sizeof(T) == 8 ? 0 : 1;
  const int ntile = ceil_div(P.nn, 16);
  const int nblk = P.nz * ntile * P.nl;
  auto kern = k_fused<T, TPW, NH>;
  if (lds > 64 * 1024)
    TRAP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(64 * nw), lds, ctx->stream, P.nn, P.ldm, P.nd, P.nth, P.nt, P.nu,
                     P.nl, ntile, nblk, kernel_store(ctx, false), Ibar, P.d_grp[pi], (int)P.grp[pi].size() / 3, P.d_slot_dir,
                     P.d_pair_off, P.d_pair_o, cf, P.c_sc, P.d_E, P.d_bma, ctx->wk.X, ctx->pre.d_prof, Eb);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

template <typename T, int TPW>
static int launch_fused_nh(trap_ctx* ctx, size_t lds, int nw, const T* Ibar, const T* cf, T* Eb) {
  switch (ctx->pb.ldm / 8) {
#define TRAP_FUSED_CASE(NHV) \
  case NHV: return launch_fused_t<T, TPW, NHV>(ctx, lds, nw, Ibar, cf, Eb);
    TRAP_FUSED_CASE(1) TRAP_FUSED_CASE(2) TRAP_FUSED_CASE(3) TRAP_FUSED_CASE(4)
    TRAP_FUSED_CASE(5) TRAP_FUSED_CASE(6) TRAP_FUSED_CASE(7) TRAP_FUSED_CASE(8)
    TRAP_FUSED_CASE(9) TRAP_FUSED_CASE(10) TRAP_FUSED_CASE(11) TRAP_FUSED_CASE(12)
    TRAP_FUSED_CASE(13) TRAP_FUSED_CASE(14) TRAP_FUSED_CASE(15) TRAP_FUSED_CASE(16)
#undef TRAP_FUSED_CASE
    default: return fail(TRAP_EINVAL, "frequency grid too large for the fused Sigma kernel");
  }
}

template <typename T>
static int launch_fused(trap_ctx* ctx, size_t lds, const T* Ibar, const T* cf, T* Eb) {
  const int nu = ctx->pb.nu;
  if (2 * nu <= 8) return launch_fused_nh<T, 1>(ctx, lds, 2 * nu, Ibar, cf, Eb);
  return launch_fused_nh<T, 2>(ctx, lds, nu, Ibar, cf, Eb);
}

// ------------------------------------------------------------------ driver
static size_t elem_size(int prec) { return prec == TRAP_FP64 ? sizeof(double) : sizeof(float); }

// stored real kernel entries of heights [z0, z0 + zc) and their contraction flops
double chunk_entries(const Problem& P, int z0, int zc) {
  const size_t a = (size_t)z0 * P.nth, b = (size_t)(z0 + zc) * P.nth;
  const long long e1 = b < P.kbase.size() ? P.kbase[b] : (long long)P.kentries;
  return (double)(e1 - P.kbase[a]);
}
double chunk_flops(const Problem& P, int z0, int zc) {
  double f = 0.0;
  for (int z = z0; z < z0 + zc; ++z) f += P.kflops_z[z];
  return f;
}
// the same for the FP32 operator's windows
double chunk_entries32(const Problem& P, int z0, int zc) {
  double e = 0.0;
  for (int z = z0; z < z0 + zc; ++z) e += P.kent32_z[z];
  return e;
}
double chunk_flops32(const Problem& P, int z0, int zc) {
  double f = 0.0;
  for (int z = z0; z < z0 + zc; ++z) f += P.kflops32_z[z];
  return f;
}

KStore kernel_store(const trap_ctx* ctx, bool fp32) {
  const Problem& P = ctx->pb;
  KStore k;
  k.hi = ctx->pre.d_Mhi;
  k.lo = ctx->pre.d_Mlo;
  k.td = P.d_td;
  k.qb = P.d_qb;
  if (fp32) {
    k.t32 = P.d_qk32;
    k.qb32 = P.d_qb32;
  }
  k.np = 2 * P.nt;
  k.nnp = P.nnp;
  k.nq = P.nq;
  k.nqb = P.nqb;
  k.pad = P.qpad;
  return k;
}

int ensure_work(trap_ctx* ctx, int prec) {
  Problem& P = ctx->pb;
  Work& K = ctx->wk;
  const size_t nz = P.nz, nd = P.nd, nn = P.nn;
  const size_t N = 4 * nz * nd * nn;
  if (!K.tmp64) {
    TRAP_TRY(dalloc_t(ctx, &K.tmp64, N));
    TRAP_TRY(dalloc_t(ctx, &K.r, N));
    TRAP_TRY(dalloc_t(ctx, &K.x, N));
    TRAP_TRY(dalloc_t(ctx, &K.Y, nz * P.nt * nd * 4));
    TRAP_TRY(dalloc_t(ctx, &K.X, nz * P.nu * P.nu * P.nl));
    TRAP_TRY(dalloc_t(ctx, &K.red, 4096));
    // height chunk: one chunk of W within 512 MiB in FP64 (half that in FP32),
    // so that the FP32 intermediate written by the contraction is still in the
    // 256 MB last-level cache when the angular sum reads it
    const size_t per_z = (size_t)P.nt * P.nslot * 2 * w_stride(nn) * 4 * sizeof(double);
    K.zchunk = (int)std::max<size_t>(1, std::min<size_t>(nz, (size_t(1) << 29) / std::max<size_t>(per_z, 1)));
  }
  const int pi = prec == TRAP_FP64 ? 0 : 1;
  if (!K.Ibar[pi]) {
    const size_t es = elem_size(prec);
    // comoving field for every height (the fused path reads all of it; the
    // chunked path uses the first chunk); W is allocated by the chunked path
    TRAP_TRY(dalloc(ctx, &K.Ibar[pi], nz * nd * nn * 4 * es));
    TRAP_TRY(dalloc(ctx, &K.Eb[pi], nz * P.nl * P.nl * nd * nn * 4 * es));
    TRAP_TRY(dalloc(ctx, &K.tmp[pi], N * es));
    TRAP_TRY(dalloc(ctx, &K.opeps[pi], N * es));
  }
  return TRAP_OK;
}

template <typename T>
static int sigma_apply_t(trap_ctx* ctx, const T* I, T* eps, int prec, int add_thermal, int normalize) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  Work& K = ctx->wk;
  hipStream_t s = ctx->stream;
  const int pi = prec == TRAP_FP64 ? 0 : 1;
  const int nz = P.nz, nd = P.nd, nn = P.nn, nt = P.nt, nth = P.nth, nl = P.nl, nu = P.nu;
  T* Ibar = static_cast<T*>(K.Ibar[pi]);
  T* W = static_cast<T*>(K.W[pi]);
  T* Eb = static_cast<T*>(K.Eb[pi]);
  const int ncls = nl * nl;
  const size_t spl_lds = (size_t)8 * nn * sizeof(double);
  // frame transforms: the context's interpolant, except in inner (linearised) applies
  const int weno = (ctx->interp == TRAP_INTERP_WENO4 && !ctx->interp_lin) ? 1 : 0;
  // the fused kernel runs only when asked for: its LDS scatter of the angular
  // sum is still slower than materialising W per height chunk
  const size_t flds = ctx->path == TRAP_PATH_FUSED ? fused_lds(ctx, prec) : 0;
  if (ctx->path == TRAP_PATH_FUSED && flds == 0)
    return fail(TRAP_EINVAL, "problem exceeds the fused Sigma kernel's limits");
  const T* cf = sizeof(T) == 8 ? (const T*)C.d_cf64 : (const T*)C.d_cf32;
  if (flds && cf) {
    // 1. comoving interpolation, all heights
    int pr = prof_begin(ctx, TRAP_STAGE_COMOVING);
    hipLaunchKernelGGL(k_spline_shift<T>, dim3(nz * nd), dim3(128), spl_lds, s, 0, nz, nd, nn, P.d_x,
                       P.d_SigT, P.d_lam, P.d_ub, -1.0, (const double*)nullptr, 1, 0, I,
                       (long long)nd * nn * 4, (long long)nn * 4, Ibar, 0, (const double*)nullptr,
                       (const double*)nullptr, weno);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    // 2. R_III factors, all heights
    pr = prof_begin(ctx, TRAP_STAGE_R3);
    const long long ny = (long long)nz * nt * nd * 4;
    hipLaunchKernelGGL(k_r3_Y<T>, dim3(ceil_div(ny, 256)), dim3(256), 0, s, 0, nz, nt, nd, nn, C.d_r3, Ibar,
                       K.Y);
    TRAP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_r3_X, dim3(nz * nu * nu * nl), dim3(256), 0, s, 0, nu, nl, nd, P.d_w, P.d_A, K.Y,
                       K.X);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    // 3. fused R_II contraction, angular/sublevel sum and R_III into eps_bar
    {
      // (the fused kernel steps through the full tile ranges)
      const double kel = chunk_entries(P, 0, nz) * (sizeof(T) / sizeof(float));
      const double flops = chunk_flops(P, 0, nz);
      const double bytes = sizeof(float) * kel + sizeof(T) * ((double)nz * nd * nn * 4 + (double)nz * nd * nd * nt * 2 * nl * 16 +
                                        (double)nz * ncls * nd * nn * 4);
      pr = prof_begin(ctx, sizeof(T) == 8 ? TRAP_STAGE_CONTRACT_FP64 : TRAP_STAGE_CONTRACT, flops, bytes);
    }
    if constexpr (sizeof(T) == sizeof(float)) {
      TRAP_TRY(launch_fused<T>(ctx, flds, Ibar, cf, Eb));
    }
    prof_end(ctx, pr);
  }
  if (!(flds && cf)) {
    // 1. comoving interpolation and R_III factors, all heights
    int pr = prof_begin(ctx, TRAP_STAGE_COMOVING);
    hipLaunchKernelGGL(k_spline_shift<T>, dim3(nz * nd), dim3(128), spl_lds, s, 0, nz, nd, nn, P.d_x,
                       P.d_SigT, P.d_lam, P.d_ub, -1.0, (const double*)nullptr, 1, 0, I,
                       (long long)nd * nn * 4, (long long)nn * 4, Ibar, 0, (const double*)nullptr,
                       (const double*)nullptr, weno);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    pr = prof_begin(ctx, TRAP_STAGE_R3);
    const long long ny = (long long)nz * nt * nd * 4;
    hipLaunchKernelGGL(k_r3_Y<T>, dim3(ceil_div(ny, 256)), dim3(256), 0, s, 0, nz, nt, nd, nn, C.d_r3, Ibar,
                       K.Y);
    TRAP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_r3_X, dim3(nz * nu * nu * nl), dim3(256), 0, s, 0, nu, nl, nd, P.d_w, P.d_A, K.Y,
                       K.X);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
  }
  for (int z0 = 0; z0 < nz && !(flds && cf); z0 += K.zchunk) {
    const int zc = std::min(K.zchunk, nz - z0);
    int pr;
    // 2. contraction
    {
      // algorithmic work of the chunk: 16 flops per in-band complex kernel
      // entry and incoming slot of its angle; bytes: the stored rows (FP32
      // values inside the FP32 windows, or values and remainders), W written
      // and the comoving field read
      const double kel = sizeof(T) == 8 ? 2.0 * chunk_entries(P, z0, zc) : chunk_entries32(P, z0, zc);
      const double flops = sizeof(T) == 8 ? chunk_flops(P, z0, zc) : chunk_flops32(P, z0, zc);
      const double bytes = sizeof(float) * kel + sizeof(T) * ((double)zc * nt * P.nslot * 2.0 * nn * 4 +
                                                               (double)zc * nd * nn * 4);
      // (the flat field's row sums are not a contraction: not recorded as one)
      pr = ctx->flat_field ? -1
                           : prof_begin(ctx, sizeof(T) == 8 ? TRAP_STAGE_CONTRACT_FP64 : TRAP_STAGE_CONTRACT, flops,
                                        bytes);
    }
    if (!W) {
      TRAP_TRY(dalloc(ctx, &K.W[pi], (size_t)K.zchunk * nt * P.nslot * 2 * w_stride(nn) * 4 * sizeof(T)));
      W = static_cast<T*>(K.W[pi]);
    }
    if constexpr (sizeof(T) == sizeof(float)) {
      int launched = launch_contract_res(ctx, ctx->stream, zc, z0, Ibar + (size_t)z0 * nd * nn * 4, W);
      if (launched == 0)
        launched = launch_contract_pipe(ctx, ctx->stream, zc, z0, Ibar + (size_t)z0 * nd * nn * 4, W);
      if (launched < 0) return launched;
      if (!launched) TRAP_TRY(launch_contract<T>(ctx, zc, z0, Ibar + (size_t)z0 * nd * nn * 4, W));
    } else if (ctx->flat_field) {
      hipLaunchKernelGGL(k_flat_contract, dim3((unsigned)((long long)zc * nth * P.nq)), dim3(64), 0, s, z0, nth,
                         nt, nn, kernel_store(ctx, false), P.d_WT, W);
      TRAP_HIP(hipGetLastError());
    } else {
      int launched = 0;
      if constexpr (sizeof(T) == sizeof(double))
        launched = launch_contract_res64(ctx, ctx->stream, zc, z0, Ibar + (size_t)z0 * nd * nn * 4, W);
      if (launched < 0) return launched;
      if (!launched) TRAP_TRY(launch_contract<T>(ctx, zc, z0, Ibar + (size_t)z0 * nd * nn * 4, W));
    }
    prof_end(ctx, pr);
    // 4. angular / sublevel sum into Eb (chunk-local heights)
    pr = prof_begin(ctx, TRAP_STAGE_ANGULAR);
    {
      // more waves per block where the directions are many and the partial
      // sums fit (up to two lower sublevels): 8 waves, so that a launch's
      // blocks are resident at once (at 128 directions and 301 frequencies,
      // 640 blocks of 16 waves ran in 2.5 rounds of one block per compute
      // unit: 0.46 ms against 0.41 ms per height with 8 waves)
      constexpr int KW = 8;
      const bool wide = nd >= 64 && nl <= 2;
      auto kern = wide ? (nl == 1 ? k_angular<T, 1, KW> : k_angular<T, 2, KW>)
                       : (nl == 1 ? k_angular<T, 1, kAngQ> : nl == 2 ? k_angular<T, 2, kAngQ>
                                                            : nl <= 4 ? k_angular<T, 4, kAngQ> : k_angular<T, 8, kAngQ>);
      const int kq = wide ? KW : kAngQ;
      // (a flat field's intermediate is per Theta: k_flat_contract)
      const bool flat = sizeof(T) == 8 && ctx->flat_field;
      hipLaunchKernelGGL(kern, dim3(zc * nd, ceil_div(nn, 64)), dim3(64 * kq), 0, s, z0, nd, nn, nu, nl,
                         flat ? nth : P.nslot, flat ? P.d_pair_theta : P.d_pair_slot, P.d_pair_index, cf, W,
                         P.c_sc, P.d_E, P.d_bma, K.X, C.d_prof, Eb + (size_t)z0 * ncls * nd * nn * 4);
    }
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
  }
  // 5. back to the observer frame, per (l, l') class, f and eps_th
  const long long npts = (long long)nz * nd * nn;
  const int prb = prof_begin(ctx, TRAP_STAGE_BACKINTERP);
  for (int l = 0; l < nl; ++l)
    for (int lp = 0; lp < nl; ++lp) {
      const int cls = l * nl + lp;
      const bool first = (cls == 0), last = (cls == ncls - 1);
      // f multiplies the sum over classes: apply it on a separate pass when ncls > 1
      hipLaunchKernelGGL(k_spline_shift<T>, dim3(nz * nd), dim3(128), spl_lds, s, 0, nz, nd, nn,
                         P.d_x, P.d_SigT, P.d_lam, P.d_ub, 1.0, P.d_sll, ncls, cls,
                         Eb + (size_t)cls * nd * nn * 4, (long long)ncls * nd * nn * 4, (long long)nn * 4,
                         eps, first ? 0 : 1, (normalize && ncls == 1) ? C.d_f : (const double*)nullptr,
                         (add_thermal && last && ncls == 1) ? C.d_epsth : (const double*)nullptr, weno);
      TRAP_HIP(hipGetLastError());
    }
  if (ncls > 1 && (normalize || add_thermal)) {
    // eps <- f * eps (Stokes I) + eps_th : reuse the shift kernel with zero shift on a copy
    T* tmp = static_cast<T*>(K.tmp[pi]);
    TRAP_HIP(hipMemcpyAsync(tmp, eps, (size_t)npts * 4 * sizeof(T), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_spline_shift<T>, dim3(nz * nd), dim3(128), spl_lds, s, 0, nz, nd, nn,
                       P.d_x, P.d_SigT, P.d_lam, P.d_ub, 0.0, (const double*)nullptr, 1, 0, tmp,
                       (long long)nd * nn * 4, (long long)nn * 4, eps, 0,
                       normalize ? C.d_f : (const double*)nullptr,
                       add_thermal ? C.d_epsth : (const double*)nullptr, 0);
    TRAP_HIP(hipGetLastError());
  }
  prof_end(ctx, prb);
  return TRAP_OK;
}

// ------------------------------------------------------------------ continuum scattering (App. A)
// Coherent dipole scattering in the observer frame: for height z and
// frequency n, M = sum_x w_x sum_j I_j(x) Acart_j(x) (a 3 x 3 complex tensor,
// Acart_j = sum_cd (A_j)_cd e_c e_d^T on the direction's axes e_a, e_b), then
//   eps_i(o) += (3/4) sigma_c Re Tr(Acart_i(o) M),
// the Rayleigh phase matrix summed over incoming directions.  One 64-lane
// block per (z, n): lanes over directions, M reduced across the wave in FP64.
__device__ inline void acart_entry(int j, const double* ea, const double* eb, int r, int c, double& re, double& im) {
  const double aa = ea[r] * ea[c], bb = eb[r] * eb[c], ab = ea[r] * eb[c], ba = eb[r] * ea[c];
  switch (j) {
    case 0: re = aa + bb; im = 0.0; break;
    case 1: re = aa - bb; im = 0.0; break;
    case 2: re = ab + ba; im = 0.0; break;
    default: re = 0.0; im = ab - ba; break;      // A_V = [[0, i], [-i, 0]]
  }
}

template <typename T>
__global__ void __launch_bounds__(64) k_cont_scatter(int nz, int nd, int nn, const double* __restrict__ ea,
                                                     const double* __restrict__ eb, const double* __restrict__ w,
                                                     const double* __restrict__ sc, const double* __restrict__ eta0,
                                                     const T* __restrict__ I, T* __restrict__ eps) {
  __shared__ double Mr[9], Mi[9];
  const int z = blockIdx.x / nn, n = blockIdx.x % nn, lane = threadIdx.x;
  double mr[9], mi[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) mr[e] = mi[e] = 0.0;
  for (int x = lane; x < nd; x += 64) {
    const T* ix = I + (((size_t)z * nd + x) * nn + n) * 4;
    const double* a = ea + 3 * x;
    const double* b = eb + 3 * x;
    for (int j = 0; j < 4; ++j) {
      const double v = w[x] * (double)ix[j];
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        double re, im;
        acart_entry(j, a, b, e / 3, e % 3, re, im);
        mr[e] += v * re;
        mi[e] += v * im;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e)
    for (int off = 32; off > 0; off >>= 1) {
      mr[e] += __shfl_xor(mr[e], off, 64);
      mi[e] += __shfl_xor(mi[e], off, 64);
    }
  if (lane == 0)
    for (int e = 0; e < 9; ++e) {
      Mr[e] = mr[e];
      Mi[e] = mi[e];
    }
  __syncthreads();
  const double s = 0.75 * sc[(size_t)z * nn + n] * eta0[z];
  for (int o = lane; o < nd; o += 64) {
    T* eo = eps + (((size_t)z * nd + o) * nn + n) * 4;
    const double* a = ea + 3 * o;
    const double* b = eb + 3 * o;
    for (int i = 0; i < 4; ++i) {
      // Re Tr(X M) = sum_rc Re(X_rc M_cr)
      double t = 0.0;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double xr, xi;
          acart_entry(i, a, b, r, c, xr, xi);
          t += xr * Mr[c * 3 + r] - xi * Mi[c * 3 + r];
        }
      eo[i] = (T)((double)eo[i] + s * t);
    }
  }
}

int sigma_apply(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal, int normalize) {
  TRAP_TRY(sigma_apply_line(ctx, I, eps, prec, add_thermal, normalize));
  Problem& P = ctx->pb;
  if (!normalize || !P.has_cont || !P.d_sc) return TRAP_OK;
  if (prec == TRAP_FP64)
    hipLaunchKernelGGL(k_cont_scatter<double>, dim3(P.nz * P.nn), dim3(64), 0, ctx->stream, P.nz, P.nd, P.nn, P.d_ea,
                       P.d_eb, P.d_w, P.d_sc, P.d_eta0, static_cast<const double*>(I), static_cast<double*>(eps));
  else
    hipLaunchKernelGGL(k_cont_scatter<float>, dim3(P.nz * P.nn), dim3(64), 0, ctx->stream, P.nz, P.nd, P.nn, P.d_ea,
                       P.d_eb, P.d_w, P.d_sc, P.d_eta0, static_cast<const float*>(I), static_cast<float*>(eps));
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

int sigma_apply_line(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal, int normalize) {
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (!ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (prec != TRAP_FP64 && prec != TRAP_FP32) return fail(TRAP_EINVAL, "unknown precision");
  if (!I || !eps) return fail(TRAP_EINVAL, "null vector");
  TRAP_TRY(ensure_work(ctx, prec));
  if (prec == TRAP_FP64) {
    if (!ctx->pre.d_Mhi || !ctx->pre.d_cf64) return fail(TRAP_ESTATE, "FP64 kernels not stored");
    return sigma_apply_t<double>(ctx, static_cast<const double*>(I), static_cast<double*>(eps), prec,
                                 add_thermal, normalize);
  }
  if (!ctx->pre.d_Mhi || !ctx->pre.d_cf32) return fail(TRAP_ESTATE, "FP32 kernels not stored (store_mask bit 1)");
  return sigma_apply_t<float>(ctx, static_cast<const float*>(I), static_cast<float*>(eps), prec,
                              add_thermal, normalize);
}

}  // namespace trap

// ------------------------------------------------------------------ grouped launches across contexts
// A serving step applies the FP32 operator of many contexts (requests) at
// once: each stage below is one launch whose blocks cover every context's
// work, with the same per-block code as the single-context kernels above, so a
// context's result does not depend on the others in the launch.  Block b
// belongs to context r with off[r] <= b < off[r + 1]; the context's sizes and
// pointers come from an argument record in device memory.

namespace trap {

__device__ __forceinline__ int find_req(int b, const int* __restrict__ off, int n) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(128) k_spline_shift_grouped(const GSpline* __restrict__ A,
                                                              const int* __restrict__ off, int n) {
  extern __shared__ double spl[];
  const int r = find_req(blockIdx.x, off, n);
  const GSpline& a = A[r];
  // the batched FP32 applies are inner (linearised) applies: spline transforms
  spline_shift_body<float>(blockIdx.x - off[r], spl, a.nz0, a.nd, a.nn, a.x, a.SigT, a.lam, a.ub, a.ub_sign, a.sll,
                           a.ncls, a.cls, a.in, a.in_z_stride, a.in_o_stride, a.out, a.accumulate, a.f, a.epsth, 0);
}

__global__ void __launch_bounds__(256) k_r3_Y_grouped(const GR3Y* __restrict__ A, const int* __restrict__ off,
                                                      int n) {
  const int r = find_req(blockIdx.x, off, n);
  const GR3Y& a = A[r];
  r3_Y_body<float>(blockIdx.x - off[r], a.z0, a.nzc, a.nt, a.nd, a.nn, a.r3, a.Ibar, a.Y);
}

__global__ void __launch_bounds__(256) k_r3_X_grouped(const GR3X* __restrict__ A, const int* __restrict__ off,
                                                      int n) {
  const int r = find_req(blockIdx.x, off, n);
  const GR3X& a = A[r];
  r3_X_body(blockIdx.x - off[r], a.z0, a.nu, a.nl, a.nd, a.w, a.A, a.Y, a.X);
}

template <int NH>
__global__ void __launch_bounds__(512, 2) k_contract_grouped(const GContract* __restrict__ A,
                                                             const int* __restrict__ off, int n) {
  extern __shared__ __align__(16) unsigned char csh[];
  float* Bs = reinterpret_cast<float*>(csh);
  const int r = find_req(blockIdx.x, off, n);
  const GContract& a = A[r];
  const int local = blockIdx.x - off[r];
  const int rb = local % a.ks.nqb, rest = local / a.ks.nqb;
  const int zl = rest % a.zc, g = rest / a.zc;     // column group slowest, as in k_contract
  if (g < a.n8)
    contract_block<float, NH, 8>(rb, g, zl, a.z0, a.nth, a.nt, a.nn, a.nd, a.ks, a.Ibar, a.cgrp, a.slot_dir, a.W,
                                 a.nslot, Bs);
  else
    contract_block<float, NH, 4>(rb, g, zl, a.z0, a.nth, a.nt, a.nn, a.nd, a.ks, a.Ibar, a.cgrp, a.slot_dir, a.W,
                                 a.nslot, Bs);
}

template <int NLM>
__global__ void __launch_bounds__(64 * kAngQ) k_angular_grouped(const GAngular* __restrict__ A,
                                                                const int* __restrict__ off, int n) {
  __shared__ float red[kAngQ][64][NLM][4];
  const int r = find_req(blockIdx.x, off, n);
  const GAngular& a = A[r];
  const int local = blockIdx.x - off[r];
  angular_body<float, NLM, kAngQ>(local % a.nbx, local / a.nbx, red, a.z0, a.nd, a.nn, a.nu, a.nl, a.nslot, a.pair_slot,
                           a.pair_index, a.cf, a.W, a.c_sc, a.E, a.bma, a.X, a.prof, a.Eb);
}

// x32 = (float) x64 (the conversion of the single-context path)
__global__ void __launch_bounds__(256) k_to_f32_grouped(const GVec* __restrict__ A, const int* __restrict__ off,
                                                        int n) {
  const int r = find_req(blockIdx.x, off, n);
  const GVec& a = A[r];
  for (long long i = (blockIdx.x - off[r]) * 256LL + threadIdx.x; i < a.N; i += (long long)a.nb * 256)
    a.x32[i] = (float)a.x64[i];
}

// y64 = (double)(x32 - f32): the FP32 difference, then the exact widening
__global__ void __launch_bounds__(256) k_finish_grouped(const GVec* __restrict__ A, const int* __restrict__ off,
                                                        int n) {
  const int r = find_req(blockIdx.x, off, n);
  const GVec& a = A[r];
  for (long long i = (blockIdx.x - off[r]) * 256LL + threadIdx.x; i < a.N; i += (long long)a.nb * 256) {
    const float d = a.x32[i] - a.f32[i];
    a.y64[i] = (double)d;
  }
}

// ---- per-device arena
namespace {

std::mutex g_arena_mu;
std::map<int, BatchArena> g_arena;

void arena_free(BatchArena& a) {
  for (StagingBuf& b : a.staging) {
    if (b.ev) {
      TRAP_NOTE(hipEventSynchronize(b.ev));
      TRAP_NOTE(hipEventDestroy(b.ev));
    }
    if (b.host) TRAP_NOTE(hipHostFree(b.host));
  }
  a.staging.clear();
  if (a.stream) TRAP_NOTE(hipStreamSynchronize(a.stream));
  for (hipEvent_t e : a.ev) TRAP_NOTE(hipEventDestroy(e));
  a.ev.clear();
  if (a.copied) TRAP_NOTE(hipEventDestroy(a.copied));
  if (a.done) TRAP_NOTE(hipEventDestroy(a.done));
  if (a.host) TRAP_NOTE(hipHostFree(a.host));
  if (a.dev) TRAP_NOTE(hipFree(a.dev));
  if (a.stream) TRAP_NOTE(hipStreamDestroy(a.stream));
  a = BatchArena();
}

// stream, events and a staging buffer of at least `bytes` (device current)
int arena_ready(BatchArena& a, size_t bytes, int nev) {
  if (!a.stream) {
    TRAP_HIP(hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking));
    TRAP_HIP(hipEventCreateWithFlags(&a.copied, hipEventDisableTiming));
    TRAP_HIP(hipEventCreateWithFlags(&a.done, hipEventDisableTiming));
  }
  while ((int)a.ev.size() < nev) {
    hipEvent_t e;
    TRAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    a.ev.push_back(e);
  }
  // the previous batch's upload must have left the staging buffer
  TRAP_HIP(hipEventSynchronize(a.copied));
  if (a.cap < bytes) {
    if (a.host) TRAP_HIP(hipHostFree(a.host));
    a.host = nullptr;
    if (a.dev) {
      TRAP_HIP(hipStreamSynchronize(a.stream));
      TRAP_HIP(hipFree(a.dev));
    }
    a.dev = nullptr;
    a.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64 << 10);
    TRAP_HIP(hipHostMalloc(reinterpret_cast<void**>(&a.host), cap));
    const hipError_t e = hipMalloc(&a.dev, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(TRAP_ENOMEM, "device allocation of the batch argument buffer failed");
    }
    a.cap = cap;
  }
  return TRAP_OK;
}

struct Blob {
  std::vector<unsigned char> h;
  template <typename S>
  size_t put(const std::vector<S>& v) {
    const size_t at = (h.size() + 63) & ~size_t(63);
    h.resize(at + std::max<size_t>(1, v.size()) * sizeof(S));
    if (!v.empty()) std::memcpy(h.data() + at, v.data(), v.size() * sizeof(S));
    return at;
  }
};

enum StageKind { SK_TO32, SK_SPLINE, SK_R3Y, SK_R3X, SK_CONTRACT, SK_CONTRACT_ONE, SK_ANGULAR, SK_COPY, SK_FORMAL,
                 SK_FINISH, SK_PC_CLS, SK_PC_FIN, SK_PC_SCAT, SK_PC_SWEEP };

struct Stage {
  int kind;
  int cls;            // NH of the contraction, sublevel class of the angular sum
  size_t args, off;   // blob offsets of the records and of the block offsets
  int n, blocks;
  size_t lds;
};

int nl_class(int nl) { return nl == 1 ? 1 : nl == 2 ? 2 : nl <= 4 ? 4 : 8; }

}  // namespace

void batch_arena_acquire(int device) {
  std::lock_guard<std::mutex> lk(g_arena_mu);
  g_arena[device].users++;
}

bool batch_arena_release(int device) {
  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto it = g_arena.find(device);
  if (it == g_arena.end()) return false;
  if (--it->second.users > 0) return false;
  arena_free(it->second);
  g_arena.erase(it);
  return true;
}

int stage_upload(trap_ctx* ctx, const void* host, size_t bytes, void* dev) {
  if (bytes == 0) return TRAP_OK;
  UploadBatch one;
  one.add(nullptr, host, bytes);
  return stage_upload_batch(ctx, one, dev);
}

int stage_upload_batch(trap_ctx* ctx, const UploadBatch& up, void* dev) {
  const size_t bytes = up.total;
  if (bytes == 0) return TRAP_OK;
  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto it = g_arena.find(ctx->device);
  if (it == g_arena.end()) return fail(TRAP_ESTATE, "internal: no shared state for the device");
  BatchArena& a = it->second;
  StagingBuf* pick = nullptr;
  for (StagingBuf& b : a.staging) {
    if (b.cap < bytes) continue;
    if (b.used) {
      const hipError_t q = hipEventQuery(b.ev);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();         // not an error: the buffer is still being read
        continue;
      }
      TRAP_HIP(q);
    }
    pick = &b;
    break;
  }
  if (!pick) {
    StagingBuf b;
    b.cap = std::max<size_t>(bytes, size_t(1) << 20);
    TRAP_HIP(hipHostMalloc(&b.host, b.cap));
    TRAP_HIP(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    a.staging.push_back(b);
    pick = &a.staging.back();
  }
  unsigned char* h = static_cast<unsigned char*>(pick->host);
  for (const UploadBatch::Item& it : up.items)
    if (it.bytes) std::memcpy(h + it.off, it.src, it.bytes);
  TRAP_HIP(hipMemcpyAsync(dev, pick->host, bytes, hipMemcpyHostToDevice, ctx->stream));
  TRAP_HIP(hipEventRecord(pick->ev, ctx->stream));
  pick->used = true;
  return TRAP_OK;
}

int sigma_batch_ready(trap_ctx* ctx) {
  Problem& P = ctx->pb;
  Work& K = ctx->wk;
  if (!ctx->has_problem || !ctx->pre.done || !ctx->pre.d_Mhi || !ctx->pre.d_cf32) return 0;
  if (ctx->path == TRAP_PATH_FUSED || ctx->prof.on) return 0;
  // the shared launches carry no continuum term
  if (P.has_cont) return 0;
  // a context whose Sigma runs in several height chunks costs several small
  // applies: in lockstep with the others it would hold every shared apply of
  // the batch, so it applies on its own stream and overlaps the shared work
  // (measured: serving throughput 7-10% higher than grouping it)
  if (K.zchunk < P.nz) return 0;
  TRAP_TRY(ensure_work(ctx, TRAP_FP32));
  if (!K.W[1])
    TRAP_TRY(dalloc(ctx, &K.W[1], (size_t)K.zchunk * P.nt * P.nslot * 2 * w_stride(P.nn) * 4 * sizeof(float)));
  return (K.v32a && K.v32b) ? 1 : 0;
}

int op_apply_batch_f32(trap_ctx** ctxs, int n, const double* const* x, double* const* y, const int* pc) {
  if (n <= 0) return TRAP_OK;
  const int device = ctxs[0]->device;
  Blob blob;
  std::vector<Stage> stages;
  auto add_stage = [&](int kind, int cls, size_t args, const std::vector<int>& cnt, size_t lds) {
    std::vector<int> off(cnt.size() + 1, 0);
    for (size_t i = 0; i < cnt.size(); ++i) off[i + 1] = off[i] + cnt[i];
    if (off.back() == 0) return;
    stages.push_back(Stage{kind, cls, args, blob.put(off), (int)cnt.size(), off.back(), lds});
  };
  auto spl_lds = [](const Problem& P) { return (size_t)8 * P.nn * sizeof(double); };
  // 0. operands to FP32
  std::vector<GVec> vec;
  std::vector<int> vcnt;
  for (int i = 0; i < n; ++i) {
    const Problem& P = ctxs[i]->pb;
    const long long N = 4LL * P.nz * P.nd * P.nn;
    const int nb = std::min(ceil_div(N, 256), 1024);
    vec.push_back(GVec{N, nb, x[i], ctxs[i]->wk.v32a, nullptr,
                       y[i]});
    vcnt.push_back(nb);
  }
  const size_t vec_at = blob.put(vec);
  add_stage(SK_TO32, 0, vec_at, vcnt, 0);
  // 1. comoving interpolation, every height
  {
    std::vector<GSpline> a;
    std::vector<int> cnt;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      a.push_back(GSpline{0, P.nd, P.nn, P.d_x, P.d_SigT, P.d_lam, P.d_ub, -1.0, nullptr, 1, 0, ctxs[i]->wk.v32a,
                          (long long)P.nd * P.nn * 4, (long long)P.nn * 4, static_cast<float*>(ctxs[i]->wk.Ibar[1]),
                          0, nullptr, nullptr});
      cnt.push_back(P.nz * P.nd);
      lds = std::max(lds, spl_lds(P));
    }
    add_stage(SK_SPLINE, 0, blob.put(a), cnt, lds);
  }
  // 2. R_III incoming factors
  {
    std::vector<GR3Y> ay;
    std::vector<GR3X> ax;
    std::vector<int> cy, cx;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      Work& K = ctxs[i]->wk;
      ay.push_back(GR3Y{0, P.nz, P.nt, P.nd, P.nn, ctxs[i]->pre.d_r3, static_cast<const float*>(K.Ibar[1]), K.Y});
      ax.push_back(GR3X{0, P.nu, P.nl, P.nd, P.d_w, P.d_A, K.Y, K.X});
      cy.push_back(ceil_div((long long)P.nz * P.nt * P.nd * 4, 256));
      cx.push_back(P.nz * P.nu * P.nu * P.nl);
    }
    add_stage(SK_R3Y, 0, blob.put(ay), cy, 0);
    add_stage(SK_R3X, 0, blob.put(ax), cx, 0);
  }
  // 3-4. per height chunk (W holds one chunk of each context): the R_II
  //      contraction, one launch per K-chunk class, then the angular /
  //      sublevel sum, one launch per sublevel class, over every context that
  //      has that chunk (the solver groups single-chunk contexts only; the
  //      walk itself takes any chunk count)
  int maxch = 0;
  for (int i = 0; i < n; ++i) maxch = std::max(maxch, ceil_div(ctxs[i]->pb.nz, ctxs[i]->wk.zchunk));
  for (int ch = 0; ch < maxch; ++ch) {
    std::map<int, std::vector<int>> by_nh, by_nl;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      if (ch * ctxs[i]->wk.zchunk >= P.nz) continue;
      by_nl[nl_class(P.nl)].push_back(i);
      // a chunk with at least two tiles per compute unit fills the device on
      // its own: it keeps the persistent pipelined contraction (launched here,
      // on the batch stream); smaller ones share one launch
      const int zc = std::min(ctxs[i]->wk.zchunk, P.nz - ch * ctxs[i]->wk.zchunk);
      const long long tiles = (long long)P.nqb * zc * ((int)P.cgrp[1].size() / 3);
      int nkc, nh;
      contract_chunks(P.ldm, &nkc, &nh);
      if (tiles >= 2LL * ctxs[i]->n_cu && contract_pipe_lds(nh, P.nslot) <= (size_t)ctxs[i]->max_lds) {
        stages.push_back(Stage{SK_CONTRACT_ONE, i, (size_t)ch, 0, 0, 0, 0});   // cls: context, args: chunk
        continue;
      }
      by_nh[nh].push_back(i);
    }
    for (auto& kv : by_nh) {
      std::vector<GContract> a;
      std::vector<int> cnt;
      for (int i : kv.second) {
        const Problem& P = ctxs[i]->pb;
        const int z0 = ch * ctxs[i]->wk.zchunk, zc = std::min(ctxs[i]->wk.zchunk, P.nz - z0);
        const int rb_n = P.nqb;
        const int ngrp = (int)P.cgrp[1].size() / 3;
        a.push_back(GContract{z0, P.nth, P.nt, P.nn, P.nd, P.cgrp_n8[1], P.nslot, zc, kernel_store(ctxs[i], true),
                              static_cast<const float*>(ctxs[i]->wk.Ibar[1]) + (size_t)z0 * P.nd * P.nn * 4,
                              P.d_cgrp[1], P.d_slot_dir, static_cast<float*>(ctxs[i]->wk.W[1])});
        cnt.push_back(rb_n * zc * ngrp);
      }
      add_stage(SK_CONTRACT, kv.first, blob.put(a), cnt,
                (size_t)8 * kv.first * ContractCfg<float>::BST * sizeof(float));
    }
    for (auto& kv : by_nl) {
      std::vector<GAngular> a;
      std::vector<int> cnt;
      for (int i : kv.second) {
        const Problem& P = ctxs[i]->pb;
        Work& K = ctxs[i]->wk;
        const int z0 = ch * K.zchunk, zc = std::min(K.zchunk, P.nz - z0);
        const int ncls = P.nl * P.nl;
        a.push_back(GAngular{z0, P.nd, P.nn, P.nu, P.nl, P.nslot, zc * P.nd, P.d_pair_slot, P.d_pair_index,
                             ctxs[i]->pre.d_cf32, static_cast<const float*>(K.W[1]), P.c_sc, P.d_E, P.d_bma, K.X,
                             ctxs[i]->pre.d_prof,
                             static_cast<float*>(K.Eb[1]) + (size_t)z0 * ncls * P.nd * P.nn * 4});
        cnt.push_back(zc * P.nd * ceil_div(P.nn, 64));
      }
      add_stage(SK_ANGULAR, kv.first, blob.put(a), cnt, 0);
    }
  }
  // 5. back to the observer frame, class by class in the single-context order;
  //    f on Stokes I in the same launch for one class, in a pass of its own over
  //    a copy for several
  int maxcls = 0;
  for (int i = 0; i < n; ++i) maxcls = std::max(maxcls, ctxs[i]->pb.nl * ctxs[i]->pb.nl);
  for (int c = 0; c < maxcls; ++c) {
    std::vector<GSpline> a;
    std::vector<int> cnt;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      const int ncls = P.nl * P.nl;
      if (c >= ncls) continue;
      const float* Eb = static_cast<const float*>(ctxs[i]->wk.Eb[1]);
      a.push_back(GSpline{0, P.nd, P.nn, P.d_x, P.d_SigT, P.d_lam, P.d_ub, 1.0, P.d_sll, ncls, c,
                          Eb + (size_t)c * P.nd * P.nn * 4, (long long)ncls * P.nd * P.nn * 4, (long long)P.nn * 4,
                          static_cast<float*>(ctxs[i]->wk.opeps[1]), c == 0 ? 0 : 1,
                          ncls == 1 ? ctxs[i]->pre.d_f : nullptr, nullptr});
      cnt.push_back(P.nz * P.nd);
      lds = std::max(lds, spl_lds(P));
    }
    add_stage(SK_SPLINE, 0, blob.put(a), cnt, lds);
  }
  {
    std::vector<GSpline> a;
    std::vector<int> cnt;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      if (P.nl == 1) continue;
      a.push_back(GSpline{0, P.nd, P.nn, P.d_x, P.d_SigT, P.d_lam, P.d_ub, 0.0, nullptr, 1, 0,
                          static_cast<const float*>(ctxs[i]->wk.tmp[1]), (long long)P.nd * P.nn * 4,
                          (long long)P.nn * 4, static_cast<float*>(ctxs[i]->wk.opeps[1]), 0, ctxs[i]->pre.d_f,
                          nullptr});
      cnt.push_back(P.nz * P.nd);
      lds = std::max(lds, spl_lds(P));
    }
    if (!a.empty()) {
      stages.push_back(Stage{SK_COPY, 0, 0, 0, 0, 0, 0});
      add_stage(SK_SPLINE, 0, blob.put(a), cnt, lds);
    }
  }
  // 6. formal solution Lambda of the emissivity, then y = x - Lambda Sigma x
  {
    std::vector<GFormal> a;
    std::vector<int> cnt;
    for (int i = 0; i < n; ++i) {
      const Problem& P = ctxs[i]->pb;
      a.push_back(GFormal{P.nz, P.nd, P.nn, ctxs[i]->formal_scheme, P.d_mu, P.d_tau, ctxs[i]->pre.d_K, P.d_WT,
                          static_cast<const float*>(ctxs[i]->wk.opeps[1]), ctxs[i]->wk.v32b});
      cnt.push_back(ceil_div((long long)P.nd * P.nn, 64));
    }
    add_stage(SK_FORMAL, 0, blob.put(a), cnt, 0);
  }
  for (int i = 0; i < n; ++i) vec[i].f32 = ctxs[i]->wk.v32b;
  add_stage(SK_FINISH, 0, blob.put(vec), vcnt, 0);
  // 7. the preconditioner of the contexts that ask for it, in place on y_i:
  //    the block-Jacobi steps of precond_apply, each kernel one launch over
  //    the contexts that still have that step
  int maxk = 0;
  for (int i = 0; pc && i < n; ++i)
    if (pc[i] > 0) {
      TRAP_TRY(precond_ensure(ctxs[i]));
      maxk = std::max(maxk, pc[i]);
    }
  auto pc_gather = [&](int step, auto src_of, int stride, bool phi) {
    std::vector<GPcCls> a;
    std::vector<GPcFin> b;
    std::vector<int> ca, cb;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      if (pc[i] < step) continue;
      const Problem& P = ctxs[i]->pb;
      const Precomp& C = ctxs[i]->pre;
      Work& K = ctxs[i]->wk;
      a.push_back(GPcCls{P.nd, P.nn, C.pc_ncmax, stride, P.d_x, P.d_SigT, P.d_lam, P.d_w, C.d_pcMem, C.d_pcMoff,
                         C.d_pcNcls, C.d_pcCub, src_of(i), K.pc_gc});
      b.push_back(GPcFin{P.nn, C.pc_ncmax, P.d_SigT, C.d_pcNcls, K.pc_gc, phi ? C.d_pcPhi : C.d_pcC, K.pc_h});
      ca.push_back(P.nz * C.pc_ncmax);
      cb.push_back(P.nz);
      lds = std::max(lds, pc_gather_lds(P.nn));
    }
    add_stage(SK_PC_CLS, 0, blob.put(a), ca, lds);
    add_stage(SK_PC_FIN, 0, blob.put(b), cb, lds);
  };
  auto pc_scatter = [&](int step, int mode, auto fill) {
    std::vector<GPcScat> a;
    std::vector<int> cnt;
    for (int i = 0; i < n; ++i) {
      if (pc[i] < step) continue;
      const Problem& P = ctxs[i]->pb;
      GPcScat g{mode, P.nz, P.nd, P.nn, 0, 1, P.d_x, P.d_lam, P.d_ub, ctxs[i]->wk.pc_h, ctxs[i]->pre.d_pcL,
                nullptr, nullptr, nullptr, nullptr};
      fill(i, g);
      a.push_back(g);
      cnt.push_back(ceil_div((long long)P.nz * P.nd * P.nn, 256));
    }
    add_stage(SK_PC_SCAT, 0, blob.put(a), cnt, 0);
  };
  for (int step = 1; step <= maxk; ++step) {
    if (step == 1) {
      pc_gather(1, [&](int i) { return (const double*)y[i]; }, 4, false);
      pc_scatter(1, 0, [&](int i, GPcScat& g) {       // x_1 = P^^-1 y
        g.src = y[i];
        g.src_stride = 4;
        const bool last = pc[i] == 1;
        g.dst = last ? y[i] : ctxs[i]->wk.pc_x;
        g.dst_stride = last ? 4 : 1;
      });
      continue;
    }
    pc_gather(step, [&](int i) { return (const double*)ctxs[i]->wk.pc_x; }, 1, true);
    pc_scatter(step, 1, [&](int i, GPcScat& g) { g.dst = ctxs[i]->wk.pc_e; });   // Sigma* x
    {
      std::vector<GPcSweep> a;
      std::vector<int> cnt;
      for (int i = 0; i < n; ++i) {
        if (pc[i] < step) continue;
        const Problem& P = ctxs[i]->pb;
        Work& K = ctxs[i]->wk;
        a.push_back(GPcSweep{P.nz, P.nd, P.nn, 4, P.d_mu, ctxs[i]->pre.d_pcF, ctxs[i]->pre.d_pcL, K.pc_e, y[i],
                             K.pc_x, K.pc_res});
        cnt.push_back(ceil_div((long long)P.nd * P.nn, 64));
      }
      add_stage(SK_PC_SWEEP, 0, blob.put(a), cnt, 0);
    }
    pc_gather(step, [&](int i) { return (const double*)ctxs[i]->wk.pc_res; }, 1, false);
    pc_scatter(step, 2, [&](int i, GPcScat& g) {      // x += P^^-1 res
      g.xin = ctxs[i]->wk.pc_x;
      g.res = ctxs[i]->wk.pc_res;
      const bool last = pc[i] == step;
      g.dst = last ? y[i] : ctxs[i]->wk.pc_x;
      g.dst_stride = last ? 4 : 1;
    });
  }

  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto it = g_arena.find(device);
  if (it == g_arena.end()) return fail(TRAP_ESTATE, "internal: no batch arena for the device");
  BatchArena& ar = it->second;
  TRAP_TRY(arena_ready(ar, blob.h.size(), n));
  // the batch starts after each context's pending work ...
  for (int i = 0; i < n; ++i) {
    TRAP_HIP(hipEventRecord(ar.ev[i], ctxs[i]->stream));
    TRAP_HIP(hipStreamWaitEvent(ar.stream, ar.ev[i], 0));
  }
  std::memcpy(ar.host, blob.h.data(), blob.h.size());
  TRAP_HIP(hipMemcpyAsync(ar.dev, ar.host, blob.h.size(), hipMemcpyHostToDevice, ar.stream));
  TRAP_HIP(hipEventRecord(ar.copied, ar.stream));
  const unsigned char* base = static_cast<const unsigned char*>(ar.dev);
  // every exit after the first launch goes through the join below, so the
  // contexts' streams stay ordered after whatever the batch stream has begun
  auto launch_stages = [&]() -> int {
  for (const Stage& st : stages) {
    const int* off = reinterpret_cast<const int*>(base + st.off);
    const void* args = base + st.args;
    switch (st.kind) {
      case SK_TO32:
        hipLaunchKernelGGL(k_to_f32_grouped, dim3(st.blocks), dim3(256), 0, ar.stream,
                           static_cast<const GVec*>(args), off, st.n);
        break;
      case SK_FINISH:
        hipLaunchKernelGGL(k_finish_grouped, dim3(st.blocks), dim3(256), 0, ar.stream,
                           static_cast<const GVec*>(args), off, st.n);
        break;
      case SK_SPLINE:
        hipLaunchKernelGGL(k_spline_shift_grouped, dim3(st.blocks), dim3(128), st.lds, ar.stream,
                           static_cast<const GSpline*>(args), off, st.n);
        break;
      case SK_R3Y:
        hipLaunchKernelGGL(k_r3_Y_grouped, dim3(st.blocks), dim3(256), 0, ar.stream,
                           static_cast<const GR3Y*>(args), off, st.n);
        break;
      case SK_R3X:
        hipLaunchKernelGGL(k_r3_X_grouped, dim3(st.blocks), dim3(256), 0, ar.stream,
                           static_cast<const GR3X*>(args), off, st.n);
        break;
      case SK_CONTRACT: {
        const GContract* a = static_cast<const GContract*>(args);
        switch (st.cls) {
#define TRAP_GCONTRACT_CASE(NHV)                                                                              \
  case NHV:                                                                                                   \
    hipLaunchKernelGGL(k_contract_grouped<NHV>, dim3(st.blocks), dim3(512), st.lds, ar.stream, a, off, st.n); \
    break;
          TRAP_GCONTRACT_CASE(1) TRAP_GCONTRACT_CASE(2) TRAP_GCONTRACT_CASE(3) TRAP_GCONTRACT_CASE(4)
          TRAP_GCONTRACT_CASE(5) TRAP_GCONTRACT_CASE(6) TRAP_GCONTRACT_CASE(7) TRAP_GCONTRACT_CASE(8)
          TRAP_GCONTRACT_CASE(9) TRAP_GCONTRACT_CASE(10) TRAP_GCONTRACT_CASE(11) TRAP_GCONTRACT_CASE(12)
          TRAP_GCONTRACT_CASE(13) TRAP_GCONTRACT_CASE(14) TRAP_GCONTRACT_CASE(15) TRAP_GCONTRACT_CASE(16)
#undef TRAP_GCONTRACT_CASE
          default:
            return fail(TRAP_EINVAL, "internal: bad contraction chunk");
        }
        break;
      }
      case SK_ANGULAR: {
        const GAngular* a = static_cast<const GAngular*>(args);
        auto kern = st.cls == 1 ? k_angular_grouped<1>
                  : st.cls == 2 ? k_angular_grouped<2>
                  : st.cls == 4 ? k_angular_grouped<4> : k_angular_grouped<8>;
        hipLaunchKernelGGL(kern, dim3(st.blocks), dim3(64 * kAngQ), 0, ar.stream, a, off, st.n);
        break;
      }
      case SK_COPY:
        for (int i = 0; i < n; ++i) {
          const Problem& P = ctxs[i]->pb;
          if (P.nl == 1) continue;
          TRAP_HIP(hipMemcpyAsync(ctxs[i]->wk.tmp[1], ctxs[i]->wk.opeps[1],
                                  (size_t)4 * P.nz * P.nd * P.nn * sizeof(float), hipMemcpyDeviceToDevice,
                                  ar.stream));
        }
        break;
      case SK_CONTRACT_ONE: {
        // cls: the context, args: the height chunk
        trap_ctx* c = ctxs[st.cls];
        const Problem& P = c->pb;
        const int z0 = (int)st.args * c->wk.zchunk, zc = std::min(c->wk.zchunk, P.nz - z0);
        const float* Ib = static_cast<const float*>(c->wk.Ibar[1]) + (size_t)z0 * P.nd * P.nn * 4;
        float* Wc = static_cast<float*>(c->wk.W[1]);
        int launched = launch_contract_res(c, ar.stream, zc, z0, Ib, Wc);
        if (launched == 0) launched = launch_contract_pipe(c, ar.stream, zc, z0, Ib, Wc);
        if (launched < 0) return launched;
        if (!launched) return fail(TRAP_EINVAL, "internal: contraction does not fit the pipelined kernel");
        break;
      }
      case SK_FORMAL:
        TRAP_TRY(launch_formal_grouped(ar.stream, static_cast<const GFormal*>(args), off, st.n, st.blocks));
        break;
      case SK_PC_CLS:
      case SK_PC_FIN:
      case SK_PC_SCAT:
        TRAP_TRY(launch_pc_grouped(ar.stream, st.kind - SK_PC_CLS, args, off, st.n, st.blocks, st.lds));
        break;
      case SK_PC_SWEEP:
        TRAP_TRY(launch_pc_sweep_grouped(ar.stream, static_cast<const GPcSweep*>(args), off, st.n, st.blocks));
        break;
    }
    TRAP_HIP(hipGetLastError());
  }
  // ... and each context's later work waits for the batch
  return TRAP_OK;
  };
  const int rc = launch_stages();
  const hipError_t e = hipEventRecord(ar.done, ar.stream);
  bool joined = e == hipSuccess;
  for (int i = 0; i < n && joined; ++i) joined = hipStreamWaitEvent(ctxs[i]->stream, ar.done, 0) == hipSuccess;
  if (!joined) {
    // without the join, wait for the batch here before any context reuses its buffers
    (void)hipGetLastError();
    const hipError_t w = hipStreamSynchronize(ar.stream);
    if (rc == TRAP_OK)
      return fail(TRAP_EDEVICE, std::string("joining the shared launches: ") +
                                    hipGetErrorString(e != hipSuccess ? e : w));
  }
  return rc;
}

}  // namespace trap
