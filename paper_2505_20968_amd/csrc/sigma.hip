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

#include "trap_internal.h"

namespace trap {

static constexpr double kInvPi = 0.31830988618379067154;

// ------------------------------------------------------------------ spline evaluation
// out[z][o][n][s] (+)= S[in[z][o][:][s]](x_n + shift) for one (l, l') class,
// flat extension outside [x_0, x_{nn-1}];  shift (x units) =
// (ub_sign * ub[z][o] + sll[z][cls]) / lam[z].  One block per (z, o): the
// column goes to LDS, the spline's second derivatives s = Sig v (Sig^T stored,
// so the reads are coalesced) are formed once, then every frequency evaluates
//   S(x) = (1-t) v_k + t v_{k+1} + h^2 [((1-t)^3 - (1-t)) s_k + (t^3 - t) s_{k+1}] / 6.
// Optionally multiplies Stokes I by f and adds eps_th.
template <typename T>
__global__ void __launch_bounds__(128) k_spline_shift(
    int nz0, int nzc, int nd, int nn, const double* __restrict__ x, const double* __restrict__ SigT,
    const double* __restrict__ lam, const double* __restrict__ ub, double ub_sign,
    const double* __restrict__ sll, int ncls, int cls, const T* __restrict__ in, long long in_z_stride,
    long long in_o_stride, T* __restrict__ out, int accumulate, const double* __restrict__ f,
    const double* __restrict__ epsth) {
  extern __shared__ double spl[];
  double* v = spl;               // [nn][4]
  double* sd = spl + 4 * nn;     // [nn][4]
  const int zl = blockIdx.x / nd, o = blockIdx.x % nd;
  const int z = nz0 + zl;
  const double L = lam[z];
  double sh = ub_sign * ub[(long long)z * nd + o];
  if (sll) sh += sll[(long long)z * ncls + cls];
  const T* src = in + zl * in_z_stride + o * in_o_stride;
  const bool shifted = sh != 0.0;
  if (shifted) {
    for (int e = threadIdx.x; e < 4 * nn; e += blockDim.x) v[e] = (double)src[e];
    __syncthreads();
    for (int m = threadIdx.x; m < nn; m += blockDim.x) {
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
        const double h = x[lo + 1] - x[lo];
        const double t = (xs - x[lo]) / h, u = 1.0 - t;
        const double cs = h * h / 6.0;
        const double wk = cs * (u * u * u - u), wk1 = cs * (t * t * t - t);
        for (int q = 0; q < 4; ++q)
          val[q] = u * v[4 * lo + q] + t * v[4 * lo + 4 + q] + wk * sd[4 * lo + q] + wk1 * sd[4 * lo + 4 + q];
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

// ------------------------------------------------------------------ R_II contraction
// One GEMM per (z, theta) over every transition at once:
//   C[(t, c, n), (sl, s)] = sum_m M[z][theta][(t, c, n)][m] * Ibar[z][dir(sl)][m][s]
// rows R = 2 nt nn (transition, real/imaginary plane, frequency), columns
// 4 nslots(theta) (incoming-direction slot, Stokes), K = nn.  Matrix cores:
// v_mfma_{f32,f64}_16x16x4 with the operands swapped (A_in = B^T, B_in = M^T)
// so that each lane's four accumulators are the four Stokes components of one
// (row, slot) entry of W -- one contiguous 16/32-byte store.
// Block: 4 waves, 64 rows (16 per wave) x up to 256 columns (16 column tiles
// held in registers), K staged through LDS in chunks of KC.
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaOp;
// Output layouts differ: for the f32 16x16x4 instruction lane l holds rows
// 4 (l/16) + r of the 16x16 result, for the f64 one rows (l/16) + 4 r.  The f64
// path stores the B tile with its 16 columns transposed as a 4x4 grid so that
// both end up with one slot's four Stokes values per lane.
template <> struct MfmaOp<float> {
  typedef floatx4_t acc_t;
  static constexpr int KC = 32;
  static constexpr bool kInterleavedRows = false;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaOp<double> {
  typedef doublex4_t acc_t;
  static constexpr int KC = 16;
  static constexpr bool kInterleavedRows = true;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int kMaxColTiles = 16;   // 256 columns = 64 slots per column group
constexpr int kRowsPerBlock = 128; // 8 waves x 16 rows

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

// Block: 8 waves = 128 rows (16 per wave) x up to 256 columns (16 column tiles in
// registers).  K is staged through LDS in chunks of KC with the next chunk's
// global loads issued before the current chunk's matrix-core work (register
// double buffering).  LDS row strides are 16 (mod 64) elements so the four
// k-rows of a fragment read fall in different bank groups.
template <typename T>
__global__ void __launch_bounds__(512) k_contract(int z0, int nth, int nt, int nn, int ldm, int nd,
                                                  const T* __restrict__ M, const T* __restrict__ Ibar,
                                                  const int* __restrict__ slot_off,
                                                  const int* __restrict__ slot_dir, T* __restrict__ W,
                                                  int nslot) {
  using Op = MfmaOp<T>;
  using acc_t = typename Op::acc_t;
  using V4 = typename Vec4<T>::type;
  constexpr int KC = Op::KC;
  constexpr int NCOL = kMaxColTiles * 16;
  constexpr int AST = kRowsPerBlock + 16;   // As[k][row]
  constexpr int BST = NCOL + 16;            // Bs[k][col]
  constexpr int APT = KC / 4;               // A elements per thread per chunk (row, 4 threads per row)
  constexpr int BPT = KC / 8;               // B k-rows per thread per chunk (8 k-lanes)
  __shared__ T As[KC * AST];
  __shared__ T Bs[KC * BST];
  const int th = blockIdx.y;
  const int zl = blockIdx.z;
  const int z = z0 + zl;
  const int R = 2 * nt * nn;
  const int row0 = blockIdx.x * kRowsPerBlock;
  if (row0 >= R) return;
  const int s0 = slot_off[th], ns = slot_off[th + 1] - s0;
  const T* Mb = M + ((size_t)z * nth + th) * (size_t)R * ldm;
  const T* Ib = Ibar + (size_t)zl * nd * nn * 4;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  // loader roles
  const int a_row = tid >> 2, a_kq = tid & 3;          // A: 4 threads per row, APT consecutive k each
  const int b_sl = tid & 63, b_ky = tid >> 6;          // B: one slot per lane, k rows b_ky + 8 i
  const int ga_row = row0 + a_row;
  const T* a_src = Mb + (size_t)min(ga_row, R - 1) * ldm;
  // output coordinates of this lane's row
  const int grow = row0 + wave * 16 + lr;
  const int rt = grow / (2 * nn), rc = (grow / nn) & 1, rn = grow % nn;
  const int nchunks = (nn + KC - 1) / KC;
  for (int sg0 = 0; sg0 < ns; sg0 += NCOL / 4) {
    const int nsg = min(NCOL / 4, ns - sg0);      // slots in this column group
    const int nsub = (4 * nsg + 15) >> 4;
    const bool b_live = b_sl < nsg;
    const int b_dir = b_live ? slot_dir[s0 + sg0 + b_sl] : 0;
    const T* b_src = Ib + (size_t)b_dir * nn * 4;
    const bool b_store = b_sl < 4 * nsub;        // zero-fill padded columns of the last tile
    acc_t acc[kMaxColTiles];
#pragma unroll
    for (int j = 0; j < kMaxColTiles; ++j)
      for (int r = 0; r < 4; ++r) acc[j][r] = T(0);
    T ra[APT];
    V4 rb[BPT];
    auto load = [&](int k0) {
#pragma unroll
      for (int i = 0; i < APT; ++i) {
        const int gk = k0 + a_kq * APT + i;
        ra[i] = (ga_row < R && gk < ldm) ? a_src[gk] : T(0);
      }
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        const int gk = k0 + b_ky + 8 * i;
        if (b_live && gk < nn) {
          rb[i] = *reinterpret_cast<const V4*>(b_src + (size_t)gk * 4);
        } else {
          rb[i].x = T(0); rb[i].y = T(0); rb[i].z = T(0); rb[i].w = T(0);
        }
      }
    };
    load(0);
    for (int c = 0; c < nchunks; ++c) {
      const int k0 = c * KC;
      if (c > 0) __syncthreads();
#pragma unroll
      for (int i = 0; i < APT; ++i) As[(a_kq * APT + i) * AST + a_row] = ra[i];
      if (b_store) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
          T* dst = Bs + (b_ky + 8 * i) * BST;
          const T v[4] = {rb[i].x, rb[i].y, rb[i].z, rb[i].w};
          if (Op::kInterleavedRows) {
            const int base = (b_sl >> 2) * 16 + (b_sl & 3);
            for (int q = 0; q < 4; ++q) dst[base + 4 * q] = v[q];
          } else {
            for (int q = 0; q < 4; ++q) dst[4 * b_sl + q] = v[q];
          }
        }
      }
      __syncthreads();
      if (c + 1 < nchunks) load(k0 + KC);
      const int ksteps = (min(KC, nn - k0) + 3) >> 2;
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        if (ks < ksteps) {
          const T bf = As[(ks * 4 + lk) * AST + wave * 16 + lr];
#pragma unroll
          for (int j = 0; j < kMaxColTiles; ++j) {
            if (j < nsub) {
              const T af = Bs[(ks * 4 + lk) * BST + j * 16 + lr];
              acc[j] = Op::run(af, bf, acc[j]);
            }
          }
        }
      }
    }
    __syncthreads();
    // lane holds C[grow][16 j + 4 lk + r], r = 0..3 -> slot 4 j + lk, Stokes r
    if (grow < R) {
#pragma unroll
      for (int j = 0; j < kMaxColTiles; ++j) {
        const int sl = 4 * j + lk;
        if (j < nsub && sl < nsg) {
          V4 o;
          o.x = acc[j][0]; o.y = acc[j][1]; o.z = acc[j][2]; o.w = acc[j][3];
          *reinterpret_cast<V4*>(W + (((((size_t)zl * nt + rt) * nslot + s0 + sg0 + sl) * 2 + rc) * nn + rn) * 4) = o;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ R_III factors
// Y[z][t][o][s] = sum_m r3[z][t][m] Ibar[z][o][m][s]
template <typename T>
__global__ void k_r3_Y(int z0, int nzc, int nt, int nd, int nn, const double2* __restrict__ r3,
                       const T* __restrict__ Ibar, double2* __restrict__ Y) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
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

// X[z][u][u'][l] = sum_o' w_o' sum_j A[z][o'][j][u][u'][l] (Y[(u',l)][o'][j] + conj Y[(u,l)][o'][j])
__global__ void k_r3_X(int z0, int nu, int nl, int nd, const double* __restrict__ w,
                       const double2* __restrict__ A, const double2* __restrict__ Y,
                       double2* __restrict__ X) {
  const int e = blockIdx.x;   // (zl, u, up, l)
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

// ------------------------------------------------------------------ angular / sublevel sum
// One block per (zl, mu index, block of 32 frequencies); thread (k, n) handles
// outgoing direction (mu, chi_k) at one frequency, so the mirror directions
// that read the same W slot sit in one block.  For a chunk of incoming
// directions the 4x4 coefficients
//   C^{u' l, l'}_ij(o, o') = (c_sc w_o'/pi) sum_u alpha_{u u'} E_i(o; u', u, l') A_j(o'; u, u', l)
// are built in LDS by the whole block; the accumulation Re sum_j C_ij W_j then
// runs without barriers.
constexpr int kAngN = 32;

template <typename T>
__global__ void __launch_bounds__(512) k_angular(
    int z0, int nd, int nchi, int nn, int nu, int nl, int nslot, int oc_max, double c_sc,
    const double* __restrict__ w, const double2* __restrict__ E, const double2* __restrict__ A,
    const double2* __restrict__ alpha, const double2* __restrict__ bma, const int* __restrict__ pair_slot,
    const T* __restrict__ W, const double2* __restrict__ X, const double2* __restrict__ prof,
    T* __restrict__ Eb) {
  extern __shared__ double2 sh[];
  const int nmu = nd / nchi;
  const int zl = blockIdx.x / nmu, imu = blockIdx.x % nmu;
  const int z = z0 + zl;
  const int nt = nu * nl;
  const int o_first = imu * nchi;
  const int k = threadIdx.x / kAngN;
  const int n = blockIdx.y * kAngN + (threadIdx.x % kAngN);
  const bool active = n < nn && k < nchi;
  const int o = o_first + k;
  double2* Cs = sh;
  int* slots = reinterpret_cast<int*>(sh + (size_t)oc_max * nu * nchi * nl * 16);
  double2* Ds = sh;
  for (int l = 0; l < nl; ++l) {
    double acc[8][4];
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 4; ++i) acc[a][i] = 0.0;
    for (int o0 = 0; o0 < nd; o0 += oc_max) {
      const int oc_n = min(oc_max, nd - o0);
      __syncthreads();
      const int nC = oc_n * nu * nchi * nl * 16;
      for (int e = threadIdx.x; e < nC; e += blockDim.x) {
        const int j = e & 3, i = (e >> 2) & 3;
        int r = e >> 4;
        const int lp = r % nl; r /= nl;
        const int kk = r % nchi; r /= nchi;
        const int upr = r % nu; r /= nu;
        const int oc = r;
        const int oo = o_first + kk, op = o0 + oc;
        const double2* Ez = E + ((size_t)z * nd + oo) * 4 * nu * nu * nl;
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
        const double sc = c_sc * w[op] * kInvPi;
        Cs[e] = make_double2(sc * re, sc * im);
      }
      for (int e = threadIdx.x; e < oc_n * nchi; e += blockDim.x) {
        const int oc = e / nchi, kk = e % nchi;
        slots[e] = pair_slot[(o_first + kk) * nd + o0 + oc];
      }
      __syncthreads();
      if (!active) continue;
      for (int oc = 0; oc < oc_n; ++oc) {
        const int sl = slots[oc * nchi + k];
        for (int upr = 0; upr < nu; ++upr) {
          const int t = upr * nl + l;
          const T* Wp = W + (((size_t)zl * nt + t) * nslot + sl) * 2 * (size_t)nn * 4;
          typedef typename Vec4<T>::type V4;
          const V4 a = *reinterpret_cast<const V4*>(Wp + (size_t)n * 4);
          const V4 b = *reinterpret_cast<const V4*>(Wp + (size_t)nn * 4 + (size_t)n * 4);
          const double wr[4] = {(double)a.x, (double)a.y, (double)a.z, (double)a.w};
          const double wi[4] = {(double)b.x, (double)b.y, (double)b.z, (double)b.w};
          const double2* Cb = Cs + (((size_t)oc * nu + upr) * nchi + k) * nl * 16;
          for (int lp = 0; lp < nl; ++lp)
            for (int i = 0; i < 4; ++i) {
              double v = 0.0;
              for (int jj = 0; jj < 4; ++jj) {
                const double2 c = Cb[(lp * 4 + i) * 4 + jj];
                v += c.x * wr[jj] - c.y * wi[jj];
              }
              acc[lp][i] += v;
            }
        }
      }
    }
    // R_III: D[k][l'][i][u][u'] = c_sc/(4 pi) (beta-alpha)_{u u'} E_i(o; u', u, l') X[u][u'][l]
    __syncthreads();
    const int nD = nchi * nl * 4 * nu * nu;
    for (int e = threadIdx.x; e < nD; e += blockDim.x) {
      const int upr = e % nu, u = (e / nu) % nu, i = (e / (nu * nu)) % 4;
      const int lp = (e / (4 * nu * nu)) % nl, kk = e / (4 * nu * nu * nl);
      const double2* Ez = E + ((size_t)z * nd + o_first + kk) * 4 * nu * nu * nl;
      const double2 b = bma[((size_t)z * nu + u) * nu + upr];
      const double2 ee = Ez[((size_t)(i * nu + upr) * nu + u) * nl + lp];
      const double2 xx = X[(((size_t)z * nu + u) * nu + upr) * nl + l];
      const double2 v = cmul(b, cmul(ee, xx));
      const double sc = c_sc * 0.25 * kInvPi;
      Ds[e] = make_double2(sc * v.x, sc * v.y);
    }
    __syncthreads();
    if (active) {
      for (int lp = 0; lp < nl; ++lp)
        for (int i = 0; i < 4; ++i) {
          double v = 0.0;
          for (int u = 0; u < nu; ++u)
            for (int upr = 0; upr < nu; ++upr) {
              const double2 d = Ds[(((k * nl + lp) * 4 + i) * nu + u) * nu + upr];
              const double2 p1 = prof[((size_t)z * nt + upr * nl + l) * nn + n];
              const double2 p2 = prof[((size_t)z * nt + u * nl + l) * nn + n];
              v += d.x * (p1.x + p2.x) - d.y * (p1.y - p2.y);
            }
          acc[lp][i] += v;
        }
      for (int lp = 0; lp < nl; ++lp) {
        T* dst = Eb + ((((size_t)zl * nl + l) * nl + lp) * nd + o) * (size_t)nn * 4 + (size_t)n * 4;
        for (int i = 0; i < 4; ++i) dst[i] = (T)acc[lp][i];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ driver
static size_t elem_size(int prec) { return prec == TRAP_FP64 ? sizeof(double) : sizeof(float); }

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
    // height chunk: keep one chunk of W (FP64) within ~1 GiB
    const size_t per_z = (size_t)P.nt * P.nslot * 2 * nn * 4 * sizeof(double);
    K.zchunk = (int)std::max<size_t>(1, std::min<size_t>(nz, (size_t(1) << 30) / std::max<size_t>(per_z, 1)));
  }
  const int pi = prec == TRAP_FP64 ? 0 : 1;
  if (!K.W[pi]) {
    const size_t es = elem_size(prec);
    const size_t zc = K.zchunk;
    TRAP_TRY(dalloc(ctx, &K.Ibar[pi], zc * nd * nn * 4 * es));
    TRAP_TRY(dalloc(ctx, &K.W[pi], zc * P.nt * P.nslot * 2 * nn * 4 * es));
    TRAP_TRY(dalloc(ctx, &K.Eb[pi], nz * P.nl * P.nl * nd * nn * 4 * es));
    TRAP_TRY(dalloc(ctx, &K.tmp[pi], N * es));
    TRAP_TRY(dalloc(ctx, &K.opeps[pi], N * es));
  }
  return TRAP_OK;
}

template <typename T>
static int sigma_apply_t(trap_ctx* ctx, const T* I, T* eps, int prec, int add_thermal, int normalize,
                         const T* Mk) {
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
  for (int z0 = 0; z0 < nz; z0 += K.zchunk) {
    const int zc = std::min(K.zchunk, nz - z0);
    const long long npts = (long long)zc * nd * nn;
    // 1. comoving interpolation
    int pr = prof_begin(ctx, TRAP_STAGE_COMOVING);
    hipLaunchKernelGGL(k_spline_shift<T>, dim3(zc * nd), dim3(128), spl_lds, s, z0, zc, nd, nn, P.d_x,
                       P.d_SigT, P.d_lam, P.d_ub, -1.0, (const double*)nullptr, 1, 0,
                       I + (size_t)z0 * nd * nn * 4, (long long)nd * nn * 4, (long long)nn * 4, Ibar, 0,
                       (const double*)nullptr, (const double*)nullptr);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    // 2. contraction
    dim3 grid(ceil_div(2LL * nt * nn, kRowsPerBlock), nth, zc);
    {
      const double kel = (double)zc * nth * nt * 2.0 * nn * P.ldm;
      const double flops = 16.0 * zc * nt * (double)nn * nn * P.nslot;
      const double bytes = sizeof(T) * (kel + (double)zc * nt * P.nslot * 2.0 * nn * 4 + (double)zc * nd * nn * 4);
      pr = prof_begin(ctx, sizeof(T) == 8 ? TRAP_STAGE_CONTRACT_FP64 : TRAP_STAGE_CONTRACT, flops, bytes);
    }
    hipLaunchKernelGGL(k_contract<T>, grid, dim3(512), 0, s, z0, nth, nt, nn, P.ldm, nd, Mk, Ibar,
                       P.d_slot_off, P.d_slot_dir, W, P.nslot);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    // 3. R_III factors
    pr = prof_begin(ctx, TRAP_STAGE_R3);
    const long long ny = (long long)zc * nt * nd * 4;
    hipLaunchKernelGGL(k_r3_Y<T>, dim3(ceil_div(ny, 256)), dim3(256), 0, s, z0, zc, nt, nd, nn, C.d_r3,
                       Ibar, K.Y);
    TRAP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_r3_X, dim3(zc * nu * nu * nl), dim3(256), 0, s, z0, nu, nl, nd, P.d_w, P.d_A,
                       K.Y, K.X);
    TRAP_HIP(hipGetLastError());
    prof_end(ctx, pr);
    // 4. angular / sublevel sum into Eb (chunk-local heights)
    pr = prof_begin(ctx, TRAP_STAGE_ANGULAR);
    {
      const int nchi = P.nchi;
      const size_t per_oc = (size_t)nu * nchi * nl * 16 * sizeof(double2) + nchi * sizeof(int);
      const int oc_max = (int)std::max<size_t>(1, std::min<size_t>(nd, (48u << 10) / per_oc));
      const size_t shb = std::max((size_t)oc_max * per_oc + 64,
                                  (size_t)nchi * nl * 4 * nu * nu * sizeof(double2));
      hipLaunchKernelGGL(k_angular<T>, dim3(zc * (nd / nchi), ceil_div(nn, kAngN)), dim3(kAngN * nchi), shb, s, z0, nd,
                         nchi, nn, nu, nl, P.nslot, oc_max, P.c_sc, P.d_w, P.d_E, P.d_A, P.d_alpha, P.d_bma,
                         P.d_pair_slot, W, K.X, C.d_prof, Eb + (size_t)z0 * ncls * nd * nn * 4);
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
                         (add_thermal && last && ncls == 1) ? C.d_epsth : (const double*)nullptr);
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
                       add_thermal ? C.d_epsth : (const double*)nullptr);
    TRAP_HIP(hipGetLastError());
  }
  prof_end(ctx, prb);
  return TRAP_OK;
}

int sigma_apply(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal, int normalize) {
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (!ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (prec != TRAP_FP64 && prec != TRAP_FP32) return fail(TRAP_EINVAL, "unknown precision");
  if (!I || !eps) return fail(TRAP_EINVAL, "null vector");
  TRAP_TRY(ensure_work(ctx, prec));
  if (prec == TRAP_FP64) {
    if (!ctx->pre.d_M64) return fail(TRAP_ESTATE, "FP64 kernels not stored");
    return sigma_apply_t<double>(ctx, static_cast<const double*>(I), static_cast<double*>(eps), prec,
                                 add_thermal, normalize, ctx->pre.d_M64);
  }
  if (!ctx->pre.d_M32) return fail(TRAP_ESTATE, "FP32 kernels not stored (store_mask bit 1)");
  return sigma_apply_t<float>(ctx, static_cast<const float*>(I), static_cast<float*>(eps), prec,
                              add_thermal, normalize, ctx->pre.d_M32);
}

}  // namespace trap
