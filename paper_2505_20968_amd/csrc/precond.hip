// Physics-based preconditioner (paper Sect. 5.2) with the block-diagonal
// local inverse of App. F, applied as a fixed number of block-Jacobi steps.
//
// P = Id - Lambda* Sigma* acts on Stokes I only (Q, U, V pass through):
// Sigma* = Ups^{nubar->nu} Phi Phi^Omega Ups^{nu->nubar} per height
// (interpolation to the comoving grid per direction, angular mean, comoving
// coupling Phi_z, interpolation back) and Lambda* the scalar DELO-linear
// formal solution with the problem's eta_I.  The local blocks
// Id - Lambda_zz Sigma*_z are inverted in closed form,
//   P^_z^-1 r = r + Lambda_zz Ups^{nubar->nu} C_z Phi^Omega Ups^{nu->nubar} r,
//   C_z = Phi_z (Id - A_z)^-1 (tables from the precompute),
// and M r = x_k with x_1 = P^^-1 r, x_{j+1} = x_j + P^^-1 (r - P x_j): a
// fixed linear map, so left-preconditioned GMRES stays plain GMRES.
//
// Per step two kinds of kernels: a per-height one (angular mean of the
// comoving field, one N_nu x N_nu matrix-vector product, spline second
// derivatives of the result) and a per-point one (interpolation back to every
// direction, combined with the local Lambda and the running iterate); the
// sweeps add the scalar formal solution with the residual fused into it.
#include <mutex>
#include <string>
#include <vector>

#include "trap_internal.h"

namespace trap {

constexpr int kGatherThreads = 512;
constexpr int kGatherParts = 4;       // partial sums per output of the spline products

// sd = Sig v for one vector of N_nu values in LDS (SigT = Sig^T, so that
// consecutive threads read consecutive entries).  The block splits the sum
// over j into kGatherParts ranges (partial sums in part[kGatherParts][nn]),
// which shortens each thread's chain of dependent loads.  Ends synchronised.
__device__ inline void pc_second_derivs(int nn, const double* __restrict__ SigT, const double* v, double* part,
                                        double* sd) {
  const int per = (kGatherThreads / kGatherParts);
  const int q = threadIdx.x / per, i0 = threadIdx.x % per;
  const int j0 = q * nn / kGatherParts, j1 = (q + 1) * nn / kGatherParts;
  for (int i = i0; i < nn; i += per) {
    // four independent chains: four loads in flight per thread
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      a0 += SigT[(size_t)j * nn + i] * v[j];
      a1 += SigT[(size_t)(j + 1) * nn + i] * v[j + 1];
      a2 += SigT[(size_t)(j + 2) * nn + i] * v[j + 2];
      a3 += SigT[(size_t)(j + 3) * nn + i] * v[j + 3];
    }
    for (; j < j1; ++j) a0 += SigT[(size_t)j * nn + i] * v[j];
    part[q * nn + i] = (a0 + a1) + (a2 + a3);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < kGatherParts; ++r) a += part[r * nn + i];
    sd[i] = a;
  }
  __syncthreads();
}

// gc[z][c][.] = Ups_c (sum_{o in c} w_o src_o): the angular sum of Doppler
// class c of height z (members mem[moff[c] .. moff[c + 1])) interpolated to
// the comoving grid.  One block per (z, c); blocks past the height's class
// count return at once.
__device__ __forceinline__ void pc_gather_cls_body(int bx, int nd, int nn, int ncmax, const double* __restrict__ x,
                                                   const double* __restrict__ SigT, const double* __restrict__ lam,
                                                   const double* __restrict__ w, const int* __restrict__ mem,
                                                   const int* __restrict__ moff, const int* __restrict__ ncls,
                                                   const double* __restrict__ cub, const double* __restrict__ src,
                                                   int stride, double* __restrict__ gc) {
  extern __shared__ double sh[];     // pc_gather_lds(nn) bytes
  double* v = sh;
  double* sd = sh + nn;
  double* part = sh + 2 * nn;       // [kGatherParts][nn]
  double* xg = sh + (2 + kGatherParts) * nn;   // the frequency grid
  const int z = bx / ncmax, c = bx % ncmax;
  if (c >= ncls[z]) return;
  for (int n = threadIdx.x; n < nn; n += blockDim.x) xg[n] = x[n];
  const double shf = cub[(size_t)z * nd + c] / lam[z];
  const int* mz = mem + (size_t)z * nd;
  const int k0 = moff[(size_t)z * (nd + 1) + c], k1 = moff[(size_t)z * (nd + 1) + c + 1];
  for (int n = threadIdx.x; n < nn; n += blockDim.x) {
    double a0 = 0.0, a1 = 0.0;
    int k = k0;
    for (; k + 2 <= k1; k += 2) {
      const int o0 = mz[k], o1 = mz[k + 1];
      a0 += w[o0] * src[(((size_t)z * nd + o0) * nn + n) * stride];
      a1 += w[o1] * src[(((size_t)z * nd + o1) * nn + n) * stride];
    }
    if (k < k1) a0 += w[mz[k]] * src[(((size_t)z * nd + mz[k]) * nn + n) * stride];
    v[n] = a0 + a1;
  }
  __syncthreads();
  pc_second_derivs(nn, SigT, v, part, sd);
  double* g = gc + ((size_t)z * ncmax + c) * nn;
  for (int m = threadIdx.x; m < nn; m += blockDim.x) g[m] = spline_at(xg, nn, v, sd, xg[m] - shf);
}

__global__ void __launch_bounds__(kGatherThreads) k_pc_gather_cls(int nd, int nn, int ncmax,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ SigT,
                                                                  const double* __restrict__ lam,
                                                                  const double* __restrict__ w,
                                                                  const int* __restrict__ mem,
                                                                  const int* __restrict__ moff,
                                                                  const int* __restrict__ ncls,
                                                                  const double* __restrict__ cub,
                                                                  const double* __restrict__ src, int stride,
                                                                  double* __restrict__ gc) {
  pc_gather_cls_body(blockIdx.x, nd, nn, ncmax, x, SigT, lam, w, mem, moff, ncls, cub, src, stride, gc);
}

// hz = Mat_z sum_c gc[z][c] with one wave per row of Mat_z, then the spline
// second derivatives of hz; hz and them go to h[z][0][.] and h[z][1][.].
// One block per height.
__device__ __forceinline__ void pc_gather_fin_body(int bx, int nn, int ncmax, const double* __restrict__ SigT,
                                                   const int* __restrict__ ncls, const double* __restrict__ gc,
                                                   const double* __restrict__ Mat, double* __restrict__ h) {
  extern __shared__ double sh[];
  double* G = sh;
  double* hv = sh + nn;
  double* part = sh + 2 * nn;       // [kGatherParts][nn]
  const int z = bx, nc = ncls[z];
  const double* gz = gc + (size_t)z * ncmax * nn;
  for (int m = threadIdx.x; m < nn; m += blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < nc; ++c) a += gz[(size_t)c * nn + m];
    G[m] = a;
  }
  __syncthreads();
  const double* Mz = Mat + (size_t)z * nn * nn;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // four rows per wave at a time (their loads in flight together; rows past
  // the end read the last row and are not stored)
  for (int n0 = 4 * wave; n0 < nn; n0 += 4 * nw) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = lane; m < nn; m += 64) {
      const double g = G[m];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] += Mz[(size_t)min(n0 + r, nn - 1) * nn + m] * g;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      for (int off = 32; off > 0; off >>= 1) a[r] += __shfl_down(a[r], off, 64);
      if (lane == 0 && n0 + r < nn) hv[n0 + r] = a[r];
    }
  }
  __syncthreads();
  double* hz = h + (size_t)z * 2 * nn;
  pc_second_derivs(nn, SigT, hv, part, hz + nn);
  for (int i = threadIdx.x; i < nn; i += blockDim.x) hz[i] = hv[i];
}

__global__ void __launch_bounds__(kGatherThreads) k_pc_gather_fin(int nn, int ncmax,
                                                                  const double* __restrict__ SigT,
                                                                  const int* __restrict__ ncls,
                                                                  const double* __restrict__ gc,
                                                                  const double* __restrict__ Mat,
                                                                  double* __restrict__ h) {
  pc_gather_fin_body(blockIdx.x, nn, ncmax, SigT, ncls, gc, Mat, h);
}

enum PcScatter { PC_FIRST = 0, PC_SIGMA = 1, PC_UPDATE = 2 };

// per point p = (z, o, n), with v = S[h_z](x_n + u_b(z, o)/lam_z):
//   PC_FIRST:  dst = src + L v            (x_1 = P^^-1 y)
//   PC_SIGMA:  dst = v                    (Sigma* x)
//   PC_UPDATE: dst = xin + res + L v      (x += P^^-1 res)
__device__ __forceinline__ void pc_scatter_body(int bx, int mode, int nz, int nd, int nn, const double* __restrict__ x,
                                                const double* __restrict__ lam, const double* __restrict__ ub,
                                                const double* __restrict__ h, const double* __restrict__ L,
                                                const double* src, int src_stride, const double* xin,
                                                const double* __restrict__ res, double* dst, int dst_stride) {
  const long long p = bx * (long long)blockDim.x + threadIdx.x;
  if (p >= (long long)nz * nd * nn) return;
  const int n = (int)(p % nn);
  const long long zo = p / nn;
  const int z = (int)(zo / nd);
  const double* hz = h + (size_t)z * 2 * nn;
  const double v = spline_at(x, nn, hz, hz + nn, x[n] + ub[zo] / lam[z]);
  double out;
  if (mode == PC_FIRST) out = src[p * src_stride] + L[p] * v;
  else if (mode == PC_SIGMA) out = v;
  else out = xin[p] + res[p] + L[p] * v;
  dst[p * dst_stride] = out;
}

__global__ void __launch_bounds__(256) k_pc_scatter(int mode, int nz, int nd, int nn, const double* __restrict__ x,
                                                    const double* __restrict__ lam, const double* __restrict__ ub,
                                                    const double* __restrict__ h, const double* __restrict__ L,
                                                    const double* src, int src_stride, const double* xin,
                                                    const double* __restrict__ res, double* dst, int dst_stride) {
  pc_scatter_body(blockIdx.x, mode, nz, nd, nn, x, lam, ub, h, L, src, src_stride, xin, res, dst, dst_stride);
}

// ------------------------------------------------------------------ shared launches across contexts
// block b of a grouped launch is context r's block b - off[r]
__device__ inline int pc_group_of(const int* __restrict__ off, int n) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kGatherThreads) k_pc_gather_cls_grouped(const GPcCls* __restrict__ A,
                                                                          const int* __restrict__ off, int n) {
  const int r = pc_group_of(off, n);
  const GPcCls& a = A[r];
  pc_gather_cls_body(blockIdx.x - off[r], a.nd, a.nn, a.ncmax, a.x, a.SigT, a.lam, a.w, a.mem, a.moff, a.ncls,
                     a.cub, a.src, a.stride, a.gc);
}

__global__ void __launch_bounds__(kGatherThreads) k_pc_gather_fin_grouped(const GPcFin* __restrict__ A,
                                                                          const int* __restrict__ off, int n) {
  const int r = pc_group_of(off, n);
  const GPcFin& a = A[r];
  pc_gather_fin_body(blockIdx.x - off[r], a.nn, a.ncmax, a.SigT, a.ncls, a.gc, a.Mat, a.h);
}

__global__ void __launch_bounds__(256) k_pc_scatter_grouped(const GPcScat* __restrict__ A,
                                                            const int* __restrict__ off, int n) {
  const int r = pc_group_of(off, n);
  const GPcScat& a = A[r];
  pc_scatter_body(blockIdx.x - off[r], a.mode, a.nz, a.nd, a.nn, a.x, a.lam, a.ub, a.h, a.L, a.src, a.src_stride,
                  a.xin, a.res, a.dst, a.dst_stride);
}

int launch_pc_grouped(hipStream_t s, int stage, const void* args, const int* off, int n, int blocks, size_t lds) {
  switch (stage) {
    case 0:
      hipLaunchKernelGGL(k_pc_gather_cls_grouped, dim3(blocks), dim3(kGatherThreads), lds, s,
                         static_cast<const GPcCls*>(args), off, n);
      break;
    case 1:
      hipLaunchKernelGGL(k_pc_gather_fin_grouped, dim3(blocks), dim3(kGatherThreads), lds, s,
                         static_cast<const GPcFin*>(args), off, n);
      break;
    default:
      hipLaunchKernelGGL(k_pc_scatter_grouped, dim3(blocks), dim3(256), 0, s, static_cast<const GPcScat*>(args),
                         off, n);
      break;
  }
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

int precond_ensure(trap_ctx* ctx) {
  Problem& P = ctx->pb;
  Work& K = ctx->wk;
  if (K.pc_h) return TRAP_OK;
  const long long ns = (long long)P.nz * P.nd * P.nn;
  TRAP_TRY(dalloc_t(ctx, &K.pc_x, ns));
  TRAP_TRY(dalloc_t(ctx, &K.pc_e, ns));
  TRAP_TRY(dalloc_t(ctx, &K.pc_res, ns));
  TRAP_TRY(dalloc_t(ctx, &K.pc_h, (size_t)P.nz * 2 * P.nn));
  TRAP_TRY(dalloc_t(ctx, &K.pc_gc, (size_t)P.nz * ctx->pre.pc_ncmax * P.nn));
  return TRAP_OK;
}

// Scratch vectors of one preconditioner apply: the iterate x, Sigma* x and the
// residual ([z][o][n] each), the per-height comoving vector with its spline
// second derivatives h [z][2][nn] and the class sums gc [z][ncmax][nn].
struct PcWork {
  double *x, *e, *res, *h, *gc;
};

static int pc_gather(trap_ctx* ctx, const PcWork& ws, const double* src, int stride, const double* Mat) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  hipLaunchKernelGGL(k_pc_gather_cls, dim3(P.nz * C.pc_ncmax), dim3(kGatherThreads),
                     pc_gather_lds(P.nn), ctx->stream, P.nd, P.nn, C.pc_ncmax, P.d_x,
                     P.d_SigT, P.d_lam, P.d_w, C.d_pcMem, C.d_pcMoff, C.d_pcNcls, C.d_pcCub, src, stride, ws.gc);
  TRAP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pc_gather_fin, dim3(P.nz), dim3(kGatherThreads), pc_gather_lds(P.nn),
                     ctx->stream, P.nn, C.pc_ncmax, P.d_SigT, C.d_pcNcls, ws.gc, Mat, ws.h);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

static int pc_scatter(trap_ctx* ctx, const PcWork& ws, int mode, const double* src, int src_stride,
                      const double* xin, const double* res, double* dst, int dst_stride) {
  Problem& P = ctx->pb;
  const long long ns = (long long)P.nz * P.nd * P.nn;
  hipLaunchKernelGGL(k_pc_scatter, dim3(ceil_div(ns, 256)), dim3(256), 0, ctx->stream, mode, P.nz, P.nd, P.nn,
                     P.d_x, P.d_lam, P.d_ub, ws.h, ctx->pre.d_pcL, src, src_stride, xin, res, dst, dst_stride);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

static int precond_check(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec) {
  if (!ctx->has_problem || !ctx->pre.pc_done) return fail(TRAP_ESTATE, "preconditioner tables not computed");
  if (!r || !out) return fail(TRAP_EINVAL, "null vector");
  if (sweeps < 1 || sweeps > 64) return fail(TRAP_EINVAL, "preconditioner sweeps must be in [1, 64]");
  if (prec != TRAP_FP64 && prec != TRAP_FP32) return fail(TRAP_EINVAL, "unknown precision");
  return TRAP_OK;
}

// out = M r with the scratch vectors ws; every value of ws that a kernel reads
// was written earlier in the same apply, so ws needs no clearing.
static int precond_apply_ws(trap_ctx* ctx, const PcWork& ws, const double* r, double* out, int sweeps, int prec) {
  Problem& P = ctx->pb;
  Precomp& C = ctx->pre;
  const long long ns = (long long)P.nz * P.nd * P.nn;
  if (out != r) TRAP_HIP(hipMemcpyAsync(out, r, 4 * ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  // x_1 = P^^-1 y with y the Stokes I of `out` (read until the last write)
  TRAP_TRY(pc_gather(ctx, ws, out, 4, C.d_pcC));
  if (sweeps == 1) return pc_scatter(ctx, ws, PC_FIRST, out, 4, nullptr, nullptr, out, 4);
  TRAP_TRY(pc_scatter(ctx, ws, PC_FIRST, out, 4, nullptr, nullptr, ws.x, 1));
  for (int k = 2; k <= sweeps; ++k) {
    // res = y - P x = y - x + Lambda* Sigma* x
    TRAP_TRY(pc_gather(ctx, ws, ws.x, 1, C.d_pcPhi));
    TRAP_TRY(pc_scatter(ctx, ws, PC_SIGMA, nullptr, 0, nullptr, nullptr, ws.e, 1));
    TRAP_TRY(launch_formal_scalar(ctx, prec, ws.e, out, 4, ws.x, ws.res));
    // x += P^^-1 res
    TRAP_TRY(pc_gather(ctx, ws, ws.res, 1, C.d_pcC));
    const bool last = k == sweeps;
    TRAP_TRY(pc_scatter(ctx, ws, PC_UPDATE, nullptr, 0, ws.x, ws.res, last ? out : ws.x, last ? 4 : 1));
  }
  return TRAP_OK;
}

int precond_apply(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec) {
  TRAP_TRY(precond_check(ctx, r, out, sweeps, prec));
  TRAP_TRY(precond_ensure(ctx));
  Work& K = ctx->wk;
  const PcWork ws{K.pc_x, K.pc_e, K.pc_res, K.pc_h, K.pc_gc};
  return precond_apply_ws(ctx, ws, r, out, sweeps, prec);
}

// ---------------------------------------------------------------- allocation-free apply
// The same apply with its scratch vectors in a file-scope device array of
// fixed size instead of context allocations.  Every device the library runs
// on holds its own copy of the array for the life of the process; its
// address on a device is looked up once, with that device current, and kept.
// Calls on one device share the array, so calls that overlap on one device
// (on different streams, or from different host threads) race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<unsigned char*> g_scratch_dev;   // per device: device address of `scratch`

static int scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(TRAP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_dev[device];
  return TRAP_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t precond_noalloc_bytes(const Problem& P, int ncmax) {
  const size_t ns = (size_t)P.nz * P.nd * P.nn;
  return 3 * align256(ns * sizeof(double)) + align256((size_t)P.nz * 2 * P.nn * sizeof(double)) +
         align256((size_t)P.nz * ncmax * P.nn * sizeof(double));
}

int precond_apply_noalloc(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec) {
  if (ctx->has_problem) {
    const size_t need = precond_noalloc_bytes(ctx->pb, ctx->pre.pc_done ? ctx->pre.pc_ncmax : 0);
    if (need > kNoAllocScratchBytes)
      return fail(TRAP_ENOMEM, "allocation-free preconditioner apply: the problem needs " + std::to_string(need) +
                                   " bytes of scratch, above the fixed " + std::to_string(kNoAllocScratchBytes));
  }
  TRAP_TRY(precond_check(ctx, r, out, sweeps, prec));
  unsigned char* base = nullptr;
  TRAP_TRY(scratch_address(ctx->device, &base));
  const Problem& P = ctx->pb;
  const size_t ns = (size_t)P.nz * P.nd * P.nn;
  PcWork ws;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    double* p = reinterpret_cast<double*>(base + off);
    off += align256(bytes);
    return p;
  };
  ws.x = carve(ns * sizeof(double));
  ws.e = carve(ns * sizeof(double));
  ws.res = carve(ns * sizeof(double));
  ws.h = carve((size_t)P.nz * 2 * P.nn * sizeof(double));
  ws.gc = carve((size_t)P.nz * ctx->pre.pc_ncmax * P.nn * sizeof(double));
  return precond_apply_ws(ctx, ws, r, out, sweeps, prec);
}

}  // namespace trap
