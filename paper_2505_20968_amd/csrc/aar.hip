// Alternating Anderson-Richardson iteration (Sect. 5.1; the method of the AAR
// paper the text cites) for the fixed point I = G(I) = Lambda (Sigma I + eps_th) + t.
// With r = G(x) - x and f = M r (M the identity or the physics-based
// preconditioner), a step is x <- x + omega f, and every period-th step an
// Anderson step
//   x <- x + beta f - (X + beta F) gamma,   gamma = argmin || f - F gamma ||,
// X, F the last `depth` differences of x and f.  Only residuals of G are
// needed, so the iteration does not assume Lambda is linear (BESSER's is not).
// Everything is FP64 on the device; the small least-squares problem is solved
// on the host from dot products (the Gram matrix of F is kept up to date one
// new column at a time).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "trap_internal.h"

namespace trap {
namespace {

constexpr int kAarMax = 16;           // deepest history
constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;
constexpr int kVecBlocks = 1024;

struct AarPtrs {
  const double* v[kAarMax + 1];
};

struct AarUpd {
  const double* X[kAarMax];
  const double* F[kAarMax];
  double g[kAarMax];
};

// part[block][j] = sum over this block's elements of a[i] * B.v[j][i], j < nb
__global__ void __launch_bounds__(kDotThreads) k_aar_dots(long long N, const double* __restrict__ a, AarPtrs B,
                                                          int nb, double* __restrict__ part) {
  double acc[kAarMax + 1];
#pragma unroll
  for (int j = 0; j < kAarMax + 1; ++j) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)kDotThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kDotThreads) {
    const double av = a[i];
#pragma unroll
    for (int j = 0; j < kAarMax + 1; ++j)
      if (j < nb) acc[j] += av * B.v[j][i];
  }
  __shared__ double red[kDotThreads / 64][kAarMax + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kAarMax + 1; ++j) {
    if (j >= nb) break;
    double v = acc[j];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nb) {
    double s = 0.0;
    for (int w = 0; w < kDotThreads / 64; ++w) s += red[w][threadIdx.x];
    part[(size_t)blockIdx.x * (kAarMax + 1) + threadIdx.x] = s;
  }
}

// out = a - b; out may be a
__global__ void k_aar_sub(long long N, const double* a, const double* b, double* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

__global__ void k_aar_axpy(long long N, double* __restrict__ x, const double* __restrict__ f, double w) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    x[i] += w * f[i];
}

__global__ void k_aar_anderson(long long N, double* __restrict__ x, const double* __restrict__ f, double beta,
                               AarUpd U, int nh) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    double v = x[i] + beta * f[i];
#pragma unroll
    for (int j = 0; j < kAarMax; ++j)
      if (j < nh) v -= U.g[j] * (U.X[j][i] + beta * U.F[j][i]);
    x[i] = v;
  }
}

// dots of a with each of b[0..nb), summed over the blocks in a fixed order
int dots(trap_ctx* ctx, long long N, const double* a, const std::vector<const double*>& b, double* out) {
  AarPtrs B{};
  const int nb = (int)b.size();
  for (int j = 0; j < nb; ++j) B.v[j] = b[j];
  hipLaunchKernelGGL(k_aar_dots, dim3(kDotBlocks), dim3(kDotThreads), 0, ctx->stream, N, a, B, nb, ctx->wk.aar_part);
  TRAP_HIP(hipGetLastError());
  std::vector<double> h((size_t)kDotBlocks * (kAarMax + 1));
  TRAP_HIP(hipMemcpyAsync(h.data(), ctx->wk.aar_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  for (int j = 0; j < nb; ++j) {
    double s = 0.0;
    for (int k = 0; k < kDotBlocks; ++k) s += h[(size_t)k * (kAarMax + 1) + j];
    out[j] = s;
  }
  return TRAP_OK;
}

// r = G(x) - x, G(x) = Lambda (Sigma x + eps_th) + t
int fixed_point_residual(trap_ctx* ctx, long long N, const double* x, double* r) {
  void* e = ctx->wk.opeps[0];
  TRAP_TRY(sigma_apply(ctx, x, e, TRAP_FP64, 1, 1));
  TRAP_TRY(formal_apply(ctx, e, r, 1, TRAP_FP64));
  hipLaunchKernelGGL(k_aar_sub, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, r, x, r);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

// solve the nh x nh normal equations (G + lambda Id) g = h by elimination with
// partial pivoting; lambda = 1e-14 trace(G) keeps a nearly dependent history
// solvable.  Returns false if a pivot vanishes.
bool normal_solve(std::vector<double> A, std::vector<double> h, int n, std::vector<double>& g) {
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += A[i * n + i];
  for (int i = 0; i < n; ++i) A[i * n + i] += 1e-14 * tr;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (!(std::fabs(A[p * n + c]) > 0.0)) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[p * n + j]);
      std::swap(h[c], h[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      h[r] -= f * h[c];
    }
  }
  g.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double v = h[i];
    for (int j = i + 1; j < n; ++j) v -= A[i * n + j] * g[j];
    g[i] = v / A[i * n + i];
  }
  for (double v : g)
    if (!std::isfinite(v)) return false;
  return true;
}

}  // namespace

// The AAR loop on the iterate x whose residual r = res(x) is already in r:
// stops when ||r|| <= target (status TRAP_OK), after `max_evals` further
// residuals (TRAP_ENOCONV) or at a non-finite residual (TRAP_ENAN); returns
// the last ||r|| in *rnorm.  The loop's work vectors and history are the
// context's AAR block (f, previous x and f, the differences).
struct AarBufs {
  double *f, *xp, *fp;
  double* X[kAarMax];
  double* F[kAarMax];
};

template <typename Res>
int aar_loop(trap_ctx* ctx, long long N, const trap_aar_opts* o, const AarBufs& B, double* x, double* r,
             double target, int max_evals, int pc_prec, Res&& res, trap_solve_stats& S, double* rnorm, int* status) {
  const int depth = o->depth;
  double* f = o->precond_sweeps > 0 ? B.f : r;
  std::vector<double> gram((size_t)kAarMax * kAarMax, 0.0);
  std::vector<int> slots;              // history slots, oldest first
  int evals = 0;
  *status = TRAP_ENOCONV;
  for (int k = 0;; ++k) {
    double rn2 = 0.0;
    TRAP_TRY(dots(ctx, N, r, {r}, &rn2));
    *rnorm = std::sqrt(rn2);
    if (!std::isfinite(*rnorm)) {
      *status = TRAP_ENAN;
      return TRAP_OK;
    }
    if (*rnorm <= target) {
      *status = TRAP_OK;
      return TRAP_OK;
    }
    if (evals >= max_evals) return TRAP_OK;
    if (o->precond_sweeps > 0) {
      TRAP_TRY(precond_apply(ctx, r, f, o->precond_sweeps, pc_prec));
      ++S.applies_precond;
    }
    if (depth > 0) {
      if (k > 0) {
        // new differences into the oldest slot once the history is full
        int sl;
        if ((int)slots.size() < depth) {
          sl = (int)slots.size();
        } else {
          sl = slots.front();
          slots.erase(slots.begin());
        }
        slots.push_back(sl);
        hipLaunchKernelGGL(k_aar_sub, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, x, B.xp, B.X[sl]);
        hipLaunchKernelGGL(k_aar_sub, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, f, B.fp, B.F[sl]);
        TRAP_HIP(hipGetLastError());
        std::vector<const double*> b;
        for (int j : slots) b.push_back(B.F[j]);
        std::vector<double> d(slots.size());
        TRAP_TRY(dots(ctx, N, B.F[sl], b, d.data()));
        for (size_t q = 0; q < slots.size(); ++q) {
          gram[(size_t)sl * kAarMax + slots[q]] = d[q];
          gram[(size_t)slots[q] * kAarMax + sl] = d[q];
        }
      }
      TRAP_HIP(hipMemcpyAsync(B.xp, x, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      TRAP_HIP(hipMemcpyAsync(B.fp, f, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    }
    bool anderson = false;
    if (depth > 0 && (k + 1) % o->period == 0 && !slots.empty()) {
      const int nh = (int)slots.size();
      std::vector<const double*> b;
      for (int j : slots) b.push_back(B.F[j]);
      std::vector<double> h(nh), A((size_t)nh * nh), g;
      TRAP_TRY(dots(ctx, N, f, b, h.data()));
      for (int i = 0; i < nh; ++i)
        for (int j = 0; j < nh; ++j) A[(size_t)i * nh + j] = gram[(size_t)slots[i] * kAarMax + slots[j]];
      if (normal_solve(A, h, nh, g)) {
        AarUpd U{};
        for (int i = 0; i < nh; ++i) {
          U.X[i] = B.X[slots[i]];
          U.F[i] = B.F[slots[i]];
          U.g[i] = g[i];
        }
        hipLaunchKernelGGL(k_aar_anderson, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, x, f, o->beta, U, nh);
        TRAP_HIP(hipGetLastError());
        anderson = true;
        ++S.outer_steps;
      }
    }
    if (!anderson) {
      hipLaunchKernelGGL(k_aar_axpy, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, x, f, o->omega);
      TRAP_HIP(hipGetLastError());
    }
    TRAP_TRY(res(x, r));
    ++evals;
    ++S.inner_iters;
  }
}

__global__ void k_aar_to_f32(long long N, const double* __restrict__ x, float* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// r = r0 - y (y FP32)
__global__ void k_aar_defect(long long N, const double* __restrict__ r0, const float* __restrict__ y,
                             double* __restrict__ r) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    r[i] = r0[i] - (double)y[i];
}

int aar_solve(trap_ctx* ctx, const trap_aar_opts* o, double* x, trap_solve_stats* st) {
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (!o || !x) return fail(TRAP_EINVAL, "null argument");
  if (!(o->tol > 0) || o->max_iters < 0 || o->depth < 0 || o->depth > kAarMax || o->period < 1 ||
      !(o->omega > 0) || !(o->beta > 0))
    return fail(TRAP_EINVAL, "bad AAR options (depth in [0, 16], period >= 1, omega, beta > 0)");
  if (o->inner != TRAP_FP64 && o->inner != TRAP_FP32) return fail(TRAP_EINVAL, "bad inner precision");
  const bool mixed = o->inner == TRAP_FP32;
  if (mixed && (!(o->inner_tol > 0 && o->inner_tol < 1) || o->max_outer < 1))
    return fail(TRAP_EINVAL, "bad refinement options (0 < inner_tol < 1, max_outer >= 1)");
  if (mixed && !ctx->pre.d_cf32) return fail(TRAP_ESTATE, "FP32 kernels not stored");
  if (o->precond_sweeps < 0 || o->precond_sweeps > 64)
    return fail(TRAP_EINVAL, "preconditioner sweeps must be in [0, 64]");
  if (o->precond_sweeps > 0 && !ctx->pre.pc_done) return fail(TRAP_ESTATE, "preconditioner tables not computed");
  const auto t0 = std::chrono::steady_clock::now();
  const Problem& P = ctx->pb;
  const long long N = 4LL * P.nz * P.nd * P.nn;
  Work& K = ctx->wk;
  TRAP_TRY(ensure_work(ctx, TRAP_FP64));
  if (mixed) TRAP_TRY(ensure_work(ctx, TRAP_FP32));
  if (o->precond_sweeps > 0) TRAP_TRY(precond_ensure(ctx));
  if (!K.aar_part) TRAP_TRY(dalloc_t(ctx, &K.aar_part, (size_t)kDotBlocks * (kAarMax + 1)));
  // r, f, previous x and f, correction d, outer residual, FP32 pair, FP32
  // reference emissivity, differences
  constexpr int kFixed = 8;
  if (K.aar_cap < o->depth) {
    TRAP_TRY(dalloc_t(ctx, &K.aar, (size_t)(kFixed + 2 * o->depth) * N));
    K.aar_cap = o->depth;
  }
  const int cap = K.aar_cap;
  AarBufs B{};
  double* r = K.aar;
  B.f = K.aar + N;
  B.xp = K.aar + 2 * N;
  B.fp = K.aar + 3 * N;
  double* d = K.aar + 4 * N;
  double* r64 = K.aar + 5 * N;
  float* v32 = reinterpret_cast<float*>(K.aar + 6 * N);     // two FP32 vectors in one FP64 slot
  float* y32 = v32 + N;
  float* eref32 = reinterpret_cast<float*>(K.aar + 7 * N);
  for (int j = 0; j < cap; ++j) {
    B.X[j] = K.aar + (size_t)(kFixed + j) * N;
    B.F[j] = K.aar + (size_t)(kFixed + cap + j) * N;
  }

  trap_solve_stats S{};
  double bn2 = 0.0;
  TRAP_TRY(dots(ctx, N, ctx->pre.d_b, {ctx->pre.d_b}, &bn2));
  const double bn = std::sqrt(bn2);
  if (!(bn > 0.0) || !std::isfinite(bn)) return fail(TRAP_EINVAL, "zero or non-finite right-hand side");
  double* r_out = mixed ? r64 : r;     // the FP64 residual G(x) - x
  // the emissivity Sigma x + eps_th of the current iterate
  const double* e_cur = static_cast<const double*>(ctx->wk.opeps[0]);
  if (o->zero_guess) {
    // G(0) is the right-hand side Lambda eps_th + t
    TRAP_HIP(hipMemsetAsync(x, 0, N * sizeof(double), ctx->stream));
    TRAP_HIP(hipMemcpyAsync(r_out, ctx->pre.d_b, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    e_cur = ctx->pre.d_epsth;
  } else {
    TRAP_TRY(fixed_point_residual(ctx, N, x, r_out));
    ++S.applies_fp64;
  }
  int status = TRAP_ENOCONV;
  double rn = 0.0;
  if (!mixed) {
    auto res = [&](const double* xx, double* rr) -> int {
      ++S.applies_fp64;
      return fixed_point_residual(ctx, N, xx, rr);
    };
    TRAP_TRY(aar_loop(ctx, N, o, B, x, r, o->tol * bn, o->max_iters, TRAP_FP64, res, S, &rn, &status));
    S.final_rel_res = rn / bn;
  } else {
    // defect correction: the FP64 residual r64 = G(x) - x, then the
    // correction d with d = r64 + Lambda Sigma d in the FP32 operator
    // (inner residual r64 - (d - Lambda Sigma d)), x += d, until ||r64|| meets tol.
    // With BESSER the inner Lambda is the Jacobian of the BESSER map at x: its
    // branches follow the source of x (the reference emissivity).
    const bool besser = ctx->formal_scheme == TRAP_FORMAL_BESSER;
    struct RefGuard {
      trap_ctx* c;
      ~RefGuard() {
        c->besser_ref = nullptr;
        c->besser_ref_prec = -1;
      }
    } guard{ctx};
    auto res = [&](const double* dd, double* rr) -> int {
      hipLaunchKernelGGL(k_aar_to_f32, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, dd, v32);
      TRAP_HIP(hipGetLastError());
      // the inner operator is linear: spline frame transforms
      ctx->interp_lin = 1;
      const int rc = operator_apply(ctx, v32, y32, TRAP_FP32);
      ctx->interp_lin = 0;
      TRAP_TRY(rc);
      hipLaunchKernelGGL(k_aar_defect, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, r64, y32, rr);
      TRAP_HIP(hipGetLastError());
      ++S.applies_fp32;
      return TRAP_OK;
    };
    for (int outer = 0;; ++outer) {
      double r2 = 0.0;
      TRAP_TRY(dots(ctx, N, r64, {r64}, &r2));
      S.final_rel_res = std::sqrt(r2) / bn;
      if (!std::isfinite(S.final_rel_res)) {
        status = TRAP_ENAN;
        break;
      }
      if (S.final_rel_res < o->tol) {
        status = TRAP_OK;
        break;
      }
      if (outer >= o->max_outer || S.inner_iters >= o->max_iters) break;
      TRAP_HIP(hipMemsetAsync(d, 0, N * sizeof(double), ctx->stream));
      TRAP_HIP(hipMemcpyAsync(r, r64, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      if (besser) {
        hipLaunchKernelGGL(k_aar_to_f32, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, e_cur, eref32);
        TRAP_HIP(hipGetLastError());
        ctx->besser_ref = eref32;
        ctx->besser_ref_prec = TRAP_FP32;
      }
      int st_in = TRAP_ENOCONV;
      // no tighter than the final tolerance needs: half of it leaves room for
      // the FP32 error of the correction
      const double target = std::max(o->inner_tol * std::sqrt(r2), 0.5 * o->tol * bn);
      TRAP_TRY(aar_loop(ctx, N, o, B, d, r, target, o->max_iters - S.inner_iters, TRAP_FP32, res, S, &rn, &st_in));
      ctx->besser_ref = nullptr;
      ctx->besser_ref_prec = -1;
      if (st_in == TRAP_ENAN) {
        status = TRAP_ENAN;
        break;
      }
      hipLaunchKernelGGL(k_aar_axpy, dim3(kVecBlocks), dim3(256), 0, ctx->stream, N, x, d, 1.0);
      TRAP_HIP(hipGetLastError());
      TRAP_TRY(fixed_point_residual(ctx, N, x, r64));
      e_cur = static_cast<const double*>(ctx->wk.opeps[0]);
      ++S.applies_fp64;
    }
  }
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = S;
  if (status == TRAP_ENOCONV) return fail(TRAP_ENOCONV, "AAR did not reach the tolerance");
  if (status == TRAP_ENAN) return fail(TRAP_ENAN, "non-finite residual");
  return TRAP_OK;
}

}  // namespace trap

int trap_aar_solve(trap_ctx* ctx, const trap_aar_opts* opts, double* I, trap_solve_stats* stats) {
  if (!ctx) return trap::fail(TRAP_EINVAL, "null context");
  trap::DeviceGuard g(ctx->device, __func__);
  return trap::aar_solve(ctx, opts, I, stats);
}
