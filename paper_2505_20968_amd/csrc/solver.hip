// Matrix-free restarted GMRES for (Id - Lambda Sigma) I = b (paper Sect. 5.1)
// with the stopping rule ||b - A I||_2 / ||b||_2 < tol.
//
// The Krylov basis, residuals and iterates live on the device in FP64; the
// Hessenberg matrix and Givens rotations (a few dozen scalars) are kept on the
// host.  Orthogonalisation is classical Gram-Schmidt applied twice (CGS2),
// which needs two block dot-products and two block updates per step.
//
// Mixed precision: with an FP32 inner operator the solve is an iterative
// refinement: r = b - A64 x (FP64 operator), d ~ A32^-1 r by GMRES with the
// FP32 operator (FP64 Arnoldi), x += d, until the FP64 residual meets tol.
#include <chrono>
#include <cmath>
#include <vector>

#include "trap_internal.h"

namespace trap {

// partial[b * ncols + k] = sum over block b of V_k . w
// partial[block][k] = sum over this block's share of i of V[k][i] w[i]; columns
// are taken eight at a time so w is read once per eight basis vectors.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Vectors have N = 4 n_z n_dir n_nu entries (a multiple of four), so every
// column of the basis is 16-byte aligned and is streamed as double2.
__global__ void __launch_bounds__(256) k_multidot(const double* __restrict__ V, int ncols, long long N,
                                                  const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[4][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long N2 = N >> 1;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (int k0 = 0; k0 < ncols; k0 += 8) {
    const int kc = min(8, ncols - k0);
    const double2* V2 = reinterpret_cast<const double2*>(V + (size_t)k0 * N);
    double s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N2;
         i += (long long)gridDim.x * blockDim.x) {
      const double2 wi = w2[i];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < kc) {
          const double2 v = V2[(size_t)q * N2 + i];
          s[q] += v.x * wi.x + v.y * wi.y;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double t = wave_sum(s[q]);
      if (lane == 0) sh[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < kc)
      partial[(size_t)blockIdx.x * ncols + k0 + threadIdx.x] =
          sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
    __syncthreads();
  }
}

// out[k] = sum over blocks of partial[b][k]; one block per column.
__global__ void __launch_bounds__(256) k_reduce_partial(const double* __restrict__ partial, int nblocks,
                                                        int ncols, double* __restrict__ out) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * ncols + k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[k] = sh[0] + sh[1] + sh[2] + sh[3];
}
// w -= sum_k h[k] V_k, four columns per step
__global__ void __launch_bounds__(256) k_multiaxpy(const double* __restrict__ V, int ncols, long long N,
                                                   const double* __restrict__ h, double* __restrict__ w) {
  const long long N2 = N >> 1;
  const double2* V2 = reinterpret_cast<const double2*>(V);
  double2* w2 = reinterpret_cast<double2*>(w);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N2;
       i += (long long)gridDim.x * blockDim.x) {
    double2 s = w2[i];
    int k = 0;
    for (; k + 4 <= ncols; k += 4) {
      const double2 a0 = V2[(size_t)k * N2 + i], a1 = V2[(size_t)(k + 1) * N2 + i];
      const double2 a2 = V2[(size_t)(k + 2) * N2 + i], a3 = V2[(size_t)(k + 3) * N2 + i];
      s.x -= h[k] * a0.x;
      s.y -= h[k] * a0.y;
      s.x -= h[k + 1] * a1.x;
      s.y -= h[k + 1] * a1.y;
      s.x -= h[k + 2] * a2.x;
      s.y -= h[k + 2] * a2.y;
      s.x -= h[k + 3] * a3.x;
      s.y -= h[k + 3] * a3.y;
    }
    for (; k < ncols; ++k) {
      const double2 a = V2[(size_t)k * N2 + i];
      s.x -= h[k] * a.x;
      s.y -= h[k] * a.y;
    }
    w2[i] = s;
  }
}

__global__ void k_scale_copy(long long N, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ void k_axpby(long long N, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void k_to_f32(long long N, double scale, const double* __restrict__ x, float* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (float)(scale * x[i]);
}

__global__ void k_from_f32(long long N, double scale, const float* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = scale * (double)x[i];
}

// flag bit 0: a non-finite entry; bit 1 (when asked): a nonzero entry
__global__ void k_nonfinite(long long N, const double* __restrict__ x, int* __restrict__ flag, int want_zero) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    if (!isfinite(x[i])) atomicOr(flag, 1);
    if (want_zero && x[i] != 0.0) atomicOr(flag, 2);
  }
}

namespace {

constexpr int kBlocks = 1024;

// y = A x with the operator in precision `prec` (x, y FP64); `lin`: an inner
// Krylov apply, whose frame transforms are the spline (a linear operator)
// whatever interpolant the context uses for its residuals
int op_apply(trap_ctx* ctx, int prec, const double* x, double* y, trap_solve_stats* st, bool lin) {
  Work& K = ctx->wk;
  const long long N = 4LL * ctx->pb.nz * ctx->pb.nd * ctx->pb.nn;
  struct LinGuard {
    trap_ctx* c;
    ~LinGuard() { c->interp_lin = 0; }
  } guard{ctx};
  ctx->interp_lin = lin ? 1 : 0;
  if (prec == TRAP_FP64) {
    TRAP_TRY(operator_apply(ctx, x, y, TRAP_FP64));
    st->applies_fp64++;
    return TRAP_OK;
  }
  hipLaunchKernelGGL(k_to_f32, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0, x, K.v32a);
  TRAP_HIP(hipGetLastError());
  TRAP_TRY(operator_apply(ctx, K.v32a, K.v32b, TRAP_FP32));
  hipLaunchKernelGGL(k_from_f32, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0, K.v32b, y);
  TRAP_HIP(hipGetLastError());
  st->applies_fp32++;
  return TRAP_OK;
}

}  // namespace

// ---------------------------------------------------------------- GMRES state machine
// One run of the (mixed-precision) restarted GMRES of a context, advanced in
// units that end at a host synchronisation point, so that many contexts can be
// advanced together with one wait per phase (trap_gmres_step_batch):
//   RESID_OUTER    r = b - A64 x and its norm             (one sync)
//   RESID_RESTART  r_k = r - A_p d and its norm           (one sync)
//   ARNOLDI        w = A_p v_j; [h, |w|^2] = [V, w]^T w    (sync 1)
//                  w -= V h; if the projection removed more than half of
//                  |w|^2, a second pass: h2 = [V, w]^T w    (sync 2)
//                  and w -= V h2; |w| and the Givens update (no sync)
// Classical Gram-Schmidt with the reorthogonalisation pass taken only when
// ||w - V h|| < ||w|| / sqrt(2) (the Daniel-Gragg-Kaufman-Stewart test).  The
// norm after a projection follows from ||w - V h||^2 = ||w||^2 - ||h||^2 (V
// orthonormal); when that difference is small it is measured directly.
enum GmresPhase { GP_RESID_OUTER = 0, GP_RESID_RESTART = 1, GP_ARNOLDI = 2, GP_DONE = 3 };

struct GmresRun {
  trap_solve_opts opts{};
  trap_solve_stats st{};
  double* x = nullptr;
  long long N = 0;
  int m = 0, prec = TRAP_FP64, phase = GP_DONE, status = TRAP_OK;
  int outer = 0, j = 0, max_outer = 1;
  int pc = 0;                 // preconditioner sweeps (0: none)
  bool p2 = false;            // an Arnoldi step waits for its second reduction
  bool begin_pending = false; // ||b|| and the initial-guess check are read at the first step
  double bnorm = 0, beta = 0, target = 0, res = 0, rel = 0;
  std::vector<double> H, cs, sn, g, h;
  double* hbuf = nullptr;     // pinned host copy of the reductions, 2 (m + 2)
  double* partial = nullptr;  // device reduction scratch
  double* dres = nullptr;
  std::chrono::steady_clock::time_point t0;
};

namespace {

int dots_async(trap_ctx* ctx, GmresRun& R, const double* V, int ncols, const double* w, double* host_out) {
  hipLaunchKernelGGL(k_multidot, dim3(kBlocks), dim3(256), 0, ctx->stream, V, ncols, R.N, w, R.partial);
  TRAP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_partial, dim3(ncols), dim3(256), 0, ctx->stream, R.partial, kBlocks, ncols,
                     R.dres);
  TRAP_HIP(hipGetLastError());
  TRAP_HIP(hipMemcpyAsync(host_out, R.dres, ncols * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  return TRAP_OK;
}

// w -= sum_k coef[k] V_k (coefficients from the host; copied through the
// second half of the pinned buffer so the copy is ordered on the stream)
int axpy_async(trap_ctx* ctx, GmresRun& R, const double* V, int ncols, const double* coef, double* w,
               double* dcoef) {
  TRAP_HIP(hipMemcpyAsync(dcoef, coef, ncols * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_multiaxpy, dim3(kBlocks), dim3(256), 0, ctx->stream, V, ncols, R.N, dcoef, w);
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

}  // namespace

// pinned host buffer layout (4 (m + 2) doubles): [0, m + 2) first reduction,
// [m + 2, 2 (m + 2)) second reduction, then the initial-guess flag, the
// update coefficients, and ||b||^2 in the last slot
static int* begin_flag(GmresRun& R) { return reinterpret_cast<int*>(R.hbuf + 2 * (R.m + 2)); }
static double* begin_bnorm2(GmresRun& R) { return R.hbuf + 4 * (R.m + 2) - 1; }

__global__ void k_fill_int(int* p, int v) {
  if (threadIdx.x == 0) p[0] = v;
}

static void run_finish(GmresRun& R, int status) {
  R.phase = GP_DONE;
  R.status = status;
  R.st.final_rel_res = R.rel;
  R.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - R.t0).count();
}

int gmres_begin(trap_ctx* ctx, const trap_solve_opts* opts, double* I) {
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (!opts || !I) return fail(TRAP_EINVAL, "null argument");
  if (!(opts->tol > 0) || opts->restart < 1 || opts->max_iters < 0)
    return fail(TRAP_EINVAL, "bad solver options");
  if (ctx->formal_scheme == TRAP_FORMAL_BESSER)
    return fail(TRAP_EINVAL, "BESSER makes Lambda nonlinear: solve with trap_aar_solve");
  const int inner = opts->inner;
  if (inner != TRAP_FP64 && inner != TRAP_FP32) return fail(TRAP_EINVAL, "bad inner precision");
  if (inner == TRAP_FP32 && !ctx->pre.d_cf32) return fail(TRAP_ESTATE, "FP32 kernels not stored");
  if (opts->precond_sweeps < 0 || opts->precond_sweeps > 64)
    return fail(TRAP_EINVAL, "preconditioner sweeps must be in [0, 64]");
  if (opts->precond_sweeps > 0 && !ctx->pre.pc_done)
    return fail(TRAP_ESTATE, "preconditioner tables not computed");
  Work& K = ctx->wk;
  const long long N = 4LL * ctx->pb.nz * ctx->pb.nd * ctx->pb.nn;
  TRAP_TRY(ensure_work(ctx, TRAP_FP64));
  if (inner == TRAP_FP32) TRAP_TRY(ensure_work(ctx, TRAP_FP32));
  const int m = opts->restart;
  if (K.V_cols < m + 1) {
    TRAP_TRY(dalloc_t(ctx, &K.V, (size_t)(m + 1) * N));
    TRAP_TRY(dalloc_t(ctx, &K.dots, (size_t)kBlocks * (m + 2) + 2 * (m + 2)));
    K.V_cols = m + 1;
  }
  if (inner == TRAP_FP32 && !K.v32a) {
    TRAP_TRY(dalloc_t(ctx, &K.v32a, N));
    TRAP_TRY(dalloc_t(ctx, &K.v32b, N));
  }
  if (!ctx->run) ctx->run = new (std::nothrow) GmresRun();
  if (!ctx->run) return fail(TRAP_ENOMEM, "host allocation failed");
  GmresRun& R = *ctx->run;
  if (R.hbuf && R.m < m) {
    TRAP_NOTE(hipHostFree(R.hbuf));
    R.hbuf = nullptr;
  }
  if (!R.hbuf) TRAP_HIP(hipHostMalloc(reinterpret_cast<void**>(&R.hbuf), 4 * (m + 2) * sizeof(double)));
  R.opts = *opts;
  R.st = trap_solve_stats{};
  R.x = I;
  R.N = N;
  R.m = m;
  R.prec = inner;
  R.outer = 0;
  R.p2 = false;
  R.pc = opts->precond_sweeps;
  // the preconditioned inner solves stop on the preconditioned residual, so
  // the true residual is refined in an outer loop in either precision
  R.max_outer = (inner == TRAP_FP64 && R.pc == 0) ? 1 : std::max(1, opts->max_outer);
  R.H.assign((size_t)(m + 1) * m, 0.0);
  R.cs.assign(m, 0.0);
  R.sn.assign(m, 0.0);
  R.g.assign(m + 1, 0.0);
  R.h.assign(m + 2, 0.0);
  R.partial = K.dots;
  R.dres = K.dots + (size_t)kBlocks * (m + 2);
  R.t0 = std::chrono::steady_clock::now();
  // the initial guess must be finite, and ||b||: enqueued here, read by the
  // first step after its synchronisation (so beginning a solve never waits)
  int* dflag = reinterpret_cast<int*>(K.red);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, dflag, 0);
  hipLaunchKernelGGL(k_nonfinite, dim3(kBlocks), dim3(256), 0, ctx->stream, N, I, dflag, opts->zero_guess ? 1 : 0);
  TRAP_HIP(hipGetLastError());
  int* hflag = begin_flag(R);
  *hflag = 0;
  TRAP_HIP(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TRAP_TRY(dots_async(ctx, R, ctx->pre.d_b, 1, ctx->pre.d_b, begin_bnorm2(R)));
  R.begin_pending = true;
  R.phase = GP_RESID_OUTER;
  R.status = 1;
  return TRAP_OK;
}

// the deferred checks of gmres_begin; false when they ended the run
static bool begin_checks(GmresRun& R) {
  if (!R.begin_pending) return true;
  R.begin_pending = false;
  if (*begin_flag(R) & 1) {
    run_finish(R, fail(TRAP_ENAN, "non-finite initial guess"));
    return false;
  }
  if (*begin_flag(R) & 2) {
    run_finish(R, fail(TRAP_EINVAL, "initial guess declared zero is not zero"));
    return false;
  }
  R.bnorm = std::sqrt(std::max(*begin_bnorm2(R), 0.0));
  if (!(R.bnorm > 0)) {
    run_finish(R, fail(TRAP_EINVAL, "zero right-hand side"));
    return false;
  }
  return true;
}

namespace {

// the operator apply that opens a unit: y = A_prec x (false when none)
bool unit_operand(trap_ctx* ctx, GmresRun& R, int* prec, const double** x, double** y) {
  Work& K = ctx->wk;
  switch (R.phase) {
    case GP_RESID_OUTER:
      *prec = TRAP_FP64;
      *x = R.x;
      *y = K.r;
      return true;
    case GP_RESID_RESTART:
      *prec = R.prec;
      *x = K.x;
      *y = K.tmp64;
      return true;
    case GP_ARNOLDI:
      *prec = R.prec;
      *x = K.V + (size_t)R.j * R.N;
      *y = K.V + (size_t)(R.j + 1) * R.N;
      return true;
    default:
      return false;
  }
}

// phase-1 work of one unit after its operator apply, up to the first
// synchronisation (pc_done: the Arnoldi vector was preconditioned in the
// shared apply already)
int unit_issue1_rest(trap_ctx* ctx, GmresRun& R, bool pc_done = false) {
  Work& K = ctx->wk;
  const long long N = R.N;
  switch (R.phase) {
    case GP_RESID_OUTER:
      hipLaunchKernelGGL(k_axpby, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0, ctx->pre.d_b, -1.0, K.r);
      TRAP_HIP(hipGetLastError());
      if (R.pc) {
        // M r into tmp64; ||r||^2 and ||M r||^2 in the first two slots
        TRAP_TRY(precond_apply(ctx, K.r, K.tmp64, R.pc, R.prec));
        R.st.applies_precond++;
        TRAP_TRY(dots_async(ctx, R, K.r, 1, K.r, R.hbuf));
        return dots_async(ctx, R, K.tmp64, 1, K.tmp64, R.hbuf + 1);
      }
      return dots_async(ctx, R, K.r, 1, K.r, R.hbuf);
    case GP_RESID_RESTART:
      hipLaunchKernelGGL(k_axpby, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0, K.r, -1.0, K.tmp64);
      TRAP_HIP(hipGetLastError());
      if (R.pc) {
        TRAP_TRY(precond_apply(ctx, K.tmp64, K.tmp64, R.pc, R.prec));
        R.st.applies_precond++;
      }
      return dots_async(ctx, R, K.tmp64, 1, K.tmp64, R.hbuf);
    case GP_ARNOLDI:
      if (R.pc && !pc_done) {
        double* w = K.V + (size_t)(R.j + 1) * N;
        TRAP_TRY(precond_apply(ctx, w, w, R.pc, R.prec));
        R.st.applies_precond++;
      }
      return dots_async(ctx, R, K.V, R.j + 2, K.V + (size_t)(R.j + 1) * N, R.hbuf);   // last entry: |w|^2
    default:
      return TRAP_OK;
  }
}

// phase-1 work of one unit (everything up to its first synchronisation)
int unit_issue1(trap_ctx* ctx, GmresRun& R) {
  int prec;
  const double* x;
  double* y;
  if (!unit_operand(ctx, R, &prec, &x, &y)) return TRAP_OK;
  if (R.phase == GP_RESID_OUTER && R.outer == 0 && R.opts.zero_guess) {
    // A 0 = 0: the first residual is b itself
    hipLaunchKernelGGL(k_scale_copy, dim3(kBlocks), dim3(256), 0, ctx->stream, R.N, 0.0, ctx->pre.d_b, y);
    TRAP_HIP(hipGetLastError());
  } else {
    TRAP_TRY(op_apply(ctx, prec, x, y, &R.st, R.phase != GP_RESID_OUTER));
  }
  return unit_issue1_rest(ctx, R);
}

// start an Arnoldi cycle from the (unnormalised) residual vector src of norm beta
int start_cycle(trap_ctx* ctx, GmresRun& R, const double* src, double beta) {
  R.beta = beta;
  std::fill(R.g.begin(), R.g.end(), 0.0);
  std::fill(R.H.begin(), R.H.end(), 0.0);
  R.g[0] = beta;
  R.j = 0;
  hipLaunchKernelGGL(k_scale_copy, dim3(kBlocks), dim3(256), 0, ctx->stream, R.N, 1.0 / beta, src, ctx->wk.V);
  TRAP_HIP(hipGetLastError());
  R.phase = GP_ARNOLDI;
  return TRAP_OK;
}

// end of an Arnoldi cycle: d += V y with H y = g; then either restart or refine
int end_cycle(trap_ctx* ctx, GmresRun& R, bool converged) {
  Work& K = ctx->wk;
  const int m = R.m, j = R.j;
  std::vector<double> y(j, 0.0);
  for (int i = j - 1; i >= 0; --i) {
    double v = R.g[i];
    for (int k = i + 1; k < j; ++k) v -= R.H[(size_t)i * m + k] * y[k];
    y[i] = v / R.H[(size_t)i * m + i];
  }
  for (int i = 0; i < j; ++i) y[i] = -y[i];
  double* hc = R.hbuf + 2 * (m + 2) + 2;   // staging of the coefficients, past the flag
  std::copy(y.begin(), y.end(), hc);
  TRAP_TRY(axpy_async(ctx, R, K.V, j, hc, K.x, R.dres));    // d -= (-y) V
  const bool out_of_iters = R.st.inner_iters >= R.opts.max_iters;
  if (converged || out_of_iters) {
    hipLaunchKernelGGL(k_axpby, dim3(kBlocks), dim3(256), 0, ctx->stream, R.N, 1.0, K.x, 1.0, R.x);
    TRAP_HIP(hipGetLastError());
    R.phase = GP_RESID_OUTER;
  } else {
    R.phase = GP_RESID_RESTART;
  }
  return TRAP_OK;
}

int arnoldi_finish(trap_ctx* ctx, GmresRun& R, double hn);

// host work after sync 1; issues phase-2 work of Arnoldi units
int unit_after1(trap_ctx* ctx, GmresRun& R) {
  Work& K = ctx->wk;
  const long long N = R.N;
  if (!begin_checks(R)) return TRAP_OK;
  switch (R.phase) {
    case GP_RESID_OUTER: {
      const double rn = std::sqrt(std::max(R.hbuf[0], 0.0));
      R.rel = rn / R.bnorm;
      if (!std::isfinite(R.rel)) {
        run_finish(R, fail(TRAP_ENAN, "non-finite residual"));
        return TRAP_OK;
      }
      if (R.rel < R.opts.tol) {
        run_finish(R, TRAP_OK);
        return TRAP_OK;
      }
      if (R.outer >= R.max_outer || R.st.inner_iters >= R.opts.max_iters) {
        run_finish(R, fail(TRAP_ENOCONV, "tolerance not reached"));
        return TRAP_OK;
      }
      R.outer++;
      R.st.outer_steps = R.outer;
      TRAP_HIP(hipMemsetAsync(K.x, 0, N * sizeof(double), ctx->stream));
      if (R.pc) {
        // the inner solve sees the preconditioned residual M r; its goal
        // scales with ||M r|| / ||r||
        const double pn = std::sqrt(std::max(R.hbuf[1], 0.0));
        if (!std::isfinite(pn) || !(pn > 0.0)) {
          run_finish(R, fail(TRAP_ENAN, "non-finite or zero preconditioned residual"));
          return TRAP_OK;
        }
        // (an FP64 inner operator has no precision floor: it aims at tol at once)
        const double goal = 0.5 * R.opts.tol * R.bnorm * (pn / rn);
        R.target = R.prec == TRAP_FP64 ? goal : std::max(R.opts.inner_tol * pn, goal);
        return start_cycle(ctx, R, K.tmp64, pn);
      }
      R.target = R.prec == TRAP_FP64 ? 0.999 * R.opts.tol * R.bnorm
                                     : std::max(R.opts.inner_tol * rn, 0.5 * R.opts.tol * R.bnorm);
      return start_cycle(ctx, R, K.r, rn);
    }
    case GP_RESID_RESTART: {
      const double beta = std::sqrt(std::max(R.hbuf[0], 0.0));
      if (beta <= R.target) {
        hipLaunchKernelGGL(k_axpby, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0, K.x, 1.0, R.x);
        TRAP_HIP(hipGetLastError());
        R.phase = GP_RESID_OUTER;
        return TRAP_OK;
      }
      return start_cycle(ctx, R, K.tmp64, beta);
    }
    case GP_ARNOLDI: {
      const int j = R.j;
      double* w = K.V + (size_t)(j + 1) * N;
      double s1 = 0.0;
      for (int i = 0; i <= j; ++i) {
        R.h[i] = R.hbuf[i];
        s1 += R.hbuf[i] * R.hbuf[i];
      }
      const double wn2 = R.hbuf[j + 1];
      TRAP_TRY(axpy_async(ctx, R, K.V, j + 1, R.hbuf, w, R.dres + (R.m + 2)));
      if (wn2 - s1 > 0.5 * wn2) return arnoldi_finish(ctx, R, std::sqrt(wn2 - s1));
      // second projection and ||w||^2 in one reduction (w is basis column j + 1)
      R.p2 = true;
      return dots_async(ctx, R, K.V, j + 2, w, R.hbuf + (R.m + 2));
    }
    default:
      return TRAP_OK;
  }
}

// host work after sync 2 (Arnoldi units only)
int unit_after2(trap_ctx* ctx, GmresRun& R) {
  if (R.phase != GP_ARNOLDI || !R.p2) return TRAP_OK;
  R.p2 = false;
  Work& K = ctx->wk;
  const long long N = R.N;
  const int j = R.j, m = R.m;
  double* w = K.V + (size_t)(j + 1) * N;
  const double* h2 = R.hbuf + (m + 2);
  double s2 = 0.0;
  for (int i = 0; i <= j; ++i) s2 += h2[i] * h2[i];
  const double wn2 = h2[j + 1];
  for (int i = 0; i <= j; ++i) R.h[i] += h2[i];
  TRAP_TRY(axpy_async(ctx, R, K.V, j + 1, h2, w, R.dres));
  double hn2 = wn2 - s2;
  if (!(hn2 > 1e-6 * wn2)) {
    // cancellation: measure the norm directly
    TRAP_TRY(dots_async(ctx, R, w, 1, w, R.hbuf));
    TRAP_HIP(hipStreamSynchronize(ctx->stream));
    hn2 = R.hbuf[0];
  }
  return arnoldi_finish(ctx, R, std::sqrt(std::max(hn2, 0.0)));
}

// |w| known: normalise w, append the Hessenberg column, rotate, test
int arnoldi_finish(trap_ctx* ctx, GmresRun& R, double hn) {
  Work& K = ctx->wk;
  const long long N = R.N;
  const int j = R.j, m = R.m;
  double* w = K.V + (size_t)(j + 1) * N;
  if (!std::isfinite(hn)) {
    run_finish(R, fail(TRAP_ENAN, "non-finite Arnoldi vector"));
    return TRAP_OK;
  }
  for (int i = 0; i <= j; ++i) R.H[(size_t)i * m + j] = R.h[i];
  R.H[(size_t)(j + 1) * m + j] = hn;
  if (hn > 0.0) {
    hipLaunchKernelGGL(k_scale_copy, dim3(kBlocks), dim3(256), 0, ctx->stream, N, 1.0 / hn, w, w);
    TRAP_HIP(hipGetLastError());
  }
  for (int i = 0; i < j; ++i) {
    const double a = R.H[(size_t)i * m + j], b = R.H[(size_t)(i + 1) * m + j];
    R.H[(size_t)i * m + j] = R.cs[i] * a + R.sn[i] * b;
    R.H[(size_t)(i + 1) * m + j] = -R.sn[i] * a + R.cs[i] * b;
  }
  const double a = R.H[(size_t)j * m + j], b = R.H[(size_t)(j + 1) * m + j];
  const double den = std::hypot(a, b);
  R.cs[j] = den > 0 ? a / den : 1.0;
  R.sn[j] = den > 0 ? b / den : 0.0;
  R.H[(size_t)j * m + j] = den;
  R.H[(size_t)(j + 1) * m + j] = 0.0;
  R.g[j + 1] = -R.sn[j] * R.g[j];
  R.g[j] = R.cs[j] * R.g[j];
  R.res = std::fabs(R.g[j + 1]);
  R.j = j + 1;
  R.st.inner_iters++;
  const bool conv = R.res <= R.target || hn == 0.0;
  if (conv || R.j == m || R.st.inner_iters >= R.opts.max_iters) return end_cycle(ctx, R, conv);
  return TRAP_OK;
}

}  // namespace

int gmres_step_batch(trap_ctx** ctxs, int n, int* status) {
  // phase 1: the FP32 operator applies of contexts on one device go through
  // shared launches; every other unit is issued on its own
  std::vector<int> grp;
  std::vector<trap_ctx*> gctx;
  std::vector<const double*> gx;
  std::vector<double*> gy;
  int gdev = -1;
  for (int i = 0; i < n; ++i) {
    GmresRun& R = *ctxs[i]->run;
    if (R.phase == GP_DONE) continue;
    DeviceGuard g(ctxs[i]->device, __func__);
    int prec;
    const double* x;
    double* y;
    if (unit_operand(ctxs[i], R, &prec, &x, &y) && prec == TRAP_FP32 &&
        (gdev < 0 || gdev == ctxs[i]->device)) {
      const int ok = sigma_batch_ready(ctxs[i]);
      if (ok < 0) {
        run_finish(R, ok);
        continue;
      }
      if (ok) {
        gdev = ctxs[i]->device;
        grp.push_back(i);
        gctx.push_back(ctxs[i]);
        gx.push_back(x);
        gy.push_back(y);
        continue;
      }
    }
    const int rc = unit_issue1(ctxs[i], R);
    if (rc < 0) run_finish(R, rc);
  }
  if (grp.size() == 1) {
    GmresRun& R = *ctxs[grp[0]]->run;
    DeviceGuard g(gdev, __func__);
    const int rc = unit_issue1(ctxs[grp[0]], R);
    if (rc < 0) run_finish(R, rc);
  } else if (grp.size() > 1) {
    DeviceGuard g(gdev, __func__);
    // Arnoldi vectors are preconditioned in place right after the apply, so
    // their preconditioner joins the shared launches
    std::vector<int> pcs(grp.size(), 0);
    for (size_t k = 0; k < grp.size(); ++k) {
      const GmresRun& R = *ctxs[grp[k]]->run;
      if (R.phase == GP_ARNOLDI && R.pc > 0) pcs[k] = R.pc;
    }
    const int rc = op_apply_batch_f32(gctx.data(), (int)gctx.size(), gx.data(), gy.data(), pcs.data());
    for (size_t k = 0; k < grp.size(); ++k) {
      GmresRun& R = *ctxs[grp[k]]->run;
      if (rc < 0) {
        run_finish(R, rc);
        continue;
      }
      R.st.applies_fp32++;
      R.st.applies_grouped++;
      if (pcs[k]) R.st.applies_precond++;
      const int rc2 = unit_issue1_rest(ctxs[grp[k]], R, pcs[k] > 0);
      if (rc2 < 0) run_finish(R, rc2);
    }
  }
  for (int i = 0; i < n; ++i) {
    GmresRun& R = *ctxs[i]->run;
    if (R.phase == GP_DONE) continue;
    DeviceGuard g(ctxs[i]->device, __func__);
    if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess) run_finish(R, fail(TRAP_EDEVICE, "stream error"));
  }
  bool any2 = false;
  for (int i = 0; i < n; ++i) {
    GmresRun& R = *ctxs[i]->run;
    if (R.phase == GP_DONE) continue;
    DeviceGuard g(ctxs[i]->device, __func__);
    const int rc = unit_after1(ctxs[i], R);
    if (rc < 0) run_finish(R, rc);
    any2 = any2 || (R.phase == GP_ARNOLDI && R.p2);
  }
  if (any2) {
    for (int i = 0; i < n; ++i) {
      GmresRun& R = *ctxs[i]->run;
      if (R.phase != GP_ARNOLDI || !R.p2) continue;
      DeviceGuard g(ctxs[i]->device, __func__);
      if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess) run_finish(R, fail(TRAP_EDEVICE, "stream error"));
    }
    for (int i = 0; i < n; ++i) {
      GmresRun& R = *ctxs[i]->run;
      DeviceGuard g(ctxs[i]->device, __func__);
      const int rc = unit_after2(ctxs[i], R);
      if (rc < 0) run_finish(R, rc);
    }
  }
  if (status)
    for (int i = 0; i < n; ++i) status[i] = ctxs[i]->run->phase == GP_DONE ? ctxs[i]->run->status : 1;
  return TRAP_OK;
}

int gmres_end(trap_ctx* ctx, trap_solve_stats* st) {
  if (!ctx->run) return fail(TRAP_ESTATE, "no solve started");
  GmresRun& R = *ctx->run;
  if (R.phase != GP_DONE) return fail(TRAP_ESTATE, "solve still running");
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  if (st) *st = R.st;
  return R.status;
}

void gmres_release(trap_ctx* ctx) {
  if (!ctx->run) return;
  if (ctx->run->hbuf) TRAP_NOTE(hipHostFree(ctx->run->hbuf));
  delete ctx->run;
  ctx->run = nullptr;
}

int gmres_solve(trap_ctx* ctx, const trap_solve_opts* opts, double* I, trap_solve_stats* st) {
  const int rc = gmres_begin(ctx, opts, I);
  if (rc < 0) {
    if (st && ctx->run) *st = ctx->run->st;
    return rc;
  }
  if (ctx->run->phase != GP_DONE) {
    int s = 1;
    while (s == 1) gmres_step_batch(&ctx, 1, &s);
  }
  const int r = gmres_end(ctx, st);
  return r == 1 ? TRAP_OK : r;
}

}  // namespace trap
