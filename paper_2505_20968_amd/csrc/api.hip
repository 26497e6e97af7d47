// C-ABI entry points of the trap library (declared in include/trap.h), the
// context's allocation bookkeeping and the operator apply y = x - Lambda Sigma x.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "trap_internal.h"

namespace trap {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

namespace {
std::mutex g_note_mu;
long long g_note_count = 0;
std::string g_note_last;
}  // namespace

void note_hip(const char* what, const char* where, hipError_t e) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();           // the failure is recorded here, not left for a later check
  std::lock_guard<std::mutex> lk(g_note_mu);
  ++g_note_count;
  g_note_last = std::string(where) + ": " + what + " -> " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}

// Device memory comes from the device's stream-ordered pool, allocated and
// returned on the context's stream: a buffer a context frees while it lives
// (a new problem's spares) stays in the pool (its release threshold is raised
// once per device) without a device-wide synchronisation; a destroyed
// context's memory is trimmed back to the device.  Devices whose runtime has
// no pool take hipMalloc / hipFree.
namespace {
std::mutex g_pool_mu;
std::set<int> g_pool_ready, g_pool_absent;
}  // namespace

void device_pool_trim(int device) {
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool_ready.count(device)) return;
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  TRAP_NOTE(hipMemPoolTrimTo(pool, 0));
}

void device_pool_setup(int device) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_ready.count(device) || g_pool_absent.count(device)) return;
  hipMemPool_t pool;
  int supported = 0;
  if (hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, device) != hipSuccess ||
      !supported || hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess) {
    (void)hipGetLastError();
    g_pool_absent.insert(device);
    return;
  }
  uint64_t keep = UINT64_MAX;
  if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) (void)hipGetLastError();
  g_pool_ready.insert(device);
}

static bool device_pooled(int device) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  return g_pool_ready.count(device) > 0;
}

int dalloc(trap_ctx* ctx, void** p, size_t bytes) {
  void* q = nullptr;
  if (bytes == 0) bytes = 16;
  // a buffer of the same size kept from the context's previous problem
  for (size_t i = 0; i < ctx->spare.size(); ++i)
    if (ctx->spare[i].bytes == bytes) {
      ctx->bufs.push_back(ctx->spare[i]);
      ctx->spare.erase(ctx->spare.begin() + i);
      *p = ctx->bufs.back().p;
      return TRAP_OK;
    }
  const bool pooled = device_pooled(ctx->device);
  hipError_t e = pooled ? hipMallocAsync(&q, bytes, ctx->stream) : hipMalloc(&q, bytes);
  if (e != hipSuccess && pooled) {
    // the pool may hold freed blocks that fit no request: return them to the
    // device (once this stream's frees have run) and try once more
    (void)hipGetLastError();
    TRAP_NOTE(hipStreamSynchronize(ctx->stream));
    device_pool_trim(ctx->device);
    e = hipMallocAsync(&q, bytes, ctx->stream);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TRAP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                 hipGetErrorString(e));
  }
  ctx->bufs.push_back(DevBuf{q, bytes, pooled});
  *p = q;
  return TRAP_OK;
}

// A context keeps the allocations of its previous problem and hands them out
// again by exact size (same-shaped problems in a row allocate and free
// nothing); spares not reused by the next problem go back when that one is
// replaced, in stream order after the context's work.
void release_spare(trap_ctx* ctx) {
  for (auto& b : ctx->spare) {
    if (b.pooled) TRAP_NOTE(hipFreeAsync(b.p, ctx->stream));
    else TRAP_NOTE(hipFree(b.p));
  }
  ctx->spare.clear();
}

void free_all(trap_ctx* ctx) {
  if (!ctx->bufs.empty()) TRAP_NOTE(hipStreamSynchronize(ctx->stream));
  gmres_release(ctx);
  release_spare(ctx);
  ctx->spare.swap(ctx->bufs);
  auto& hs = ctx->host_spare;
  hs.td = std::move(ctx->pb.td);
  hs.qk = std::move(ctx->pb.qk);
  hs.qk32 = std::move(ctx->pb.qk32);
  hs.qb = std::move(ctx->pb.qb);
  hs.qb32 = std::move(ctx->pb.qb32);
  hs.tofs = std::move(ctx->pb.tofs);
  ctx->pb = Problem();
  ctx->pre = Precomp();
  ctx->wk = Work();
  ctx->has_problem = false;
}

int UploadBatch::commit(trap_ctx* ctx) {
  if (items.empty()) return TRAP_OK;
  void* base = nullptr;
  TRAP_TRY(dalloc(ctx, &base, total));
  for (const Item& it : items)
    if (it.dst) *it.dst = static_cast<unsigned char*>(base) + it.off;
  return stage_upload_batch(ctx, *this, base);
}

template <typename T>
__global__ void k_sub_from(long long N, const T* __restrict__ x, T* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i] - y[i];
}

int operator_apply(trap_ctx* ctx, const void* x, void* y, int prec) {
  if (prec != TRAP_FP64 && prec != TRAP_FP32) return fail(TRAP_EINVAL, "unknown precision");
  TRAP_TRY(ensure_work(ctx, prec));
  const int pi = prec == TRAP_FP64 ? 0 : 1;
  void* e = ctx->wk.opeps[pi];
  TRAP_TRY(sigma_apply(ctx, x, e, prec, 0, 1));
  TRAP_TRY(formal_apply(ctx, e, y, 0, prec));
  const long long N = 4LL * ctx->pb.nz * ctx->pb.nd * ctx->pb.nn;
  if (prec == TRAP_FP64)
    hipLaunchKernelGGL(k_sub_from<double>, dim3(1024), dim3(256), 0, ctx->stream, N,
                       static_cast<const double*>(x), static_cast<double*>(y));
  else
    hipLaunchKernelGGL(k_sub_from<float>, dim3(1024), dim3(256), 0, ctx->stream, N,
                       static_cast<const float*>(x), static_cast<float*>(y));
  TRAP_HIP(hipGetLastError());
  return TRAP_OK;
}

int prof_begin(trap_ctx* ctx, int stage, double flops, double bytes) {
  Prof& P = ctx->prof;
  if (!P.on) return -1;
  if (P.used == P.rec.size()) {
    ProfRec r{stage, nullptr, nullptr, 0.0, 0.0};
    if (hipEventCreate(&r.a) != hipSuccess) return -1;
    if (hipEventCreate(&r.b) != hipSuccess) {
      TRAP_NOTE(hipEventDestroy(r.a));
      return -1;
    }
    P.rec.push_back(r);
  }
  ProfRec& r = P.rec[P.used];
  r.stage = stage;
  r.flops = flops;
  r.bytes = bytes;
  TRAP_NOTE(hipEventRecord(r.a, ctx->stream));
  return static_cast<int>(P.used++);
}

void prof_end(trap_ctx* ctx, int idx) {
  if (idx < 0) return;
  TRAP_NOTE(hipEventRecord(ctx->prof.rec[idx].b, ctx->stream));
}

static void prof_clear(trap_ctx* ctx, bool release) {
  if (release) {
    for (auto& r : ctx->prof.rec) {
      TRAP_NOTE(hipEventDestroy(r.a));
      TRAP_NOTE(hipEventDestroy(r.b));
    }
    ctx->prof.rec.clear();
  }
  ctx->prof.used = 0;
}

}  // namespace trap

using namespace trap;

extern "C" {

int trap_hip_notes(long long* count, char* buf, size_t n) {
  std::lock_guard<std::mutex> lk(trap::g_note_mu);
  if (count) *count = trap::g_note_count;
  if (buf && n > 0) {
    const size_t k = std::min(n - 1, trap::g_note_last.size());
    std::memcpy(buf, trap::g_note_last.data(), k);
    buf[k] = 0;
  }
  return TRAP_OK;
}

const char* trap_last_error(void) { return g_last_error.c_str(); }

int trap_create(trap_ctx** out, int device, void* stream) {
  if (!out) return fail(TRAP_EINVAL, "null output pointer");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(TRAP_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(TRAP_EINVAL, "device index out of range");
  trap_ctx* ctx = new (std::nothrow) trap_ctx();
  if (!ctx) return fail(TRAP_ENOMEM, "host allocation failed");
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    ctx->max_lds = std::min(lds, 160 * 1024);
  else
    (void)hipGetLastError();
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    ctx->n_cu = ncu;
  else
    (void)hipGetLastError();
  batch_arena_acquire(device);
  device_pool_setup(device);
  *out = ctx;
  return TRAP_OK;
}

int trap_destroy(trap_ctx* ctx) {
  if (!ctx) return TRAP_OK;
  DeviceGuard g(ctx->device, __func__);
  prof_clear(ctx, true);
  free_all(ctx);
  release_spare(ctx);
  if (ctx->side) {
    TRAP_NOTE(hipStreamSynchronize(ctx->side));
    TRAP_NOTE(hipStreamDestroy(ctx->side));
  }
  if (ctx->ev_fork) TRAP_NOTE(hipEventDestroy(ctx->ev_fork));
  if (ctx->ev_join) TRAP_NOTE(hipEventDestroy(ctx->ev_join));
  (void)batch_arena_release(ctx->device);
  // the context's memory goes back to the device once its stream-ordered
  // frees have run: freed blocks kept in the pool are invisible to every
  // other allocator, the runtime's own (kernel scratch) included, so a
  // stream of contexts of different sizes would otherwise exhaust the device
  TRAP_NOTE(hipStreamSynchronize(ctx->stream));
  device_pool_trim(ctx->device);
  delete ctx;
  return TRAP_OK;
}

int trap_set_problem(trap_ctx* ctx, const trap_atom_desc* atom, const trap_problem_desc* prob) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  free_all(ctx);
  int s = build_problem(ctx, atom, prob);
  if (s != TRAP_OK) {
    std::string msg = g_last_error;
    free_all(ctx);
    return fail(s, msg);
  }
  if (ctx->pb.nl > 8 || ctx->pb.nu > 16 || ctx->pb.nchi > 16 || ctx->pb.nchi * ctx->pb.nl > 32) {
    free_all(ctx);
    return fail(TRAP_EINVAL, "too many sublevels or azimuths (n_lower <= 8, n_upper <= 16, n_chi <= 16, n_chi * n_lower <= 32)");
  }
  // the upload is in flight on the context's stream (from a pinned buffer the
  // device's pool keeps until the copy has finished); later work is ordered after it
  ctx->has_problem = true;
  return TRAP_OK;
}

int trap_precompute(trap_ctx* ctx, int store_mask) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (store_mask & ~3) return fail(TRAP_EINVAL, "store_mask has unknown bits");
  DeviceGuard g(ctx->device, __func__);
  return run_precompute(ctx, store_mask);
}

int trap_precompute_preconditioner(trap_ctx* ctx) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (ctx->pre.pc_done) return TRAP_OK;
  DeviceGuard g(ctx->device, __func__);
  return run_precompute_precond(ctx);
}

int trap_apply_preconditioner(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return precond_apply(ctx, r, out, sweeps, prec);
}

int trap_apply_preconditioner_noalloc(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return precond_apply_noalloc(ctx, r, out, sweeps, prec);
}

int trap_preconditioner_tables(trap_ctx* ctx, double* phi, double* c, double* lloc) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem || !ctx->pre.pc_done) return fail(TRAP_ESTATE, "preconditioner tables not computed");
  DeviceGuard g(ctx->device, __func__);
  const Problem& P = ctx->pb;
  const size_t nmat = (size_t)P.nz * P.nn * P.nn, nloc = (size_t)P.nz * P.nd * P.nn;
  if (phi) TRAP_HIP(hipMemcpyAsync(phi, ctx->pre.d_pcPhi, nmat * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (c) TRAP_HIP(hipMemcpyAsync(c, ctx->pre.d_pcC, nmat * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (lloc) TRAP_HIP(hipMemcpyAsync(lloc, ctx->pre.d_pcL, nloc * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  return TRAP_OK;
}

int trap_apply_sigma(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return sigma_apply(ctx, I, eps, prec, add_thermal, 1);
}

int trap_formal_solve(trap_ctx* ctx, const void* eps, void* I, int with_boundary, int prec) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return formal_apply(ctx, eps, I, with_boundary, prec);
}

int trap_apply_operator(trap_ctx* ctx, const void* x, void* y, int prec) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (!x || !y) return fail(TRAP_EINVAL, "null vector");
  DeviceGuard g(ctx->device, __func__);
  return operator_apply(ctx, x, y, prec);
}

int trap_rhs(trap_ctx* ctx, double* b_out) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (!b_out) return fail(TRAP_EINVAL, "null vector");
  DeviceGuard g(ctx->device, __func__);
  const size_t N = 4ull * ctx->pb.nz * ctx->pb.nd * ctx->pb.nn;
  TRAP_HIP(hipMemcpyAsync(b_out, ctx->pre.d_b, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return TRAP_OK;
}

int trap_gmres_solve(trap_ctx* ctx, const trap_solve_opts* opts, double* I, trap_solve_stats* stats) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return gmres_solve(ctx, opts, I, stats);
}

int trap_emergent(trap_ctx* ctx, const double* I, double* host_out) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (!I || !host_out) return fail(TRAP_EINVAL, "null pointer");
  DeviceGuard g(ctx->device, __func__);
  const Problem& P = ctx->pb;
  const size_t rec = (size_t)P.nn * 4;
  const double* top = I + (size_t)(P.nz - 1) * P.nd * rec;
  size_t k = 0;
  for (int o = 0; o < P.ngrid; ++o) {
    if (P.mu[o] <= 0.0) continue;
    TRAP_HIP(hipMemcpyAsync(host_out + k * rec, top + (size_t)o * rec, rec * sizeof(double),
                            hipMemcpyDeviceToHost, ctx->stream));
    ++k;
  }
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  return TRAP_OK;
}

int trap_formal_from_field(trap_ctx* ctx, const double* I, int n_dir_in, double* out) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  if (!I || !out) return fail(TRAP_EINVAL, "null vector");
  const Problem& P = ctx->pb;
  if (n_dir_in != P.nd && n_dir_in != P.ngrid)
    return fail(TRAP_EINVAL, "n_dir_in must be n_dir or the quadrature count n_mu * n_chi");
  const size_t rec = (size_t)P.nn * 4 * sizeof(double);
  const size_t N = (size_t)P.nz * P.nd * rec;
  const char* ib = reinterpret_cast<const char*>(I);
  const char* ob = reinterpret_cast<const char*>(out);
  if (ib < ob + N && ob < ib + (size_t)P.nz * n_dir_in * rec) return fail(TRAP_EINVAL, "out overlaps I");
  DeviceGuard g(ctx->device, __func__);
  TRAP_TRY(ensure_work(ctx, TRAP_FP64));
  const double* x = I;
  if (n_dir_in != P.nd) {
    // the quadrature directions per height into the full layout, the rings zero
    TRAP_HIP(hipMemcpy2DAsync(out, P.nd * rec, I, P.ngrid * rec, P.ngrid * rec, P.nz, hipMemcpyDeviceToDevice,
                              ctx->stream));
    TRAP_HIP(hipMemset2DAsync(reinterpret_cast<char*>(out) + P.ngrid * rec, P.nd * rec, 0, (P.nd - P.ngrid) * rec,
                              P.nz, ctx->stream));
    x = out;
  }
  void* e = ctx->wk.opeps[0];
  TRAP_TRY(sigma_apply(ctx, x, e, TRAP_FP64, 1, 1));   // Sigma I + eps_th
  TRAP_TRY(formal_apply(ctx, e, out, 1, TRAP_FP64));   // Lambda (...) + t
  return TRAP_OK;
}

int trap_emergent_los(trap_ctx* ctx, const double* I, double* host_out) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  if (!I || !host_out) return fail(TRAP_EINVAL, "null pointer");
  const Problem& P = ctx->pb;
  if (P.nlos == 0) return fail(TRAP_EINVAL, "the problem has no lines of sight");
  DeviceGuard g(ctx->device, __func__);
  const size_t rec = (size_t)P.nn * 4;
  const double* top = I + ((size_t)(P.nz - 1) * P.nd + P.ngrid) * rec;   // the rings follow the quadrature
  TRAP_HIP(hipMemcpyAsync(host_out, top, (size_t)(P.nd - P.ngrid) * rec * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  return TRAP_OK;
}

int trap_get_info(const trap_ctx* ctx, trap_info* info) {
  if (!ctx || !info) return fail(TRAP_EINVAL, "null argument");
  if (!ctx->has_problem) return fail(TRAP_ESTATE, "no problem loaded");
  const Problem& P = ctx->pb;
  std::memset(info, 0, sizeof(*info));
  info->n_z = P.nz;
  info->n_nu = P.nn;
  info->n_dir = P.nd;
  info->n_theta = P.nth;
  info->n_slots = P.nslot;
  info->n_up = P.nu;
  info->n_lo = P.nl;
  info->n_trans = P.nt;
  info->n_unknowns = 4ull * P.nz * P.nd * P.nn;
  // the banded store: FP32 values (the FP32 kernel) and FP32 remainders (with
  // the values, the FP64 kernel)
  const double kel = (double)P.kentries;
  info->bytes_kernel_fp64 = P.kentries * 8;
  info->bytes_kernel_fp32 = P.kentries * 4;
  info->kernel_entries = (long long)P.band_nnz;
  info->band_reach = P.band_reach;
  size_t tot = 0;
  for (auto& b : ctx->bufs) tot += b.bytes;
  for (auto& b : ctx->spare) tot += b.bytes;
  info->bytes_device_total = tot;
  // per stored complex kernel entry: 4 Stokes columns x (real, imag) multiply-adds = 16 flops per slot
  info->flops_contraction = chunk_flops(P, 0, P.nz);
  // algorithmic bytes: every stored kernel entry read once (FP32 values; FP64
  // adds the remainders), Ibar read, W written once
  const double wbytes = (double)P.nz * P.nt * P.nslot * 2.0 * P.nn * 4;
  const double ibytes = (double)P.nz * P.nd * P.nn * 4;
  info->bytes_contraction_fp64 = 8.0 * (kel + wbytes + ibytes);
  info->bytes_contraction_fp32 = 4.0 * (chunk_entries32(P, 0, P.nz) + wbytes + ibytes);
  info->flops_contraction_fp32 = chunk_flops32(P, 0, P.nz);
  info->kernel_entries_fp32 = (long long)P.band_nnz32;
  info->band_reach_fp32 = P.band_reach32;
  info->kernel_rows_mirrored = P.rows_mirrored;
  return TRAP_OK;
}

int trap_kernel_rows(trap_ctx* ctx, int z, int theta, int t, double* theta_out, double* shift_out,
                     double* host_out) {
  if (!ctx || !host_out) return fail(TRAP_EINVAL, "null argument");
  if (!ctx->has_problem || !ctx->pre.done) return fail(TRAP_ESTATE, "precompute not run");
  const Problem& P = ctx->pb;
  if (z < 0 || z >= P.nz || theta < 0 || theta >= P.nth || t < 0 || t >= P.nt)
    return fail(TRAP_EINVAL, "kernel index out of range");
  DeviceGuard g(ctx->device, __func__);
  const size_t zt = (size_t)z * P.nth + theta, nn = P.nn;
  const long long first = P.kbase[zt];
  const long long last = zt + 1 < P.kbase.size() ? P.kbase[zt + 1] : (long long)P.kentries;
  const size_t cnt = (size_t)(last - first);
  std::vector<float> hi(cnt), lo(cnt);
  TRAP_HIP(hipMemcpyAsync(hi.data(), ctx->pre.d_Mhi + first, cnt * sizeof(float), hipMemcpyDeviceToHost,
                          ctx->stream));
  TRAP_HIP(hipMemcpyAsync(lo.data(), ctx->pre.d_Mlo + first, cnt * sizeof(float), hipMemcpyDeviceToHost,
                          ctx->stream));
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  std::fill(host_out, host_out + 2 * nn * nn, 0.0);
  for (int c = 0; c < 2; ++c)
    for (size_t n = 0; n < nn; ++n) {
      int q, lr;
      row_tile(P.qpad, 2 * P.nt, P.nn, 2 * t + c, (int)n, &q, &lr);
      const unsigned w = P.qk[zt * P.nq + q];
      const int a = (int)(w & 0xffffu), b = (int)(w >> 16);
      const size_t row = (size_t)P.tofs[zt * P.nq + q] + (size_t)lr * (b - a);
      for (int m = a; m < b && m < (int)nn; ++m)
        host_out[(c * nn + n) * nn + m] = (double)hi[row + m - a] + (double)lo[row + m - a];
    }
  if (theta_out) *theta_out = P.theta[theta];
  if (shift_out) {
    std::vector<double> st(P.nt);
    TRAP_HIP(hipMemcpy(st.data(), P.d_st + (size_t)z * P.nt, P.nt * sizeof(double), hipMemcpyDeviceToHost));
    *shift_out = st[t];
  }
  return TRAP_OK;
}

int trap_faddeeva(int device, const double* v, const double* a, int n, double* out) {
  if (!v || !a || !out || n < 0) return fail(TRAP_EINVAL, "null argument or negative count");
  for (int i = 0; i < n; ++i)
    if (!(a[i] >= 0.0) || !std::isfinite(v[i])) return fail(TRAP_EINVAL, "points need finite v and a >= 0");
  if (n == 0) return TRAP_OK;
  DeviceGuard g(device, __func__);
  return faddeeva_eval(device, v, a, n, out);
}

int trap_gmres_begin(trap_ctx* ctx, const trap_solve_opts* opts, double* I) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return gmres_begin(ctx, opts, I);
}

int trap_gmres_step_batch(trap_ctx** ctxs, int n, int* status) {
  if (n < 0 || (n > 0 && (!ctxs || !status))) return fail(TRAP_EINVAL, "null argument");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(TRAP_EINVAL, "null context in batch");
    if (!ctxs[i]->run) return fail(TRAP_ESTATE, "trap_gmres_begin not called for a context in the batch");
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return fail(TRAP_EINVAL, "context listed twice in batch");
  }
  return gmres_step_batch(ctxs, n, status);
}

int trap_gmres_end(trap_ctx* ctx, trap_solve_stats* stats) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  return gmres_end(ctx, stats);
}

int trap_set_prd_mode(trap_ctx* ctx, int mode) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (mode != TRAP_PRD_AD && mode != TRAP_PRD_AA) return fail(TRAP_EINVAL, "unknown PRD mode");
  ctx->prd_mode = mode;
  return TRAP_OK;
}

int trap_set_interpolation(trap_ctx* ctx, int mode) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (mode != TRAP_INTERP_SPLINE && mode != TRAP_INTERP_WENO4) return fail(TRAP_EINVAL, "unknown interpolation");
  if (ctx->pre.done && mode != ctx->interp)
    return fail(TRAP_ESTATE, "the interpolation is fixed once trap_precompute has run for the problem");
  ctx->interp = mode;
  return TRAP_OK;
}

int trap_set_formal_scheme(trap_ctx* ctx, int scheme) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (scheme != TRAP_FORMAL_DELO_LINEAR && scheme != TRAP_FORMAL_DELOPAR && scheme != TRAP_FORMAL_BESSER)
    return fail(TRAP_EINVAL, "unknown formal scheme");
  if (ctx->pre.done && scheme != ctx->formal_scheme)
    return fail(TRAP_ESTATE, "the formal scheme is fixed once trap_precompute has run for the problem");
  ctx->formal_scheme = scheme;
  return TRAP_OK;
}

int trap_set_path(trap_ctx* ctx, int path) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  if (path != TRAP_PATH_AUTO && path != TRAP_PATH_FUSED && path != TRAP_PATH_CHUNKED)
    return fail(TRAP_EINVAL, "unknown Sigma path");
  ctx->path = path;
  return TRAP_OK;
}

int trap_profile(trap_ctx* ctx, int enable) {
  if (!ctx) return fail(TRAP_EINVAL, "null context");
  DeviceGuard g(ctx->device, __func__);
  if (enable) {
    TRAP_HIP(hipStreamSynchronize(ctx->stream));
    prof_clear(ctx, false);
  }
  ctx->prof.on = enable != 0;
  return TRAP_OK;
}

int trap_stage_times(trap_ctx* ctx, trap_stage_stats* out) {
  if (!ctx || !out) return fail(TRAP_EINVAL, "null argument");
  DeviceGuard g(ctx->device, __func__);
  std::memset(out, 0, sizeof(*out));
  TRAP_HIP(hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < ctx->prof.used; ++i) {
    const ProfRec& r = ctx->prof.rec[i];
    float ms = 0.0f;
    TRAP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.stage >= 0 && r.stage < TRAP_STAGE_COUNT) {
      out->ms[r.stage] += ms;
      out->launches[r.stage] += 1;
    }
    const int pi = r.stage == TRAP_STAGE_CONTRACT_FP64 ? 1 : 0;
    out->flops_contraction[pi] += r.flops;
    out->bytes_contraction[pi] += r.bytes;
  }
  return TRAP_OK;
}

int trap_footprint(const trap_atom_desc* atom, const trap_problem_desc* prob, int store_mask,
                   size_t* bytes) {
  if (!bytes) return fail(TRAP_EINVAL, "null output");
  int err = 0;
  *bytes = estimate_bytes(atom, prob, store_mask, &err);
  if (err) return fail(TRAP_EINVAL, "bad problem description");
  return TRAP_OK;
}

}  // extern "C"
