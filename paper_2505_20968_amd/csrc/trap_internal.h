// Internal definitions of the trap library: context layout, error helpers,
// launch helpers and small device utilities shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/trap.h"

namespace trap {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define TRAP_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::trap::fail(TRAP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRAP_TRY(call)              \
  do {                              \
    int s_ = (call);                \
    if (s_ != TRAP_OK) return s_;   \
  } while (0)

// ---------------------------------------------------------------- complex helpers
struct cplx { double re, im; };

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// ---------------------------------------------------------------- device buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool pooled = false;     // from the device's stream-ordered pool (freed with hipFreeAsync)
};

// ---------------------------------------------------------------- host tables written in full
// An allocator whose resize leaves trivially constructible elements
// unwritten (default-initialised): for large host tables that are filled
// completely right afterwards, often by several threads, so that no serial
// zero fill precedes the work and each page is first touched by its writer.
template <typename T>
struct DefaultInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = DefaultInitAlloc<U>;
  };
  DefaultInitAlloc() = default;
  template <typename U>
  DefaultInitAlloc(const DefaultInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <typename T>
using host_vec = std::vector<T, DefaultInitAlloc<T>>;

// ---------------------------------------------------------------- banded kernel store
// Each R_II kernel row is nonzero only where the Gaussian factor of F reaches
// (Sect. 2.4, App. C) plus the reach of the cardinal spline basis (its band).
// The contraction multiplies 16-row wave tiles; the store keeps, per tile,
// the 16 rows over the union of their bands (columns lo .. hi - 1, multiples
// of 8) as one dense [16][hi - lo] block.  The GEMM rows of (z, theta) are
// np = 2 nt planes (transition t, real/imaginary c, p = 2 t + c) of nnp rows:
// nnp = nn, or nn padded to 16 when that wastes less work than tiles that
// straddle two planes.  Tiles are numbered in `block order` (tile_row0: first
// row of each), eight per block of the contraction; td holds each tile's
// store offset and column range, qb each block's range as lo | hi << 16.
struct TileDesc {
  long long off;    // store index of the tile's row 0, column lo
  int lo, hi;       // column range, multiples of 8
};
struct KStore {
  const float* hi = nullptr;          // FP32 kernel values
  const float* lo = nullptr;          // FP32 remainders: hi + lo is the FP64 kernel
  const TileDesc* td = nullptr;       // [nz][nth][nq]
  const unsigned* qb = nullptr;       // [nz][nth][nqb]
  // optional column windows inside td / qb (lo | hi << 16) that the products
  // step through (the FP32 operator's), the addresses still from td
  const unsigned* t32 = nullptr;      // [nz][nth][nq]
  const unsigned* qb32 = nullptr;     // [nz][nth][nqb]
  int np = 0, nnp = 0, nq = 0, nqb = 0;
  int pad = 0;
};

// row stride (frequencies) of the contraction's intermediate W[z][t][slot][c][n][s]:
// the frequency count rounded up to 8, so that every row of W starts on a
// 128-byte boundary in FP32 (the contraction's 256-byte tile runs and the
// angular sum's 1 KB reads then cover whole cache lines)
__host__ __device__ inline int w_stride(int nn) { return (nn + 7) & ~7; }

// first GEMM row of wave tile q (block order)
__host__ __device__ inline int tile_row0(int pad, int np, int nnp, int q) {
  return pad ? (q % np) * nnp + 16 * (q / np) : 16 * q;
}

// wave tile and row within it of GEMM row (plane p, frequency n)
__host__ __device__ inline void row_tile(int pad, int np, int nn, int p, int n, int* q, int* lr) {
  if (pad) {
    *q = (n >> 4) * np + p;
    *lr = n & 15;
  } else {
    const int r = p * nn + n;
    *q = r >> 4;
    *lr = r & 15;
  }
}

// ---------------------------------------------------------------- context
// Index conventions (all row-major, last index fastest):
//   vectors        V[z][o][n][s]
//   spline map     P[k][p][m]      interval k (0..nn-2), power p of t=(x-x_k)/h_k, node m
//   kernels        banded, in 16-row tiles (KStore): row (z, theta, plane p = 2 t + c, n),
//                  c = 0 real / 1 imaginary, in tile q at row lr, columns [lo_q, hi_q)
//                  at base[z][theta] + tofs[z][theta][q] + lr (hi_q - lo_q); FP32 hi and
//                  lo words (hi = the FP32 kernel, hi + lo the FP64 one)
//   W intermediate W[zc][t][slot][c][n][s]   (height chunk zc)
//   eps_bar        Eb[z][l][l'][o][n][s]
//   coefficients   cf[z][p][t][c][l'][i][j]  p = pair index in slot-major order; c = 0 multiplies
//                  Re W, c = 1 multiplies Im W
//   E table        E[z][o][i][u'][u][l']   = d_{u'l'}^T Acart_i(o) d^*_{u l'}
//   A table        A[z][o'][j][u][u'][l]   = d_{u l}^T Acart_j(o')/2 d^*_{u' l}
//   transitions    t = u * n_lo + l
struct Problem {
  int nz = 0, nn = 0, nmu = 0, nchi = 0, nd = 0;
  int nlos = 0, ngrid = 0;                 // line-of-sight rings; quadrature directions nmu * nchi
  // kernel rows by mirror symmetry (empty: every row is computed).  On a grid
  // symmetric about x = 0 the rows of shift s and -s satisfy
  // M_s[n][m] = conj(M_{-s}[nn-1-n][nn-1-m]); row_role[t] = -1: all rows of t
  // computed; = t: rows n <= nn-1-n computed, the others mirrored from t; = t2
  // < t: every row mirrored from the fully computed t2
  std::vector<int> row_role;
  long long rows_mirrored = 0;             // complex kernel rows per (height, angle) taken from mirror images
  std::vector<double> los_mu;              // [nlos] mu of each zero-weight ring
  int nth = 0, nslot = 0, nu = 0, nl = 0, nt = 0;
  int max_slots_per_theta = 0;
  int ldm = 0;                             // row length of the precompute's dense row scratch (multiple of 8)
  // banded kernel store (see KStore): spline reach in nodes, the layout of
  // the tiles, the stored real entries, the complex entries inside the rows'
  // own bands, and the algorithmic flops of one contraction per height
  // (16 per in-band complex entry and incoming slot of its angle)
  int band_reach = 0;
  int nnp = 0, nq = 0, nqb = 0, qpad = 0;
  std::vector<long long> kbase;
  host_vec<int> tofs;
  std::vector<int> qrow0;
  host_vec<unsigned> qk, qb;
  size_t kentries = 0;
  double band_nnz = 0.0;
  std::vector<double> kflops_z;
  host_vec<TileDesc> td;
  TileDesc* d_td = nullptr;
  unsigned* d_qb = nullptr;
  // the FP32 operator's narrower window inside each tile and block (lo | hi
  // << 16, columns, multiples of 8): the same stored rows cut where the
  // kernel falls below the FP32 operator's resolution (kernel_bands); its
  // reach, in-band complex entries, stored real entries and flops per height
  int band_reach32 = 0;
  host_vec<unsigned> qk32, qb32;
  double band_nnz32 = 0.0;
  std::vector<double> kflops32_z, kent32_z;
  unsigned* d_qk32 = nullptr;
  unsigned* d_qb32 = nullptr;
  double c_abs = 0, c_sc = 0;
  // host copies used by host-side logic
  std::vector<double> x, mu, w, tau, lam, a, eps, WT, eta0, dnuD;
  std::vector<double> theta;               // [nth]
  int prd_mode = 0;                        // TRAP_PRD_AD or TRAP_PRD_AA
  // scattering angles at which kernel rows are computed: the Theta table (AD)
  // or the Gauss-Legendre nodes of the angle average (AA, weights theta_rw)
  std::vector<double> theta_rows, theta_rw;
  int nth_rows = 0;
  std::vector<int> slot_off;               // [nth+1]
  std::vector<int> slot_dir;               // [nslot]
  std::vector<int> slot_theta;             // [nslot]
  std::vector<int> pair_slot;              // [nd][nd] slot of (theta(o,i), i)
  std::vector<int> pair_theta;             // [nd][nd]
  std::vector<int> pair_off;               // [nslot+1] pairs (o, o') of each slot, slot-major
  std::vector<int> pair_o;                 // [nd*nd]   outgoing direction of each pair
  std::vector<int> pair_dir;               // [nd*nd]   incoming direction of each pair
  std::vector<int> pair_index;             // [nd][nd]  pair index of (o, o')
  // slot groups for the fused Sigma kernel: {theta, first slot, slot count}
  std::vector<int> grp[2];                 // [0] FP64 (8 slots), [1] FP32 (16 slots)
  int grp_maxpairs[2] = {0, 0};            // most pairs in one group
  // column groups of the R_II contraction {theta, first slot, slot count} per
  // precision: FP64 <= 16 slots; FP32 <= 32, the cgrp_n8 groups of 17..32 slots first
  std::vector<int> cgrp[2];
  int cgrp_n8[2] = {0, 0};
  // the FP32 groups by decreasing work (both classes interleaved): the
  // resident-field contraction's work order; its unit ticket and finished-block
  // count (zero between launches: the last block to finish resets them)
  std::vector<int> cord, unit_ctr;
  std::vector<int> cord0;                  // the same order for the FP64 groups (at most 16 slots)
  // device copies
  double *d_x = nullptr, *d_P = nullptr, *d_mu = nullptr, *d_w = nullptr, *d_tau = nullptr;
  double *d_Sig = nullptr;                 // [nn][nn] second-derivative map of the spline
  double *d_SigT = nullptr;                // its transpose
  double *d_lam = nullptr, *d_a = nullptr, *d_eps = nullptr, *d_WT = nullptr, *d_eta0 = nullptr;
  double *d_ub = nullptr;                  // [nz][nd] reduced Doppler shift (u units)
  double *d_st = nullptr;                  // [nz][nt] reduced transition shifts
  double *d_sll = nullptr;                 // [nz][nl][nl] lower-level shifts
  double *d_theta = nullptr;               // [nth]
  double *d_theta_rows = nullptr;          // [nth_rows]
  double *d_theta_rw = nullptr;            // [nth_rows] AA weights
  int *d_slot_theta = nullptr, *d_slot_dir = nullptr, *d_slot_off = nullptr, *d_pair_slot = nullptr;
  int* d_pair_theta = nullptr;             // [nd][nd] Theta index of each pair (flat-field applies)
  int *d_pair_off = nullptr, *d_pair_o = nullptr, *d_pair_dir = nullptr, *d_pair_index = nullptr;
  int *d_grp[2] = {nullptr, nullptr};
  int *d_cgrp[2] = {nullptr, nullptr};
  int* d_cord = nullptr;
  int* d_unit_ctr = nullptr;
  int* d_cord0 = nullptr;
  double2 *d_E = nullptr, *d_A = nullptr;  // see above
  double2 *d_alpha = nullptr, *d_bma = nullptr; // [nz][nu][nu]
  double *d_g = nullptr;                   // [nz][nt][nd][4] geometric factors of K
  // continuum (App. A): kappa_c, sigma_c [nz][nn] relative to the line-centre
  // absorption, and the polarisation axes of each direction for its scattering
  bool has_cont = false;
  std::vector<double> kc, sc;
  double *d_kc = nullptr, *d_sc = nullptr, *d_ea = nullptr, *d_eb = nullptr;
  // physics-based preconditioner (unmagnetised, unpolarised, angle-averaged,
  // K = Q = 0): transitions of the zero-field atom grouped by frequency
  // (pc_nk classes, energy differences pc_dE in Hz); per height the weights
  // of the class kernels in the comoving coupling (R_II: real and imaginary
  // planes, pc_cr / pc_ci [nz][nk]; R_III: four complex [nk][nk] blocks
  // pc_X [nz][4][nk][nk]); directions grouped by Doppler shift per height
  // (pc_mem [nz][nd] directions ordered by class, class c holding
  // pc_mem[pc_moff[c] .. pc_moff[c + 1]) of its height, pc_moff [nz][nd + 1];
  // pc_cub [nz][nd] class shifts in u units, pc_ncls [nz] class count)
  int pc_nk = 0;
  std::vector<double> pc_dE, pc_cr, pc_ci, pc_cub;
  std::vector<double2> pc_X;
  std::vector<int> pc_mem, pc_moff, pc_ncls;
};

struct Precomp {
  bool done = false;
  int store_mask = 0;
  double *d_K = nullptr;      // [z][o][n][8]: kQ,kU,kV,rQ,rU,rV (over eta_I), 1/eta_I, eta_I/eta_0
  double *d_epsth = nullptr;  // [z][o][n][4]
  double *d_f = nullptr;      // [z][o][n]
  float *d_Mhi = nullptr;     // banded kernels: FP32 values (the FP32 kernel)
  float *d_Mlo = nullptr;     //   and the FP32 remainders (hi + lo = the FP64 kernel)
  double2 *d_r3 = nullptr;    // [z][t][n] R_III incoming weights
  double2 *d_prof = nullptr;  // [z][t][n] outgoing profiles on the comoving grid
  double *d_b = nullptr;      // right-hand side, FP64 vector
  double *d_Mtmp = nullptr;   // AA: kernels at the Theta nodes of one height chunk, FP64
  double *d_cf64 = nullptr;   // angular coefficients [z][pair][t][c][l'][i][j], FP64
  float *d_cf32 = nullptr;    //   and FP32
  double *d_Gt = nullptr;     // Gaussian factor table of the kernel precompute (uniform grids)
  double2 *d_Vt = nullptr;    // Faddeeva factor table of the kernel precompute (uniform grids)
  double *d_Lrow = nullptr;   // local part of the kernel rows, [rows][ldm] (height chunk)
  double *d_Grow = nullptr;   // second-derivative weights of the kernel rows, [rows][ldm]
  int2* d_gspan = nullptr;    // node span of each complex row's nonzero weights (height chunk)
  int zc_rows = 0;            // heights per precompute chunk
  // preconditioner tables (FP64), present once pc_done
  bool pc_done = false;
  double *d_pcPhi = nullptr;  // [z][n][m] comoving coupling Phi_z
  double *d_pcC = nullptr;    // [z][n][m] Phi_z (Id - A_z)^-1
  double *d_pcL = nullptr;    // [z][o][n] local Lambda (diagonal of the scalar formal solution)
  double2 *d_pcF = nullptr;   // [z][o][n] scalar DELO step into z: (exp(-dtau), psi_u / eta_I upwind)
  double *d_pcA = nullptr;    // [z][m'][m] A_z, then the Gauss-Jordan scratch [z][nn][2 nn]
  double *d_pcM = nullptr;    // [z][k][c][n][ldm] angle-averaged kernels of the zero-field classes
  double2 *d_pcR3 = nullptr;  // [z][k][n] R_III weights of the classes
  double2 *d_pcProf = nullptr;// [z][k][n] profiles of the classes on the comoving grid
  double *d_pcSt = nullptr;   // [z][k] class shifts (u units)
  double *d_pcCr = nullptr, *d_pcCi = nullptr;
  double2 *d_pcX = nullptr;
  int *d_pcMem = nullptr, *d_pcMoff = nullptr, *d_pcNcls = nullptr;
  double *d_pcCub = nullptr;
  double *d_pcTheta = nullptr, *d_pcRw = nullptr;   // Gauss-Legendre angles and weights of the average
  int pc_ncmax = 0;            // most Doppler-shift classes at one height
};

struct Work {
  // scratch for the Sigma apply, per precision
  void *Ibar[2] = {nullptr, nullptr};
  void *W[2] = {nullptr, nullptr};
  void *Eb[2] = {nullptr, nullptr};
  void *tmp[2] = {nullptr, nullptr};     // internal to the Sigma apply
  void *opeps[2] = {nullptr, nullptr};   // emissivity inside the operator apply
  double2 *Y = nullptr;       // [z][t][o][4]
  double2 *X = nullptr;       // [z][u][u'][l]
  int zchunk = 1;
  // solver vectors
  double *V = nullptr;        // Krylov basis, (restart+1) x N
  float *v32a = nullptr, *v32b = nullptr;
  double *r = nullptr, *x = nullptr, *tmp64 = nullptr, *red = nullptr;
  double *dots = nullptr;     // reduction scratch for the block dot-products
  int V_cols = 0;
  // preconditioner sweeps: Stokes-I fields [z][o][n] and per-height vectors
  double *pc_x = nullptr, *pc_e = nullptr, *pc_res = nullptr;
  double *pc_h = nullptr;     // [z][2][nn]: comoving vector and its spline second derivatives
  double *pc_gc = nullptr;    // [z][class][nn]: comoving interpolation of each Doppler class's angular sum
  // alternating Anderson-Richardson: r, f, previous x and f, then `aar_cap`
  // differences of x and of f, all N long; block partial dot products
  double *aar = nullptr, *aar_part = nullptr;
  int aar_cap = -1;
};

struct ProfRec {
  int stage;
  hipEvent_t a, b;
  double flops, bytes;
};

struct GmresRun;   // solver state of one context (solver.hip)

struct Prof {
  bool on = false;
  std::vector<ProfRec> rec;      // records [0, used) are live; events are reused
  size_t used = 0;
};

}  // namespace trap

struct trap_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool has_problem = false;
  trap::Problem pb;
  // the previous problem's largest host tables (tile layout of the banded
  // store), handed to the next problem so that refilling them touches no new
  // pages when the sizes repeat
  struct {
    trap::host_vec<trap::TileDesc> td;
    trap::host_vec<unsigned> qk, qk32, qb, qb32;
    trap::host_vec<int> tofs;
  } host_spare;
  trap::Precomp pre;
  trap::Work wk;
  trap::Prof prof;
  trap::GmresRun* run = nullptr;    // state of the current GMRES solve
  int path = 0;                     // TRAP_PATH_* of trap.h
  int prd_mode = 0;                 // TRAP_PRD_* of trap.h, applied at trap_set_problem
  int formal_scheme = 0;            // TRAP_FORMAL_* of trap.h
  int interp = 0;                   // TRAP_INTERP_* of trap.h: the frame transforms of Sigma
  int flat_field = 0;               // nonzero while the FP64 apply of the normalisation runs: its
                                    // field is W_T in Stokes I at every direction and frequency
  int interp_lin = 0;               // nonzero while an inner (linearised) Krylov apply runs:
                                    // its transforms are the spline whatever `interp` says
  // while set: BESSER formal solutions in this precision are linearised about
  // this reference emissivity (device vector of the full layout)
  const void* besser_ref = nullptr;
  int besser_ref_prec = -1;
  int max_lds = 64 * 1024;          // device limit of LDS bytes per block
  int n_cu = 256;                   // compute units of the device
  // the preconditioner tables are built on a stream of the library's own
  // (default priority), forked after the propagation matrix of the precompute
  // and joined back before the context's later work
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool fork_recorded = false;
  std::vector<trap::DevBuf> bufs;   // every allocation of the current problem
  std::vector<trap::DevBuf> spare;  // the previous problem's allocations, reused by size
};

namespace trap {
// allocation helper (records into ctx->bufs)
int dalloc(trap_ctx* ctx, void** p, size_t bytes);
void free_all(trap_ctx* ctx);        // current allocations become spares (older spares are freed)
void release_spare(trap_ctx* ctx);

template <typename T>
int dalloc_t(trap_ctx* ctx, T** p, size_t count) {
  return dalloc(ctx, reinterpret_cast<void**>(p), count * sizeof(T));
}
// Host -> device copy of `bytes` from pageable host memory through a pinned
// staging buffer of the device's pool (sigma.hip): returns once the data is in
// the staging buffer; the copy itself is enqueued on the context's stream.
int stage_upload(trap_ctx* ctx, const void* host, size_t bytes, void* dev);
struct UploadBatch;
// the same for every item of a batch, gathered into one staging buffer at the
// batch's offsets and copied to dev with one transfer
int stage_upload_batch(trap_ctx* ctx, const UploadBatch& up, void* dev);

// Many host arrays uploaded as one device allocation (256-byte aligned items,
// at least 16 bytes each) with one staged copy.
struct UploadBatch {
  struct Item {
    void** dst;
    const void* src;
    size_t bytes, off;
  };
  std::vector<Item> items;
  size_t total = 0;
  void add(void** dst, const void* src, size_t bytes) {
    const size_t off = (total + 255) & ~size_t(255);
    items.push_back(Item{dst, src, bytes, off});
    total = off + (bytes ? bytes : 16);
  }
  template <typename T, typename A>
  void add(T** dst, const std::vector<T, A>& v) {
    add(reinterpret_cast<void**>(dst), v.data(), v.size() * sizeof(T));
  }
  int commit(trap_ctx* ctx);
};

// Gauss-Legendre nodes and weights on [0, 1] (host_setup.cpp)
void gauss_legendre_unit(int n, std::vector<double>& t, std::vector<double>& w);

// Value at xs of the not-a-knot spline through v on the nodes x (second
// derivatives sd from the spline's second-derivative map), extended flat
// beyond the end nodes.
__device__ inline double spline_at(const double* __restrict__ x, int nn, const double* v, const double* sd,
                                   double xs) {
  if (xs <= x[0]) return v[0];
  if (xs >= x[nn - 1]) return v[nn - 1];
  int lo = 0, hi = nn - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= xs) lo = mid; else hi = mid;
  }
  const double h = x[lo + 1] - x[lo];
  const double t = (xs - x[lo]) / h, u = 1.0 - t;
  const double cs = h * h / 6.0;
  return u * v[lo] + t * v[lo + 1] + cs * (u * u * u - u) * sd[lo] + cs * (t * t * t - t) * sd[lo + 1];
}

// host setup (host_setup.cpp)
int build_problem(trap_ctx* ctx, const trap_atom_desc* atom, const trap_problem_desc* pd);
// the banded layout of the kernel store for the loaded grids (fills the band
// fields of P from P.x, P.lam, P.theta / P.theta_rows, P.nt, P.ldm, the slot
// counts and the spline's second-derivative map sig [nn][nn])
void kernel_bands(Problem& P, const std::vector<double>& sig);
// the store's device view of a context (after trap_set_problem and the precompute)
// the store as the contraction kernels see it; fp32: with the FP32 windows
KStore kernel_store(const trap_ctx* ctx, bool fp32);
// stored real kernel entries of heights [z0, z0 + zc) and their algorithmic
// contraction flops (sigma.hip)
double chunk_entries(const Problem& P, int z0, int zc);
double chunk_flops(const Problem& P, int z0, int zc);
double chunk_entries32(const Problem& P, int z0, int zc);
double chunk_flops32(const Problem& P, int z0, int zc);
size_t estimate_bytes(const trap_atom_desc* atom, const trap_problem_desc* pd, int store_mask,
                      int* err);

// precompute (precompute.hip) and the layout of its scratch (host_setup.cpp):
// factor tables on uniform grids reaching ntail virtual intervals past the grid
// ends, and the height chunk zc_tab of the row scratch
struct PrecompLayout {
  bool uniform = false;
  double h = 0.0;
  int ntail = 0, nd2 = 0, zc_tab = 1;
  size_t bytes = 0;     // device scratch: tables and the row stores of one chunk
};
PrecompLayout precomp_layout(int nz, int nn, int ldm, int nt, int nthr, bool aa, const double* x,
                             const double* lam);
int run_precompute(trap_ctx* ctx, int store_mask);
// the device Faddeeva function at n host points (precompute.hip)
int faddeeva_eval(int device, const double* v, const double* a, int n, double* out);

// applies (sigma.hip, formal.hip)
// (normalize != 0: the App. E factor on the line part and, with a continuum,
// its coherent scattering; sigma_apply_line is the line part alone)
int sigma_apply(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal, int normalize);
int sigma_apply_line(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal, int normalize);
int formal_apply(trap_ctx* ctx, const void* eps, void* I, int with_boundary, int prec);
int operator_apply(trap_ctx* ctx, const void* x, void* y, int prec);
int ensure_work(trap_ctx* ctx, int prec);

// solver (solver.hip)
int gmres_solve(trap_ctx* ctx, const trap_solve_opts* opts, double* I, trap_solve_stats* st);
int gmres_begin(trap_ctx* ctx, const trap_solve_opts* opts, double* I);
int gmres_step_batch(trap_ctx** ctxs, int n, int* status);
int gmres_end(trap_ctx* ctx, trap_solve_stats* st);
void gmres_release(trap_ctx* ctx);

// ---------------------------------------------------------------- grouped launches
// Arguments of one context in a launch that covers several contexts (one
// record per context, in device memory; blocks [off[r], off[r + 1]) are
// context r's).
struct GSpline {
  int nz0, nd, nn;
  const double *x, *SigT, *lam, *ub;
  double ub_sign;
  const double* sll;
  int ncls, cls;
  const float* in;
  long long in_z_stride, in_o_stride;
  float* out;
  int accumulate;
  const double *f, *epsth;
};
struct GR3Y {
  int z0, nzc, nt, nd, nn;
  const double2* r3;
  const float* Ibar;
  double2* Y;
};
struct GR3X {
  int z0, nu, nl, nd;
  const double* w;
  const double2* A;
  const double2* Y;
  double2* X;
};
struct GContract {
  int z0, nth, nt, nn, nd, n8, nslot, zc;
  KStore ks;
  const float* Ibar;
  const int* cgrp;
  const int* slot_dir;
  float* W;
};
struct GAngular {
  int z0, nd, nn, nu, nl, nslot, nbx;
  const int *pair_slot, *pair_index;
  const float* cf;
  const float* W;
  double c_sc;
  const double2 *E, *bma, *X, *prof;
  float* Eb;
};
struct GFormal {
  int nz, nd, nn, scheme;
  const double *mu, *tau, *K8, *WT;
  const float* eps;
  float* I;
};
// preconditioner stages of a shared apply (precond.hip, formal.hip)
struct GPcCls {
  int nd, nn, ncmax, stride;
  const double *x, *SigT, *lam, *w;
  const int *mem, *moff, *ncls;
  const double *cub, *src;
  double* gc;
};
// LDS of the preconditioner's gather kernels (per block): the vector, its
// spline second derivatives, four rows of partial sums and a copy of the
// frequency grid (the spline evaluations search it there).
constexpr size_t pc_gather_lds(int nn) { return (size_t)7 * nn * sizeof(double); }
struct GPcFin {
  int nn, ncmax;
  const double* SigT;
  const int* ncls;
  const double *gc, *Mat;
  double* h;
};
struct GPcScat {
  int mode, nz, nd, nn, src_stride, dst_stride;
  const double *x, *lam, *ub, *h, *L, *src, *xin, *res;
  double* dst;
};
struct GPcSweep {
  int nz, nd, nn, y_stride;
  const double* mu;
  const double2* F;
  const double *L, *e, *y, *x;
  double* res;
};
// stage 0: class sums, 1: per-height finish, 2: per-point scatter
int launch_pc_grouped(hipStream_t s, int stage, const void* args, const int* off, int n, int blocks, size_t lds);
int launch_pc_sweep_grouped(hipStream_t s, const GPcSweep* args, const int* off, int n, int blocks);
int precond_ensure(trap_ctx* ctx);     // the sweep buffers of a context
struct GVec {              // FP64 <-> FP32 conversions around the FP32 operator
  long long N;
  int nb;
  const double* x64;       // in: operand
  float* x32;              // operand in FP32
  const float* f32;        // Lambda Sigma x in FP32
  double* y64;             // out: x - Lambda Sigma x
};

// Per-device state shared by the contexts of a device: for grouped launches a
// stream, a pinned staging buffer and its device copy for the argument records,
// and events; pinned buffers for host-to-device uploads.  Created with the
// first context on a device and released with the last (freeing pinned
// memory waits for the device, so it is not done per context).
struct StagingBuf {
  void* host = nullptr;       // pinned
  size_t cap = 0;
  hipEvent_t ev = nullptr;    // recorded after the copy out of the buffer
  bool used = false;
};
struct BatchArena {
  hipStream_t stream = nullptr;
  unsigned char* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  hipEvent_t copied = nullptr, done = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<StagingBuf> staging;   // pinned buffers of stage_upload
  int users = 0;
};
void batch_arena_acquire(int device);
// true when the device's last context released it
bool batch_arena_release(int device);
// return the device pool's unused memory to the device (no context left on it)
void device_pool_trim(int device);
// 1 when the context's FP32 operator can join a grouped apply (W allocated
// for all heights at once), 0 when it cannot, < 0 on error
int sigma_batch_ready(trap_ctx* ctx);
// y_i = x_i - Lambda Sigma x_i in FP32 for every context (operands FP64), on
// the device's batch stream, ordered after and before each context's stream
// pc[i] > 0: apply context i's preconditioner with pc[i] block-Jacobi steps to
// y_i in place (shared launches as well); pc may be null
int op_apply_batch_f32(trap_ctx** ctxs, int n, const double* const* x, double* const* y, const int* pc = nullptr);
int launch_formal_grouped(hipStream_t s, const GFormal* args, const int* off, int n, int blocks);

// physics-based preconditioner (Sect. 5.2, App. F): tables after the kernel
// precompute (precompute.hip); out = M r for FP64 vectors, `sweeps`
// block-Jacobi steps, the scalar formal solution in precision prec
// (precond.hip; out may equal r)
int run_precompute_precond(trap_ctx* ctx);
int precond_apply(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec);
// the same apply with its scratch in a fixed device array (no allocation):
// kNoAllocScratchBytes per device, shared by every call on that device
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
size_t precond_noalloc_bytes(const Problem& P, int ncmax);
int precond_apply_noalloc(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec);
// local Lambda and step coefficients of the scalar formal solution, and the
// sweep of Lambda* with the fused residual res = y - x + Lambda* e
// (formal.hip; the sweep's arithmetic is FP64 whatever prec)
int launch_pc_local_lambda(trap_ctx* ctx);
int launch_formal_scalar(trap_ctx* ctx, int prec, const double* e, const double* y, int y_stride,
                         const double* x, double* res);

// HIP calls whose failure cannot change what the caller gets (releases,
// synchronisations in teardown, profiling events) go through note_hip: a
// failure is recorded with the call's text and the place (trap_hip_notes
// reads the count and the latest record) and the thread's last-error slot is
// cleared, so it cannot reappear as the error of a later launch check.
void note_hip(const char* what, const char* where, hipError_t e);
#define TRAP_NOTE(call) ::trap::note_hip(#call, __func__, (call))

// Every entry point holds one.  A HIP error already pending in the thread's
// last-error slot when the entry point starts (left by a call outside the
// library, or by a library call that did not check it) is recorded with the
// entry point's name (trap_hip_notes) and cleared, so that the launch checks
// inside (hipGetLastError after each launch) report this call's own errors.
struct DeviceGuard {
  int prev = -1;
  DeviceGuard(int dev, const char* entry) {
    const hipError_t stale = hipGetLastError();
    if (stale != hipSuccess) note_hip("error pending at entry", entry, stale);
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) TRAP_NOTE(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) TRAP_NOTE(hipSetDevice(prev));
  }
};

inline int ceil_div(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

// profiling: returns a record index (or -1 when profiling is off)
int prof_begin(trap_ctx* ctx, int stage, double flops = 0.0, double bytes = 0.0);
void prof_end(trap_ctx* ctx, int idx);

}  // namespace trap
