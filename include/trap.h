/*
 * trap.h -- C ABI of the MI355X (gfx950) library for the linearised polarised
 * PRD transfer problem of Riva et al., "A numerical approach for modelling the
 * polarisation signals of strong resonance lines with partial frequency
 * redistribution".
 *
 * The problem is the linear system (Sect. 2.7, Eq. linear_system)
 *     (Id - Lambda Sigma) I = Lambda eps_th + t,
 * with Sigma the scattering operator (Eq. eps_sc_l with R = R_II + R_III,
 * Eqs. RQIIKKp, G and RIIIQKKp, evaluated in the comoving frame of Sect. 4.1
 * through the intermediate W of App. D, normalised as in App. E) and Lambda the
 * formal solution (Sect. 3, ray sweeps: DELO-linear, DELOPAR or BESSER).  It
 * is solved by mixed-precision GMRES (Sect. 5.1), optionally with the
 * physics-based preconditioner of Sect. 5.2 and App. F, or by alternating
 * Anderson-Richardson iteration (the only choice with BESSER).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vector layout: a Stokes field or emissivity is a contiguous device array
 *   V[z][o][n][s]  (n_z x n_dir x n_nu x 4), z = height index from the bottom
 *   (z_min) to the top, o = direction index mu-major (mu ascending from -1 to
 *   1, n_mu/2 Gauss-Legendre nodes per hemisphere, then any line-of-sight
 *   rings) and chi-minor (chi_k = 2 pi k / n_chi), n = frequency node,
 *   s = Stokes (I, Q, U, V).
 *   Positive Q is parallel to the limb (perpendicular to the vertical plane
 *   containing the ray); (e_Q, e_perp, Omega) is right-handed; the V sign makes
 *   eta_V = (phi_r - phi_b) cos(theta_B)/2.
 *   Emissivities are per unit reduced frequency and per unit frequency-
 *   integrated absorption coefficient (eps * dnu_D / k); only eps/eta_I enters.
 * Precision codes: TRAP_FP64 vectors are double, TRAP_FP32 vectors are float.
 * Ownership: device pointers passed in are owned by the caller and must stay
 *   valid until the work enqueued on the context's stream has completed.  Host
 *   descriptor arrays are read during the call only.  The context owns every
 *   allocation it makes and frees it in trap_destroy.
 * Streams: work is enqueued on the stream given to trap_create (a hipStream_t,
 *   NULL = default stream).  trap_set_problem (after its host work),
 *   trap_precompute, trap_apply_sigma, trap_formal_solve, trap_apply_operator,
 *   trap_formal_from_field and trap_gmres_begin are asynchronous;
 *   trap_gmres_solve, trap_gmres_end, trap_aar_solve, trap_emergent and
 *   trap_emergent_los synchronise the stream.
 * Errors: every call returns a trap_status; negative values are failures and
 *   trap_last_error() returns a thread-local message.  A failed call leaves the
 *   context usable.  No call aborts or throws.
 */
#ifndef TRAP_H
#define TRAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct trap_ctx trap_ctx;

typedef enum {
  TRAP_OK = 0,
  TRAP_EINVAL = -1,   /* bad argument or problem description */
  TRAP_ENOMEM = -2,   /* device allocation failed or memory budget exceeded */
  TRAP_EDEVICE = -3,  /* HIP runtime error */
  TRAP_ENOCONV = -4,  /* iteration did not reach the tolerance */
  TRAP_ESTATE = -5,   /* calls out of order (e.g. apply before precompute) */
  TRAP_ENAN = -6      /* non-finite value detected */
} trap_status;

typedef enum { TRAP_FP64 = 0, TRAP_FP32 = 1 } trap_prec;

/* Atomic model (Sect. 2.2; Table 1 for the two-term lines).
 * kind 0: two-level atom J_l -> J_u with Lande factors g_l, g_u.
 * kind 1: two-term atom (L_l, S) -> (L_u, S) in L-S coupling; the upper term is
 *   treated in the Paschen-Back regime with the fine-structure splitting
 *   E(J = L_u + S) - E(J = |L_u - S|) = fs_split_x reference Doppler widths,
 *   centred on the line frequency; the lower term has linear Zeeman splitting.
 * r_E = Gamma_E / (Gamma_R + Gamma_I), the elastic share of the damping. */
typedef struct {
  int kind;
  double lambda0_A;   /* line-centre wavelength, Angstrom */
  double mass_amu;    /* atomic mass */
  double J_l, J_u, g_l, g_u;
  int L_l, L_u;
  double S;
  double fs_split_x;
  double r_E;
} trap_atom_desc;

/* Grids and atmosphere (Sects. 2.5, 4.2, 6.1).  Host arrays, bottom to top.
 * x: frequency nodes in units of the reference Doppler width dnu_D(T_ref),
 *    x = (nu0 - nu)/dnu_D_ref, strictly increasing, bracketing 0, n_nu >= 4.
 * tau_line: vertical field-free line-centre optical depth, strictly decreasing,
 *    > 0.  T (K), xi (km/s), a (damping), eps (photon destruction), W_T (Wien
 *    function) have n_z entries; v is [n_z][3] km/s cartesian (z up); B is
 *    [n_z][3] = (|B| in G, theta_B, chi_B) in the atmospheric frame.
 * n_mu (even, >= 2) Gauss-Legendre mu nodes in total, n_chi >= 1 azimuths.
 * kappa_c, sigma_c (optional, NULL = none; either may be NULL alone):
 *    continuum true absorption and scattering coefficients (App. A),
 *    [n_z][n_nu], >= 0, in units of the height's field-free line-centre
 *    absorption coefficient.  They add kappa_c + sigma_c to the diagonal of
 *    the propagation matrix, kappa_c W_T to the thermal emissivity of Stokes I
 *    (LTE) and coherent dipole scattering sigma_c sum_j R_ij I_j (observer
 *    frame, R the Rayleigh phase matrix) to the normalised Sigma.
 * n_los, los_mu (optional, n_los = 0 / NULL = none; n_los <= 16): lines of
 *    sight off the quadrature, each mu in (0, 1] (the emergent profiles of
 *    Sect. 6 are shown at such mu values).  Each adds a ring of the n_chi
 *    azimuths after the n_mu * n_chi quadrature directions, with zero
 *    quadrature weight: the rays carry their own propagation matrix,
 *    emissivity and formal solution but take no part in the angular
 *    integrals, so the solution on the quadrature directions is the one
 *    without them.  Every device vector then holds
 *    n_dir = (n_mu + n_los) * n_chi directions. */
typedef struct {
  int n_z, n_nu, n_mu, n_chi;
  const double* x;
  const double* tau_line;
  const double* T;
  const double* xi;
  const double* a;
  const double* eps;
  const double* W_T;
  const double* v;
  const double* B;
  double T_ref;
  const double* kappa_c;
  const double* sigma_c;
  int n_los;
  const double* los_mu;
} trap_problem_desc;

/* Sizes of the discrete problem (filled by trap_get_info). */
typedef struct {
  int n_z, n_nu, n_dir, n_theta, n_slots, n_up, n_lo, n_trans;
  size_t n_unknowns;            /* 4 n_z n_dir n_nu */
  size_t bytes_kernel_fp64;     /* stored R_II kernels, FP64 */
  size_t bytes_kernel_fp32;     /* stored R_II kernels, FP32 */
  size_t bytes_device_total;    /* everything the context holds on the device */
  double flops_contraction;     /* algorithmic flops of one R_II contraction */
  double bytes_contraction_fp64;/* algorithmic HBM bytes of one contraction */
  double bytes_contraction_fp32;
  long long kernel_rows_mirrored; /* per height and scattering angle: complex kernel rows
                                     filled from the mirror image of a computed row
                                     (frequency grid symmetric about 0 and transition shifts
                                     in +-s pairs, as M_s[n][m] = conj(M_-s[N-1-n][N-1-m])) */
  long long kernel_entries;     /* complex kernel entries inside the rows' bands (Sect. 4.3):
                                   each row keeps the columns its redistribution function
                                   reaches (6.6 Gaussian widths 2 sin(Theta/2)) plus the reach
                                   of the spline basis (entries below 1e-13 of the row dropped);
                                   flops_contraction counts 16 per entry and incoming slot.
                                   The store holds 16-row tiles over the union of their rows'
                                   bands: bytes_kernel_fp32 / 4 real entries */
  int band_reach;               /* that reach, in frequency nodes */
  /* The FP32 operator steps through narrower column windows of the same
     stored tiles: knot intervals within 4.6 Gaussian widths and the reach
     where the spline map falls below 1e-9 (what it leaves out is below the
     FP32 sum's resolution).  Its complex entries, flops (16 per entry and
     incoming slot) and reach; bytes_contraction_fp32 counts the stored
     entries inside those windows. */
  double flops_contraction_fp32;
  long long kernel_entries_fp32;
  int band_reach_fp32;
} trap_info;

typedef struct {
  double tol;          /* stop when ||b - A x|| / ||b|| < tol (Sect. 5.1) */
  int restart;         /* GMRES restart length m (Arnoldi basis size) */
  int max_iters;       /* total inner iterations allowed */
  int max_outer;       /* iterative-refinement steps (mixed precision) */
  trap_prec inner;     /* precision of the inner operator (FP64 = plain GMRES) */
  double inner_tol;    /* relative reduction asked of each inner solve */
  int zero_guess;      /* nonzero: I holds zeros on entry, so the first residual is b
                          itself and its operator apply is skipped (TRAP_EINVAL at the
                          first step if I is not zero) */
  int precond_sweeps;  /* 0: no preconditioner; k in [1, 64]: left preconditioning with
                          k block-Jacobi steps on P (trap_apply_preconditioner; needs
                          trap_precompute_preconditioner).  The inner solves then stop on
                          the preconditioned residual, refined in FP64 as with an FP32
                          inner operator (also for FP64: up to max_outer steps) until
                          the true residual meets tol */
} trap_solve_opts;

typedef struct {
  int outer_steps;
  int inner_iters;
  int applies_fp64;
  int applies_fp32;
  int applies_grouped;    /* FP32 applies made in launches shared with other contexts */
  int applies_precond;    /* preconditioner applications */
  double final_rel_res;   /* FP64 true residual at exit */
  double ms_total;
} trap_solve_stats;

/* Create a context on HIP device `device` enqueuing on `stream` (hipStream_t). */
int trap_create(trap_ctx** out, int device, void* stream);
/* Free every device allocation of the context and the context itself. */
int trap_destroy(trap_ctx* ctx);

/* Load a problem: per-height physics on the host in FP64 (Doppler widths,
 * damping split, branching ratios alpha/beta of App. B, sublevel energies and
 * dipole vectors, angular tables, scattering-angle table of Sect. 4.2, cubic-
 * spline coefficient maps of Sect. 6.2), uploaded to the device with one copy
 * enqueued on the context's stream (the call returns once the host work is
 * done).  Replaces any previous problem of the context (waiting for the work
 * still queued on it); the previous problem's device allocations are kept and
 * reused by size for the new one, those left over are freed at the next
 * trap_set_problem or at trap_destroy (trap_get_info counts them). */
int trap_set_problem(trap_ctx* ctx, const trap_atom_desc* atom, const trap_problem_desc* prob);

/* Device-side precompute (Sect. 4.3, App. C-E): the propagation matrix and
 * thermal emissivity, the R_II kernels M[z][Theta][t] (FP64 Faddeeva, product
 * integration over frequency) stored in FP64 and/or FP32, the R_III weights,
 * the normalisation factor f (one Sigma apply on a flat field) and the right-
 * hand side b = Lambda eps_th + t.  store_mask: bit 0 = FP64 kernels, bit 1 =
 * FP32 kernels (FP64 is always built for f and b).  Asynchronous: the work is
 * enqueued on the context's stream, and later calls on the context are
 * ordered after it. */
int trap_precompute(trap_ctx* ctx, int store_mask);

/* Physics-based preconditioner (Sect. 5.2) with the block-diagonal local
 * inverse of App. F.  P = Id - Lambda* Sigma* in the unmagnetised,
 * unpolarised, angle-averaged setting, multipole K = Q = 0: Sigma* maps Stokes
 * I to a Stokes-I emissivity through the comoving interpolation per
 * direction, the angular mean, a comoving frequency coupling Phi_z (N_nu x
 * N_nu, zero-field R_II averaged over Theta with 25 Gauss-Legendre nodes, plus
 * R_III) and the interpolation back; Lambda* is the DELO-linear solution of
 * Stokes I with the problem's eta_I and no polarisation terms.  P is the
 * identity on Q, U, V.
 * trap_precompute_preconditioner builds, after trap_precompute, per height
 * Phi_z, the local Lambda (the diagonal of Lambda* at the height) and
 * C_z = Phi_z (Id - A_z)^-1 with A_z of App. F (FP64, Gauss-Jordan with
 * partial pivoting; a singular Id - A_z gives non-finite tables, which a
 * solve reports as TRAP_ENAN).  Asynchronous; once per problem (later calls
 * return at once).  Device memory: about 5 n_z N_nu^2 + 4 n_z n_dir N_nu
 * doubles plus the kernel scratch (trap_footprint with store_mask bit 2).
 * trap_apply_preconditioner: out = M r for FP64 device vectors
 * [z][Omega][n][4] (out may equal r): x_1 = P^^-1 r_I,
 * x_{k+1} = x_k + P^^-1 (r_I - P x_k), `sweeps` in [1, 64] steps, then
 * out_I = x_sweeps and out_{Q,U,V} = r_{Q,U,V}.  The scalar formal solutions
 * inside run in `prec`, the rest in FP64.  Asynchronous.
 * trap_preconditioner_tables copies Phi [n_z][N_nu][N_nu], C [n_z][N_nu][N_nu]
 * and the local Lambda [n_z][n_dir][N_nu] to host arrays (any may be NULL);
 * synchronises. */
int trap_precompute_preconditioner(trap_ctx* ctx);
int trap_apply_preconditioner(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec);
int trap_preconditioner_tables(trap_ctx* ctx, double* phi, double* c, double* lloc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the apply of
 * trap_apply_preconditioner (same arguments, same kernels, same result) with
 * its scratch vectors (the iterate, Sigma* x, the residual and the per-height
 * comoving vectors, about 3 n_z n_dir N_nu + (2 + classes) n_z N_nu doubles)
 * taken from a fixed 128 MiB device array instead of context allocations.  It
 * calls no hipMalloc, hipFree or other allocating routine; the caller passes
 * r and out as for trap_apply_preconditioner.  Each device the library runs
 * on holds its own copy of the array until the process ends (its address is
 * looked up at the first call on the device).  Every call on a device shares
 * that device's array and leaves its contents behind (each apply writes every
 * value it reads, so no clearing is needed): calls that overlap on one device
 * (other streams, other host threads) race and must be serialised by the
 * caller.  TRAP_ENOMEM, with the sizes in the message, for a problem whose
 * scratch exceeds the array; otherwise the errors of
 * trap_apply_preconditioner.  Asynchronous on the context's stream. */
int trap_apply_preconditioner_noalloc(trap_ctx* ctx, const double* r, double* out, int sweeps, int prec);

/* eps = Sigma I (Eq. matrix_form_2 without eps_th): comoving interpolation,
 * R_II contraction with the stored kernels, angular/sublevel sum, R_III,
 * back-interpolation and the factor f on Stokes I.  If add_thermal != 0 the
 * thermal emissivity eps_th is added.  I and eps are device arrays in `prec`. */
int trap_apply_sigma(trap_ctx* ctx, const void* I, void* eps, int prec, int add_thermal);

/* I = Lambda eps (+ t if with_boundary): ray sweeps with the context's formal
 * scheme (Sect. 3; trap_set_formal_scheme). */
int trap_formal_solve(trap_ctx* ctx, const void* eps, void* I, int with_boundary, int prec);

/* Formal solver of Lambda (Sect. 3).  TRAP_FORMAL_DELO_LINEAR (default): S and
 * K'I linear between the upwind and current points.  TRAP_FORMAL_DELOPAR: S
 * integrated with the parabola through the upwind, current and downwind
 * points (weights from the moments int_0^m t^k e^{-t} dt, FP64), K'I linear.
 * TRAP_FORMAL_BESSER: S a quadratic Bezier curve between the upwind and
 * current points whose control point follows the tangent at the current point
 * of the parabola through the three points (slope zero at a local extremum)
 * and is kept inside the range of the two end values, per Stokes component;
 * K'I linear.  The range limit makes Lambda slightly nonlinear (Sect. 6.2), so
 * a BESSER problem is solved by trap_aar_solve (GMRES returns TRAP_EINVAL).
 * In both three-point schemes a ray's last point takes the DELO-linear step.
 * Applies to trap_formal_solve, the operator, the right-hand side and
 * trap_formal_from_field, so it is set before trap_precompute (TRAP_ESTATE
 * when changed after it for the loaded problem; a new problem frees it
 * again).  The preconditioner's scalar sweep stays DELO-linear. */
enum { TRAP_FORMAL_DELO_LINEAR = 0, TRAP_FORMAL_DELOPAR = 1, TRAP_FORMAL_BESSER = 2 };
int trap_set_formal_scheme(trap_ctx* ctx, int scheme);

/* Interpolant of the frequency transforms between the observer and the
 * comoving frame (Sect. 4.1: the comoving field Ibar(u) = I(u - u_b) before
 * the scattering integral and the emissivity back to the observer frame
 * after it).  TRAP_INTERP_SPLINE (default): the not-a-knot cubic spline of
 * Sect. 6.2, flat beyond the grid ends.  TRAP_INTERP_WENO4: the
 * non-oscillatory interpolation that Sect. 4.1 names as the remedy for
 * oscillating profiles under strong velocities, read as a fourth-order
 * weighted essentially non-oscillatory scheme: on [x_i, x_{i+1}] the two
 * quadratics through {x_{i-1}, x_i, x_{i+1}} and {x_i, x_{i+1}, x_{i+2}},
 * q_k = v_i + d (u - x_i) + D_k (u - x_i)(u - x_{i+1}) (d, D_k the first and
 * second divided differences), are blended with weights a_k / (a_1 + a_2),
 * a_k = g_k / (e + (h_i^2 D_k)^2)^2, g_1 = (x_{i+2} - u) / (x_{i+2} - x_{i-1}),
 * g_2 = 1 - g_1, e = 1e-12 times the mean square of the four values plus
 * 1e-150; the first and last intervals take their one quadratic; flat beyond
 * the ends; per Stokes component, in FP64.  The kernel rows keep the spline
 * basis.  The blend depends on the data, so Sigma is then nonlinear: it is
 * used by trap_apply_sigma, trap_apply_operator, the normalisation factor f,
 * every FP64 residual of trap_gmres_solve / trap_gmres_begin and every
 * evaluation of G in trap_aar_solve, while the inner Krylov and
 * defect-correction applies (which need a linear operator) keep the spline,
 * so the outer refinement converges to the nonlinear fixed point when the two
 * transforms are close; where they are not (shifts of several grid steps on a
 * coarse grid) trap_aar_solve with inner = TRAP_FP64 iterates G itself.  Set
 * before trap_precompute (TRAP_ESTATE when changed after it for the loaded
 * problem; a new problem frees it again); TRAP_EINVAL for an unknown mode. */
enum { TRAP_INTERP_SPLINE = 0, TRAP_INTERP_WENO4 = 1 };
int trap_set_interpolation(trap_ctx* ctx, int mode);

/* y = (Id - Lambda Sigma) x, the operator of Eq. linear_system (with BESSER,
 * whose Lambda is not linear, x - Lambda(Sigma x) evaluated as written). */
int trap_apply_operator(trap_ctx* ctx, const void* x, void* y, int prec);

/* Copy b = Lambda eps_th + t (FP64, computed by trap_precompute) into b_out. */
int trap_rhs(trap_ctx* ctx, double* b_out_device);

/* Solve Eq. linear_system by restarted GMRES (Sect. 5.1).  With opts->inner =
 * TRAP_FP64 this is plain FP64 GMRES; with TRAP_FP32 the Krylov solves use the
 * FP32 operator while the Arnoldi vectors, the residual and the iterative-
 * refinement updates are FP64.  I is FP64 device memory: initial guess in,
 * solution out.  Returns TRAP_ENOCONV if tol is not reached.  Synchronises. */
int trap_gmres_solve(trap_ctx* ctx, const trap_solve_opts* opts, double* I, trap_solve_stats* stats);

/* Options of the alternating Anderson-Richardson iteration (Sect. 5.1; the
 * method of the AAR paper the text cites). */
typedef struct {
  double tol;          /* stop when ||G(I) - I|| / ||G(0)|| < tol, G(I) = Lambda (Sigma I + eps_th) + t */
  int max_iters;       /* residual evaluations allowed */
  int depth;           /* Anderson history: the last `depth` differences, 0..16 (0 = Richardson) */
  int period;          /* every period-th step is an Anderson step, >= 1 */
  double omega;        /* Richardson relaxation, > 0 */
  double beta;         /* Anderson relaxation, > 0 */
  int zero_guess;      /* nonzero: I is set to zero first (its first G is the right-hand side) */
  int precond_sweeps;  /* 0, or k in [1, 64]: f = M r with k block-Jacobi steps of the
                          physics-based preconditioner (needs
                          trap_precompute_preconditioner; its scalar sweeps in the
                          precision of the iteration they serve) */
  trap_prec inner;     /* TRAP_FP64: the iteration above on G in FP64.  TRAP_FP32: defect
                          correction, each step the FP64 residual r = G(I) - I, then the
                          iteration above on d = r + Lambda Sigma d with the FP32 operator
                          (for BESSER its Jacobian at I: each point's branch follows the
                          source of I), to max(inner_tol ||r||, tol ||G(0)|| / 2), and
                          I <- I + d, at most max_outer times */
  double inner_tol;    /* 0 < inner_tol < 1 (TRAP_FP32 only) */
  int max_outer;       /* >= 1 (TRAP_FP32 only) */
} trap_aar_opts;

/* Solve I = G(I) = Lambda (Sigma I + eps_th) + t, the fixed-point form of
 * Eq. linear_system, by alternating Anderson-Richardson iteration, all in FP64
 * on the device: with r = G(I) - I and f = M r (M the identity or the
 * preconditioner), each step is I <- I + omega f, except every period-th,
 * which is I <- I + beta f - (X + beta F) gamma with gamma the least-squares
 * coefficients of f on the last `depth` differences F of f (X those of I;
 * normal equations solved on the host).  It needs no linearity of Lambda, so
 * it also solves BESSER problems.  I is FP64 device memory: initial guess in,
 * solution out.  stats: outer_steps = Anderson steps, inner_iters = residuals
 * of the iteration, applies_fp64 / applies_fp32 = evaluations of G (FP64) and
 * of the FP32 operator.  The (8 + 2 depth) FP64 work vectors are allocated at
 * the first call with that depth (not counted by trap_footprint).
 * Returns TRAP_ENOCONV if tol is not reached.  Synchronises. */
int trap_aar_solve(trap_ctx* ctx, const trap_aar_opts* opts, double* I, trap_solve_stats* stats);

/* Batched solving for a serving loop: the solve of trap_gmres_solve split into
 * steps so that many contexts (requests) advance together.
 * trap_gmres_begin checks the options and enqueues the check of the initial
 * guess I (FP64 device memory, overwritten with the solution; must stay valid
 * until the solve ends) and the computation of ||b||; it does not wait.  A
 * non-finite initial guess (TRAP_ENAN) or a zero right-hand side
 * (TRAP_EINVAL) ends the solve at its first step.
 * trap_gmres_step_batch advances each of the n distinct contexts by one unit
 * (one Arnoldi iteration, or one FP64 residual of the refinement loop): the
 * device work of all contexts is enqueued on their own streams before the call
 * waits, so work of different contexts overlaps on the device, and the host
 * synchronises at most twice per step for the whole batch.  status[i] is 1
 * while context i is running, then its final trap_status.  Finished contexts
 * may stay in the batch (they are skipped).
 * trap_gmres_end returns the final status and statistics of a finished solve
 * (TRAP_ESTATE while it is still running).
 * Contexts of one device whose step applies the FP32 operator, that do not
 * record stage times and whose Sigma runs in one height chunk share the
 * launches of that apply (a context with several chunks applies on its own
 * stream, so it does not hold the shared applies of smaller ones): each
 * stage of the operator is one launch over all of them, on a stream the
 * library keeps per device (ordered after each context's earlier work and
 * before its later work through events).
 * The arithmetic of a context does not depend on the other contexts of the
 * batch: each block of a shared launch runs the single-context code on one
 * context's data, so a request's solution is the same alone and in any mix. */
int trap_gmres_begin(trap_ctx* ctx, const trap_solve_opts* opts, double* I);
int trap_gmres_step_batch(trap_ctx** ctxs, int n, int* status);
int trap_gmres_end(trap_ctx* ctx, trap_solve_stats* stats);

/* Emergent Stokes vectors at z_max for the mu > 0 quadrature directions:
 * host_out[o_up][n][4] (FP64, n_mu/2 * n_chi x n_nu x 4).  Synchronises. */
int trap_emergent(trap_ctx* ctx, const double* I, double* host_out);

/* The formal solution of a given radiation field's emissivity (FP64):
 * out = Lambda (Sigma I + eps_th) + t on every ray, as in the iteration of
 * Eq. linear_system; for a converged solution this is the extra formal
 * solution that gives the emergent profiles along the off-grid lines of
 * sight (Sect. 6).  I is FP64 device memory holding n_dir_in directions per
 * height: either all n_dir, or only the n_mu * n_chi quadrature directions
 * (the solution of a context of the same problem without lines of sight;
 * the line-of-sight rings carry zero weight, so they are read as zero).
 * out is FP64 device memory of the full layout (n_dir directions); it may
 * not overlap I.  TRAP_EINVAL for another n_dir_in, TRAP_ESTATE before
 * trap_precompute.  Asynchronous on the context's stream. */
int trap_formal_from_field(trap_ctx* ctx, const double* I, int n_dir_in, double* out);

/* Emergent Stokes vectors at z_max along the lines of sight:
 * host_out[los][chi][n][4] (FP64, n_los x n_chi x n_nu x 4) read from the
 * full-layout FP64 device vector I (a solution of the problem with its
 * rings, or the output of trap_formal_from_field).  TRAP_EINVAL when the
 * problem has no lines of sight.  Synchronises. */
int trap_emergent_los(trap_ctx* ctx, const double* I, double* host_out);

/* Sizes and algorithmic work of the loaded problem. */
int trap_get_info(const trap_ctx* ctx, trap_info* info);

/* Device bytes a context needs for this problem with the given kernel store
 * mask (for admission control): every allocation of trap_set_problem,
 * trap_precompute (including its scratch) and a solve with restart <= 40,
 * in the angle-dependent layout; with store_mask bit 2 also those of
 * trap_precompute_preconditioner and of preconditioned solves.  Host arithmetic only; does not touch the
 * device. */
int trap_footprint(const trap_atom_desc* atom, const trap_problem_desc* prob, int store_mask,
                   size_t* bytes);

/* Diagnostics of the stored kernels and of the device Faddeeva function.
 * trap_kernel_rows copies the FP64 R_II kernel M[z][theta][t] (Sect. 4.3; rows
 * n, columns m of the comoving spline basis, real plane then imaginary plane,
 * zero outside each row's stored band) to host_out [2][n_nu][n_nu], with the
 * scattering angle (radians; for the angle-averaged mode theta = 0 names the
 * averaged kernel) and the transition's reduced shift s_t (u units) of that
 * height; TRAP_ESTATE before trap_precompute, TRAP_EINVAL for indices out of
 * range.  Synchronises.
 * trap_faddeeva evaluates the library's device Faddeeva function
 * W(a, v) = w(v + i a) (Sect. 2.4; Weideman's rational expansion, a continued
 * fraction far out) at n points (v[i], a[i]), a >= 0, into out [n][2] (real,
 * imaginary); host arrays; allocates and frees device scratch; synchronises
 * the device. */
int trap_kernel_rows(trap_ctx* ctx, int z, int theta, int t, double* theta_out, double* shift_out,
                     double* host_out);
int trap_faddeeva(int device, const double* v, const double* a, int n, double* out);

/* Per-stage device timing.  trap_profile(ctx, 1) starts recording HIP events
 * around every kernel launch of the listed stages on the context's stream
 * (and clears earlier records); trap_profile(ctx, 0) stops.  trap_stage_times
 * synchronises the stream and returns, per stage, the summed elapsed device
 * milliseconds and the launch count since recording started, plus the
 * algorithmic flops of the R_II contraction launches recorded (16 per complex
 * kernel entry per incoming-direction slot). */
enum { TRAP_STAGE_COMOVING = 0, TRAP_STAGE_CONTRACT = 1, TRAP_STAGE_R3 = 2, TRAP_STAGE_ANGULAR = 3,
       TRAP_STAGE_BACKINTERP = 4, TRAP_STAGE_FORMAL = 5, TRAP_STAGE_KERNEL_ROWS = 6,
       TRAP_STAGE_CONTRACT_FP64 = 7, TRAP_STAGE_COUNT = 8 };
/* TRAP_STAGE_CONTRACT counts FP32 contraction launches, TRAP_STAGE_CONTRACT_FP64
 * the FP64 ones; flops/bytes are kept per precision (index 0 FP32, 1 FP64). */
typedef struct {
  double ms[TRAP_STAGE_COUNT];
  int launches[TRAP_STAGE_COUNT];
  double flops_contraction[2];
  double bytes_contraction[2];  /* algorithmic bytes of the recorded contraction launches */
} trap_stage_stats;
int trap_profile(trap_ctx* ctx, int enable);
int trap_stage_times(trap_ctx* ctx, trap_stage_stats* out);

/* Angle-dependent (default) or angle-averaged partial frequency redistribution
 * for R_II (Sect. 5.2, Eq. R_AA): in the AA mode every pair of directions uses
 * the kernel (1/2) int_0^pi sin(Theta) M(Theta) dTheta, evaluated with the
 * 25-node Gauss-Legendre rule in Theta of App. C.  The mode takes effect at
 * the next trap_set_problem.  trap_footprint sizes the AD layout, which bounds
 * the AA one from above for Theta tables of 25 angles or more. */
enum { TRAP_PRD_AD = 0, TRAP_PRD_AA = 1 };
int trap_set_prd_mode(trap_ctx* ctx, int mode);

/* Choice of Sigma implementation (both compute the same operator):
 * TRAP_PATH_AUTO (default) and TRAP_PATH_CHUNKED materialise the R_II
 * intermediate W per chunk of heights (contraction, then angular sum).
 * TRAP_PATH_FUSED uses one kernel that keeps W on chip and scatters the angular
 * sum into LDS; it handles FP32 applies of problems within its limits (padded
 * frequency count <= 128, 2..8 upper sublevels, LDS within the device's
 * per-block limit) and makes other applies fail with TRAP_EINVAL. */
enum { TRAP_PATH_AUTO = 0, TRAP_PATH_FUSED = 1, TRAP_PATH_CHUNKED = 2 };
int trap_set_path(trap_ctx* ctx, int path);

/* Thread-local description of the last failure. */
const char* trap_last_error(void);

/* HIP failures the library noticed outside any failing call's own return:
 * teardown and bookkeeping calls whose failure changes nothing the caller
 * gets (releases, synchronisations in trap_destroy, profiling events), and a
 * HIP error already pending in the thread when an entry point starts (left
 * by an earlier call of the caller's or of a runtime component).  Each is
 * recorded with the call (or "error pending at entry") and the function or
 * entry point, and cleared so that it cannot surface as a later launch's
 * error.  *count receives the number recorded in the process; buf (n bytes)
 * the latest record, NUL-terminated.  Either may be NULL. */
int trap_hip_notes(long long* count, char* buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* TRAP_H */
