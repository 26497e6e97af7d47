"""Sigma, Lambda and the linear solve (oracle, FP64).

Vector layout: I[z][Omega][n][s], z slowest, Stokes s fastest (Sect. 2.6,
lexicographic ordering; Sigma is block-diagonal in z).

Per-height physics (Sects. 2.3, 6.1):
  dnu_D(z) = (nu0/c) sqrt(2 k T / M + xi^2);  reduced frequency u = x * lam,
  lam = dnu_D_ref / dnu_D(z), dnu_D_ref = dnu_D(T_ref, xi = 0);
  a = (G_R + G_I + G_E)/(4 pi dnu_D);  eps = G_I/(G_R + G_I);
  G_E = r_E (G_R + G_I);
  u_b(Omega) = (nu0/c)(v . Omega)/dnu_D = (v . Omega)/v_th;
  alpha_{u,u'} = G_R/(G_R + G_I + G_E + 2 pi i nu_{u,u'}),
  beta_{u,u'}  = G_R/(G_R + G_I + 2 pi i nu_{u,u'})       (App. B).

Quantities are per unit reduced frequency: eta~ = eta dnu_D / k and
eps~ = eps dnu_D / k.  The transfer only needs the source vector eps/eta_I
and the ray optical depth, so k itself never appears.

Absorption (the propagation matrix, Sect. 2.1 and LL04 ch. 7): the 2x2
transverse Jones operator of the medium is
  N(nu) = c_abs sum_{u,l} Phi_{ul}(nu) (P d_ul^*)(P d_ul)^T,
  Phi_{ul} = conj(W(a, u + u_b + s_ul))/sqrt(pi),
where P projects on (e_a, e_b); the coherency C = <E E^dagger> obeys
dC/ds = -(N C + C N^dagger)/2, which gives K_{jk} = Tr((N A_k + A_k N^dagger) A_j)/4
for the Stokes matrices A = (1, sigma_z, sigma_x, -sigma_y) with
S_j = Tr(C A_j).  The sign of A_V makes eta_V = (phi_r - phi_b) cos(theta_B)/2
for sigma components with M_u - M_l = +1 (phi_b) and -1 (phi_r).

Emission (Eq. eps_sc_l with Eqs. RQIIKKp, G, RIIIQKKp, evaluated as in
App. D Eq. eps_sc_II_exp, in the comoving frame of Sect. 4.1):
  eps_bar^II_i(Omega, u; l, l') = c_sc/(2 pi) sum_{u,u'} alpha_{u u'} sum_{Omega'} w_{Omega'}
      sum_j E_i(u', u, l'; Omega) A_j(u, u', l; Omega')
      [W_{u' l, j}(Omega', Theta, u) + conj(W_{u l, j}(Omega', Theta, u))]
  with E_i(u', u, l') = d_{u'l'}^T Acart_i(Omega) d_{u l'}^*,
       A_j(u, u', l)  = d_{u l}^T Acart_j(Omega')/2 d_{u' l}^*,
       Acart_j = sum_ab (A_j)_ab e_a e_b^T,
       W_{t,j}(Omega', Theta, u_n) = sum_m M_{Theta t}[n, m] Ibar_j(Omega', u_m);
  eps_bar^III likewise with (beta - alpha)/(4 pi) and the separable incoming
  and outgoing factors of Eq. RIIIQKKp;
  eps^sc_i(Omega, u_n) = sum_{l,l'} S[eps_bar_i(Omega, .; l, l')](u_n + u_b(Omega) + u_{l,l'});
  eps^sc_I *= f (App. E normalisation).

Continuum (App. A), optional: true absorption kappa_c and scattering sigma_c
(given relative to the field-free line-centre absorption eta_0 of each
height) add kappa_c + sigma_c to the diagonal of K only; the thermal
continuum emission is kappa_c W_T (LTE, Stokes I); the scattering is
coherent in the observer frame with the dipole (Rayleigh) phase matrix,
  eps^c_i(Omega, nu) = sigma_c sum_{Omega'} w_{Omega'} sum_j R_ij(Omega, Omega') I_j(Omega', nu),
  R_ij = (3/4) Re Tr(Acart_i(Omega) Acart_j(Omega')),
which is the K = 0, 1, 2 multipole sum of App. A with unit weights; it joins
the normalised Sigma (the App. E factor f is computed from the line alone).

Formal solution (Sect. 3): trapezoidal ray optical depth
  dtau = (eta_I/eta_0 (z_k) + eta_I/eta_0 (z_k+1))/2 |dtau_line| / |mu|,
eta_0 = field-free line-centre value, and DELO-linear steps
  (Id + psi_c K'_c) I_c = (e^{-dtau} Id - psi_u K'_u) I_u + psi_u S_u + psi_c S_c,
K' = K/eta_I - Id, S = eps/eta_I, with psi_u = [1 - e^{-x}(1+x)]/x and
psi_c = [x - 1 + e^{-x}]/x.  Boundaries: (W_T(z_min), 0, 0, 0) entering from
below, nothing from above (Sect. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.sparse.linalg import LinearOperator, gmres

from .atom import build_atom
from .grids import angular_grid, theta_table, SplineBasis, weno4_interpolate
from .redistribution import SQRT_PI, faddeeva, kernel_matrix, kernel_matrix_aa, r3_weights

C_CGS = 2.99792458e10
K_B = 1.380649e-16
AMU = 1.66053906660e-24

# Stokes matrices A_j (S_j = Tr(C A_j)), I, Q, U, V
A_STOKES = np.array([[[1, 0], [0, 1]],
                     [[1, 0], [0, -1]],
                     [[0, 1], [1, 0]],
                     [[0, 1j], [-1j, 0]]], dtype=complex)


@dataclass
class OracleProblem:
    prob: object
    ang: dict
    theta: np.ndarray
    pair: np.ndarray
    basis: SplineBasis
    lam: np.ndarray
    dnuD: np.ndarray
    ub: np.ndarray            # [z, Omega]
    atoms: list
    s_ul: np.ndarray          # [z, n_u, n_l] profile shifts (reduced)
    s_ll: np.ndarray          # [z, n_l, n_l] lower-level shifts u_{l,l'}
    alpha: np.ndarray         # [z, n_u, n_u]
    beta: np.ndarray
    K: np.ndarray             # [z, Omega, n, 4, 4]
    eta0: np.ndarray          # [z]
    eps_th: np.ndarray        # [z, Omega, n, 4]
    Acart: np.ndarray         # [Omega, 4, 3, 3]
    opts: dict
    M: dict = field(default_factory=dict)
    r3: dict = field(default_factory=dict)
    f: np.ndarray = None      # [z, Omega, n]
    sigma_c: np.ndarray = None  # [z, n] continuum scattering coefficient (K units)
    cont: np.ndarray = None     # [z, n] continuum opacity kappa_c + sigma_c on the diagonal of K


def _acart(ang):
    ea, eb = ang["e_a"], ang["e_b"]
    basis = np.stack([ea, eb], axis=1)          # [Omega, 2(a,b), 3]
    return np.einsum("jab,oax,oby->ojxy", A_STOKES, basis, basis)


def setup(prob, opts=None) -> OracleProblem:
    """Per-height physics, angular grid, Theta table, propagation matrix.

    opts (test switches, all default off):
      alpha_zero:   alpha = 0 (complete redistribution: R_III carries beta)
      no_RII, no_RIII: drop one redistribution term
      zero_profile_shifts: transitions at the zero-field frequency in all
                    profiles while alpha/beta keep the sublevel splittings
      normalize:    apply the App. E factor f (default True)
      aa:           angle-averaged R_II (Sect. 5.2, Eq. R_AA) in place of the
                    angle-dependent kernel (default False)
      formal:       'linear' (DELO-linear, default), 'delopar' or 'besser' formal solver
      interp:       'spline' (default, Sect. 6.2) or 'weno4' (the non-oscillatory
                    interpolation named in Sect. 4.1, grids.weno4_interpolate)
                    for the observer/comoving frequency transforms; the kernel
                    rows keep the spline basis.  'weno4' makes Sigma nonlinear.
    """
    opts = dict({"normalize": True}, **(opts or {}))
    atom = prob.atom
    nu0 = C_CGS / (atom.lambda0_A * 1e-8)
    mass = atom.mass_amu * AMU
    vth = np.sqrt(2.0 * K_B * prob.T / mass + (prob.xi * 1e5) ** 2)
    vth_ref = np.sqrt(2.0 * K_B * prob.T_ref / mass)
    dnuD = nu0 * vth / C_CGS
    dnuD_ref = nu0 * vth_ref / C_CGS
    lam = dnuD_ref / dnuD
    ang = angular_grid(prob.n_mu, prob.n_chi, getattr(prob, "los_mu", None))
    theta, pair = theta_table(ang["dirs"])
    basis = SplineBasis(prob.x)
    nz, nd, nn = prob.n_z, prob.n_dir, prob.n_nu
    ub = (prob.v * 1e5) @ ang["dirs"].T / vth[:, None]
    atoms = [build_atom(atom, *prob.B[z], dnuD_ref) for z in range(nz)]
    nU = atoms[0].E_u.size
    nL = atoms[0].E_l.size
    s_ul = np.zeros((nz, nU, nL))
    s_ll = np.zeros((nz, nL, nL))
    alpha = np.zeros((nz, nU, nU), complex)
    beta = np.zeros((nz, nU, nU), complex)
    K = np.zeros((nz, nd, nn, 4, 4))
    eta0 = np.zeros(nz)
    Acart = _acart(ang)
    for z in range(nz):
        at = atoms[z]
        s_ul[z] = (at.E_u[:, None] - at.E_l[None, :]) / dnuD[z]
        s_ll[z] = (at.E_l[:, None] - at.E_l[None, :]) / dnuD[z]
        if opts.get("zero_profile_shifts"):
            s_ul[z] = 0.0
            s_ll[z] = 0.0
        g_tot = 4.0 * np.pi * prob.a[z] * dnuD[z]
        g_ri = g_tot / (1.0 + atom.r_E)
        g_r = (1.0 - prob.eps[z]) * g_ri
        nuuu = at.E_u[:, None] - at.E_u[None, :]
        alpha[z] = g_r / (g_tot + 2j * np.pi * nuuu)
        beta[z] = g_r / (g_ri + 2j * np.pi * nuuu)
        if opts.get("alpha_zero"):
            alpha[z] = 0.0
        eta0[z] = faddeeva(prob.a[z], 0.0).real / SQRT_PI
        # propagation matrix per (Omega, n)
        u = lam[z] * prob.x
        arg = u[None, :, None, None] + ub[z][:, None, None, None] + s_ul[z][None, None]
        Phi = np.conj(faddeeva(prob.a[z], arg)) / SQRT_PI          # [Om, n, u, l]
        pa = np.einsum("oi,uli->oul", ang["e_a"], np.conj(at.d))    # e_a . d^*
        pb = np.einsum("oi,uli->oul", ang["e_b"], np.conj(at.d))
        P = np.stack([pa, pb], axis=1)                               # [Om, 2, u, l]
        Nt = np.einsum("oaul,obul->oulab", P, np.conj(P))            # (e_a.d^*)(e_b.d)
        Nmed = at.c_abs * np.einsum("onul,oulab->onab", Phi, Nt)
        Ndag = np.conj(np.swapaxes(Nmed, -1, -2))
        t1 = np.einsum("onab,kbc,jca->onjk", Nmed, A_STOKES, A_STOKES)
        t2 = np.einsum("kab,onbc,jca->onjk", A_STOKES, Ndag, A_STOKES)
        K[z] = 0.25 * (t1 + t2).real
    eps_th = (prob.eps * prob.W_T)[:, None, None, None] * K[:, :, :, 0, :]
    kc = np.zeros((nz, nn))
    sc = np.zeros((nz, nn))
    if getattr(prob, "kappa_c", None) is not None:
        kc = np.asarray(prob.kappa_c, float) * eta0[:, None]
    if getattr(prob, "sigma_c", None) is not None:
        sc = np.asarray(prob.sigma_c, float) * eta0[:, None]
    for s in range(4):
        K[:, :, :, s, s] += (kc + sc)[:, None, :]
    eps_th[..., 0] += (kc * prob.W_T[:, None])[:, None, :]
    op = OracleProblem(prob=prob, ang=ang, theta=theta, pair=pair, basis=basis, lam=lam,
                       dnuD=dnuD, ub=ub, atoms=atoms, s_ul=s_ul, s_ll=s_ll, alpha=alpha,
                       beta=beta, K=K, eta0=eta0, eps_th=eps_th, Acart=Acart, opts=opts,
                       sigma_c=sc, cont=kc + sc)
    if opts["normalize"]:
        op.f = normalization(op)
    else:
        op.f = np.ones((nz, nd, nn))
    return op


def _kernel(op, z, th, u, l):
    # heights with identical (Theta, shift, damping, grid scale) share a kernel;
    # the angle-averaged kernel is the same for every pair
    if op.opts.get("aa"):
        key = ("aa", float(op.s_ul[z, u, l]), float(op.prob.a[z]), float(op.lam[z]))
        if key not in op.M:
            op.M[key] = kernel_matrix_aa(op.s_ul[z, u, l], op.prob.a[z], op.lam[z], op.basis)
        return op.M[key]
    key = (float(op.theta[th]), float(op.s_ul[z, u, l]), float(op.prob.a[z]), float(op.lam[z]))
    if key not in op.M:
        op.M[key] = kernel_matrix(op.theta[th], op.s_ul[z, u, l], op.prob.a[z],
                                  op.lam[z], op.basis)
    return op.M[key]


def _r3(op, z, u, l):
    key = (float(op.s_ul[z, u, l]), float(op.prob.a[z]), float(op.lam[z]))
    if key not in op.r3:
        op.r3[key] = r3_weights(op.s_ul[z, u, l], op.prob.a[z], op.lam[z], op.basis)
    return op.r3[key]


def _frame_interp(op, values, y):
    """Frequency transform between the observer and comoving grids (Sect. 4.1):
    the interpolant of values[n, ...] on the grid evaluated at y."""
    if op.opts.get("interp", "spline") == "weno4":
        return weno4_interpolate(op.basis.x, values, y, axis=0)
    return op.basis.interpolate(values, y, axis=0)


def comoving_field(op, z, Iz, o):
    """Ibar(u_m) = I(u_m - u_b(Omega')) for incoming direction o at height z (Sect. 4.1)."""
    return _frame_interp(op, Iz[o], op.prob.x - op.ub[z, o] / op.lam[z])


def sigma_height(op, z, Iz, normalize=True):
    """eps^sc at height z for the local field Iz[Omega, n, 4]."""
    prob = op.prob
    at = op.atoms[z]
    nd, nn = prob.n_dir, prob.n_nu
    nU, nL = at.E_u.size, at.E_l.size
    x = prob.x
    lam = op.lam[z]
    w = op.ang["w"]
    # 1. comoving field: Ibar(u_m) = S[I](u_m - u_b(Omega'))
    Ibar = np.empty_like(Iz)
    for o in range(nd):
        Ibar[o] = comoving_field(op, z, Iz, o)
    # 2. W for every ordered pair (outgoing Omega, incoming Omega')
    W = np.zeros((nU, nL, nd, nd, nn, 4), complex)
    if not op.opts.get("no_RII"):
        for u in range(nU):
            for l in range(nL):
                for o in range(nd):
                    for oi in range(nd):
                        W[u, l, o, oi] = _kernel(op, z, op.pair[o, oi], u, l) @ Ibar[oi]
    # 3. R_III incoming factor Y_{ul, j}(Omega') and outgoing profiles on the comoving grid
    Y = np.zeros((nU, nL, nd, 4), complex)
    prof = np.zeros((nU, nL, nn), complex)
    if not op.opts.get("no_RIII"):
        for u in range(nU):
            for l in range(nL):
                Y[u, l] = np.einsum("m,omj->oj", _r3(op, z, u, l), Ibar)
                prof[u, l] = faddeeva(prob.a[z], lam * x + op.s_ul[z, u, l])
    # 4. angular and sublevel sums, every pair explicitly
    d = at.d
    # E[o, i, u', u, l'] = d[u', l']^T Acart_i(o) d[u, l']^*
    E = np.einsum("prx,oixy,qry->oipqr", d, op.Acart, np.conj(d))
    # A[o', j, u, u', l] = d[u, l]^T Acart_j(o')/2 d[u', l]^*
    A = 0.5 * np.einsum("qlx,ojxy,ply->ojqpl", d, op.Acart, np.conj(d))
    al = op.alpha[z]
    bma = op.beta[z] - op.alpha[z]
    eps_bar = np.zeros((nL, nL, nd, nn, 4))
    for l in range(nL):
        for lp in range(nL):
            # 4x4 coefficients per (Omega, Omega', u, u'), quadrature weight included
            Cf = np.einsum("oipq,xjqp->oxijqp", E[..., lp], A[..., l])
            Cf = Cf * (at.c_sc * w)[None, :, None, None, None, None]
            # R_II: alpha_{u u'} [W_{u' l} + conj(W_{u l})]
            term_II = (np.einsum("oxijqp,qp,poxnj->oni", Cf, al, W[:, l])
                       + np.einsum("oxijqp,qp,qoxnj->oni", Cf, al, np.conj(W[:, l])))
            # R_III: (beta - alpha)_{u u'} (Y_{u'l} + conj Y_{ul})(prof_{u'l} + conj prof_{ul});
            # outgoing profiles on the comoving grid carry the shift s_{u,l}, the
            # back-interpolation adds u_{l,l'}
            inc = Y[:, l][None, :, :, :] + np.conj(Y[:, l])[:, None, :, :]      # [u, u', o', j]
            outp = prof[:, l][None, :, :] + np.conj(prof[:, l])[:, None, :]   # [u, u', n]
            term_III = np.einsum("oxijqp,qp,qpxj,qpn->oni", Cf, bma, inc, outp)
            eps_bar[l, lp] = (term_II / (2.0 * np.pi) + term_III / (4.0 * np.pi)).real
    # 5. back to the observer frame with the lower-level shift of each (l, l')
    out = np.zeros((nd, nn, 4))
    for l in range(nL):
        for lp in range(nL):
            for o in range(nd):
                y = x + (op.ub[z, o] + op.s_ll[z, l, lp]) / lam
                out[o] += _frame_interp(op, eps_bar[l, lp, o], y)
    if normalize:
        out[..., 0] *= op.f[z]
        if op.sigma_c is not None and np.any(op.sigma_c[z] != 0.0):
            out += continuum_scattering(op, z, Iz)
    return out


def rayleigh_matrix(Acart, o, x):
    """R[i, j] = (3/4) Re Tr(Acart_i(Omega_o) Acart_j(Omega_x)): the dipole
    scattering phase matrix from direction x into direction o."""
    return 0.75 * np.einsum("iab,jba->ij", Acart[o], Acart[x]).real


def continuum_scattering(op, z, Iz):
    """Coherent continuum scattering at height z (App. A) for the field Iz[Omega, n, 4]."""
    nd = op.prob.n_dir
    w = op.ang["w"]
    out = np.zeros_like(Iz)
    for o in range(nd):
        for x in range(nd):
            out[o] += w[x] * (Iz[x] @ rayleigh_matrix(op.Acart, o, x).T)
    return op.sigma_c[z][None, :, None] * out


def normalization_height(op, z):
    """App. E at height z: f = (1 - eps) W_T eta_I / eps^sc_I[I = (W_T, 0, 0, 0)], Stokes I only,
    with the line's own eta_I (the continuum takes no part in it)."""
    prob = op.prob
    Iz = np.zeros((prob.n_dir, prob.n_nu, 4))
    Iz[..., 0] = prob.W_T[z]
    num = sigma_height(op, z, Iz, normalize=False)[..., 0]
    ref = (1.0 - prob.eps[z]) * prob.W_T[z] * (op.K[z, :, :, 0, 0] - op.cont[z][None, :])
    # no line scattering (eps = 1): nothing to normalise
    return np.where(num != 0.0, ref / np.where(num != 0.0, num, 1.0), 1.0)


def normalization(op):
    """App. E normalisation factor for every height."""
    prob = op.prob
    f = np.ones((prob.n_z, prob.n_dir, prob.n_nu))
    for z in range(prob.n_z):
        f[z] = normalization_height(op, z)
    return f


def sigma_apply(op, I, normalize=True):
    """eps^sc = Sigma I for the full vector I[z, Omega, n, 4]."""
    out = np.zeros_like(I)
    for z in range(op.prob.n_z):
        out[z] = sigma_height(op, z, I[z], normalize=normalize)
    return out


def _psi(x):
    """DELO-linear weights psi_u, psi_c and exp(-x), series for small x."""
    x = np.asarray(x, float)
    ex = np.exp(-x)
    small = x < 0.1
    psi_u = np.empty_like(x)
    psi_c = np.empty_like(x)
    xl = np.where(small, 1.0, x)
    psi_u[~small] = ((1.0 - ex * (1.0 + xl)) / xl)[~small]
    psi_c[~small] = ((xl - 1.0 + ex) / xl)[~small]
    xs = x[small]
    # sum_{m>=2} (-1)^m (m-1) x^(m-1)/m!  and  sum_{m>=2} (-1)^m x^(m-1)/m!
    pu = np.zeros_like(xs)
    pc = np.zeros_like(xs)
    fact = 1.0
    for m in range(2, 22):
        fact *= m
        pu += (-1.0) ** m * (m - 1) * xs ** (m - 1) / fact
        pc += (-1.0) ** m * xs ** (m - 1) / fact
    psi_u[small] = pu
    psi_c[small] = pc
    return psi_u, psi_c, ex


def _exp_moments(m):
    """E_k = int_0^m t^k e^{-t} dt for k = 0, 1, 2 (power series below m = 0.5,
    where the closed forms cancel)."""
    m = np.asarray(m, float)
    ex = np.exp(-m)
    E0 = -np.expm1(-m)
    E1 = E0 - m * ex
    E2 = 2.0 * E1 - m * m * ex
    small = m < 0.5
    if np.any(small):
        ms = m[small]
        s = [np.zeros_like(ms) for _ in range(3)]
        term = np.ones_like(ms)              # (-1)^j m^j / j!
        for j in range(30):
            for k in range(3):
                s[k] += term * ms ** (k + 1) / (k + j + 1)
            term = -term * ms / (j + 1)
        E0 = np.where(small, 0.0, E0)
        E1 = np.where(small, 0.0, E1)
        E2 = np.where(small, 0.0, E2)
        E0[small], E1[small], E2[small] = s
    return E0, E1, E2


def _psi_parabolic(m, p):
    """Weights of S at the upwind (M), current (O) and downwind (P) points for
    int_0^m e^{-t} S(t) dt with S the parabola through the three points, t
    measured from O back along the ray (M at t = m, P at t = -p)."""
    E0, E1, E2 = _exp_moments(m)
    wM = (E2 + p * E1) / (m * (m + p))
    wO = -(E2 + (p - m) * E1 - m * p * E0) / (m * p)
    wP = (E2 - m * E1) / (p * (m + p))
    return wM, wO, wP


def _bezier_weights(m):
    """Weights of the upwind value, the control point and the current value for
    int_0^m e^{-t} B(t) dt, t the optical distance back from the current point
    and B the quadratic Bezier curve from the upwind point (t = m) to the
    current point (t = 0): its Bernstein factors are (t/m)^2, 2 (t/m)(1 - t/m)
    and (1 - t/m)^2, integrated through the moments E_k of the exponential."""
    E0, E1, E2 = _exp_moments(m)
    wM = E2 / (m * m)
    wC = 2.0 * (E1 / m - E2 / (m * m))
    wO = E0 - 2.0 * E1 / m + E2 / (m * m)
    return wM, wC, wO


def _besser_control(SM, SO, SP, hM, hP):
    """Control point of the Bezier source between the upwind (M) and current
    (O) points: the tangent at O of the parabola through M, O, P (zero where O
    is a local extremum), followed back half the interval, and kept inside the
    range spanned by S_M and S_O (no overshoot).  Componentwise."""
    dM = (SO - SM) / hM
    dP = (SP - SO) / hP
    dO = np.where(dM * dP > 0.0, (hM * dP + hP * dM) / (hM + hP), 0.0)
    c = SO - 0.5 * hM * dO
    return np.clip(c, np.minimum(SM, SO), np.maximum(SM, SO))


def formal_solve(op, eps, boundary=True, I_bottom=None, scheme=None):
    """Lambda eps (+ t if boundary): DELO sweeps along every ray.

    scheme 'linear' (default, or op.opts['formal']): DELO-linear, S and K'I
    linear between the upwind and current points.  'delopar': S parabolic
    through the upwind, current and downwind points, K'I linear (the
    DELOPAR integrator named in Sect. 3).  'besser': S a quadratic Bezier
    curve between the upwind and current points whose control point follows
    the three-point tangent at the current point and is kept inside the
    range of the two end values (no overshoot; this makes Lambda slightly
    nonlinear in eps, Sect. 6.2), K'I linear.  In both three-point schemes
    the last point of a ray, which has no downwind point, takes the
    DELO-linear step."""
    scheme = scheme or op.opts.get("formal", "linear")
    if scheme not in ("linear", "delopar", "besser"):
        raise ValueError(f"unknown formal scheme {scheme}")
    prob = op.prob
    nz, nd, nn = prob.n_z, prob.n_dir, prob.n_nu
    K = op.K
    etaI = K[..., 0, 0]                                  # [z, o, n]
    Kp = K / etaI[..., None, None] - np.eye(4)
    S = eps / etaI[..., None]
    ratio = etaI / op.eta0[:, None, None]
    mu = op.ang["mu"]
    dtl = np.abs(np.diff(prob.tau_line))                 # [nz-1]
    I = np.zeros((nz, nd, nn, 4))
    for o in range(nd):
        up = mu[o] > 0
        order = range(nz) if up else range(nz - 1, -1, -1)
        order = list(order)
        Icur = np.zeros((nn, 4))
        if up and boundary:
            if I_bottom is None:
                Icur[:, 0] = prob.W_T[0]
            else:
                Icur = np.array(I_bottom[o], float)
        I[order[0], o] = Icur
        for k in range(1, nz):
            zu, zc = order[k - 1], order[k]
            x = 0.5 * (ratio[zu, o] + ratio[zc, o]) * dtl[min(zu, zc)] / abs(mu[o])
            pu, pc, ex = _psi(x)
            lhs = np.eye(4)[None] + pc[:, None, None] * Kp[zc, o]
            rhs = (ex[:, None, None] * np.eye(4)[None] - pu[:, None, None] * Kp[zu, o])
            if scheme == "delopar" and k + 1 < nz:
                zd = order[k + 1]
                xd = 0.5 * (ratio[zc, o] + ratio[zd, o]) * dtl[min(zc, zd)] / abs(mu[o])
                wM, wO, wP = _psi_parabolic(x, xd)
                src = wM[:, None] * S[zu, o] + wO[:, None] * S[zc, o] + wP[:, None] * S[zd, o]
            elif scheme == "besser" and k + 1 < nz:
                zd = order[k + 1]
                xd = 0.5 * (ratio[zc, o] + ratio[zd, o]) * dtl[min(zc, zd)] / abs(mu[o])
                c = _besser_control(S[zu, o], S[zc, o], S[zd, o], x[:, None], xd[:, None])
                wM, wC, wO = _bezier_weights(x)
                src = wM[:, None] * S[zu, o] + wC[:, None] * c + wO[:, None] * S[zc, o]
            else:
                src = pu[:, None] * S[zu, o] + pc[:, None] * S[zc, o]
            b = np.einsum("nij,nj->ni", rhs, Icur) + src
            Icur = np.linalg.solve(lhs, b[..., None])[..., 0]
            I[zc, o] = Icur
    return I


def apply_operator(op, x):
    """(Id - Lambda Sigma) x, with Lambda without boundary radiation."""
    return x - formal_solve(op, sigma_apply(op, x), boundary=False)


def rhs(op):
    """b = Lambda eps_th + t."""
    return formal_solve(op, op.eps_th, boundary=True)


def solve(op, tol=1e-12, method="gmres", restart=200, maxiter=4000):
    """Solution of (Id - Lambda Sigma) I = Lambda eps_th + t."""
    if op.opts.get("interp", "spline") == "weno4":
        raise ValueError("the non-oscillatory transforms make Sigma nonlinear: "
                         "solve its fixed point with solve_aar")
    b = rhs(op)
    shape = b.shape
    n = b.size
    if method == "dense":
        A = np.empty((n, n))
        e = np.zeros(n)
        for k in range(n):
            e[:] = 0.0
            e[k] = 1.0
            A[:, k] = apply_operator(op, e.reshape(shape)).ravel()
        return np.linalg.solve(A, b.ravel()).reshape(shape)
    Aop = LinearOperator((n, n), matvec=lambda v: apply_operator(op, v.reshape(shape)).ravel(),
                         dtype=float)
    xsol, info = gmres(Aop, b.ravel(), rtol=tol, atol=0.0, restart=restart, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge (info={info})")
    return xsol.reshape(shape)


def fixed_point_map(op, I):
    """G(I) = Lambda (Sigma I + eps_th) + t with the problem's formal solver.
    The solution of Eq. linear_system is its fixed point; with BESSER, whose
    Lambda is not linear, the fixed point is the definition of the solution."""
    return formal_solve(op, sigma_apply(op, I) + op.eps_th, boundary=True)


def solve_aar(op, tol=1e-12, omega=1.0, beta=1.0, depth=7, period=6, maxiter=3000, precond=None):
    """Alternating Anderson-Richardson iteration (Sect. 5.1, the method of the
    cited AAR paper) for the fixed point of G.  With r = G(x) - x and
    f = M r (M = precond, a callable, or the identity), every step is a
    Richardson step x <- x + omega f except every `period`-th, which is an
    Anderson step x <- x + beta f - (X + beta F) gamma, gamma the least-squares
    solution of F gamma = f over the last `depth` differences F of f (X those
    of x).  Stops when ||r|| / ||G(0)|| < tol, the paper's relative residual.
    Returns (x, steps)."""
    b = fixed_point_map(op, np.zeros_like(op.eps_th))
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b - x
    Xh, Fh = [], []
    x_prev = f_prev = None
    for k in range(maxiter):
        if np.linalg.norm(r) / bn < tol:
            return x, k
        f = precond(r) if precond is not None else r
        if x_prev is not None and depth > 0:
            Xh.append((x - x_prev).ravel())
            Fh.append((f - f_prev).ravel())
            if len(Xh) > depth:
                Xh.pop(0)
                Fh.pop(0)
        x_prev, f_prev = x, f
        if depth > 0 and (k + 1) % period == 0 and Fh:
            F = np.stack(Fh, axis=1)
            X = np.stack(Xh, axis=1)
            gamma = np.linalg.lstsq(F, f.ravel(), rcond=None)[0]
            x = x + beta * f - ((X + beta * F) @ gamma).reshape(x.shape)
        else:
            x = x + omega * f
        r = fixed_point_map(op, x) - x
    raise RuntimeError("oracle AAR did not converge")


def emergent(op, I):
    """Stokes vectors at z_max for every outgoing (mu > 0) quadrature direction: [o, n, 4]."""
    ng = op.ang["n_grid"]
    up = op.ang["mu"][:ng] > 0
    return I[-1][:ng][up]


def los_emergent(op, I_grid):
    """Emergent Stokes vectors along the off-grid lines of sight, [los, chi, n, 4].

    Given the radiation field on the quadrature directions (I_grid[z, o, n, 4],
    o < n_grid; a converged solution), the emissivity eps = Sigma I + eps_th
    is evaluated for every direction, the lines of sight included, and one
    formal solution with the boundary radiation gives I = Lambda eps + t along
    them (the extra formal solution after convergence, Sect. 6).  The lines of
    sight carry zero quadrature weight, so whatever stands there in the input
    does not matter; they are set to zero."""
    prob = op.prob
    ng, nl, nc = op.ang["n_grid"], op.ang["n_los"], prob.n_chi
    if nl == 0:
        raise ValueError("the problem has no off-grid lines of sight")
    x = np.zeros((prob.n_z, prob.n_dir, prob.n_nu, 4))
    x[:, :ng] = np.asarray(I_grid)[:, :ng]
    full = formal_solve(op, sigma_apply(op, x) + op.eps_th, boundary=True)
    return full[-1, ng:].reshape(nl, nc, prob.n_nu, 4)
