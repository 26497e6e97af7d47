"""Seeded synthetic inputs for the polarised PRD transfer problem.

This module only *describes* problems: atom constants, frequency and angle grid
sizes, and atmosphere columns (temperature, line-centre optical depth, damping,
photon-destruction probability, Wien function, bulk velocity, magnetic field).
It holds none of the method's arithmetic (no Doppler widths, profiles,
redistribution functions or transfer).  Both the GPU path and the CPU oracle
read the same description.

The paper (Sect. 6.1) works on the FAL-C model with HanleRT-TIC/RH inputs,
none of which are available here.  The generators below stand in for them:
they take the *shape* of a chromosphere (temperature minimum, plateau, sharp
transition-region jump) and the paper's height domain z in [-100, 2219.43] km
(Sect. 6.3), with seeded random damping, fields and velocities.

Column order is bottom (z_min) to top (z_max).  The line-centre optical depth
``tau_line`` is the vertical field-free line-centre depth: it decreases
upward and is strictly positive at the top node.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

__all__ = ["Atom", "Problem", "cfg1", "cfg2", "cfg3", "cfg4", "tiny",
           "serving_stream", "two_level_atom", "two_term_atom"]


@dataclass(frozen=True)
class Atom:
    """Atomic model constants (paper Sect. 2.2; Table 1 for the two-term lines).

    kind:  "two_level" (J_l -> J_u, each level with its own Lande factor) or
           "two_term"  (L_l -> L_u with spin S, L-S coupling, Paschen-Back
           upper term, linear-Zeeman lower term).
    fs_split_x: two-term only, energy of the J=L+S level minus the J=L-S level
           of the upper term, in units of the reference Doppler width.
    r_E:   Gamma_E / (Gamma_R + Gamma_I), the elastic-collision share that
           sets the R_III weight (the configs leave it open; 1 is used).
    """
    kind: str
    lambda0_A: float
    mass_amu: float
    J_l: float = 0.0
    J_u: float = 1.0
    g_l: float = 0.0
    g_u: float = 1.0
    L_l: int = 0
    L_u: int = 1
    S: float = 0.0
    fs_split_x: float = 0.0
    r_E: float = 1.0


def two_level_atom() -> Atom:
    """J_l=0 -> J_u=1 resonance line with Ca I 4227-like constants."""
    return Atom(kind="two_level", lambda0_A=4227.0, mass_amu=40.08,
                J_l=0.0, J_u=1.0, g_l=0.0, g_u=1.0)


def two_term_atom(lambda0_A: float, mass_amu: float, fs_split_x: float) -> Atom:
    """2S_1/2 -> 2P_{1/2,3/2} doublet (Mg II h&k-like or H I Ly-alpha-like)."""
    return Atom(kind="two_term", lambda0_A=lambda0_A, mass_amu=mass_amu,
                L_l=0, L_u=1, S=0.5, fs_split_x=fs_split_x)


@dataclass
class Problem:
    """One forward-solve request: atom, grids and atmosphere columns."""
    name: str
    atom: Atom
    x: np.ndarray              # [n_nu] frequency nodes, x = (nu0 - nu)/dnu_D_ref
    n_mu: int                  # total Gauss-Legendre mu nodes (n_mu/2 per hemisphere)
    n_chi: int                 # trapezoid azimuths
    tau_line: np.ndarray       # [n_z] vertical field-free line-centre optical depth
    T: np.ndarray              # [n_z] K
    xi: np.ndarray             # [n_z] microturbulence, km/s
    a: np.ndarray              # [n_z] damping parameter
    eps: np.ndarray            # [n_z] photon-destruction probability
    W_T: np.ndarray            # [n_z] Wien function, 1 at the bottom
    v: np.ndarray              # [n_z, 3] bulk velocity, km/s, cartesian, z up
    B: np.ndarray              # [n_z, 3] (|B| in G, theta_B rad, chi_B rad)
    z_km: Optional[np.ndarray] = None
    # continuum (App. A): true absorption and scattering coefficients per height
    # and frequency, [n_z, n_nu], in units of the height's field-free
    # line-centre absorption coefficient; None = no continuum
    kappa_c: Optional[np.ndarray] = None
    sigma_c: Optional[np.ndarray] = None
    # off-grid lines of sight: mu values in (0, 1], each a ring of the n_chi
    # azimuths after the quadrature directions, with zero quadrature weight
    los_mu: Optional[np.ndarray] = None
    T_ref: float = 6000.0      # temperature that defines dnu_D_ref
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)

    @property
    def n_z(self) -> int:
        return int(self.tau_line.shape[0])

    @property
    def n_nu(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_los(self) -> int:
        return 0 if self.los_mu is None else int(np.asarray(self.los_mu).size)

    @property
    def n_dir_grid(self) -> int:
        return self.n_mu * self.n_chi

    @property
    def n_dir(self) -> int:
        return (self.n_mu + self.n_los) * self.n_chi

    @property
    def n_unknowns(self) -> int:
        return 4 * self.n_z * self.n_nu * self.n_dir

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def _chromosphere_T(z: np.ndarray) -> np.ndarray:
    """Temperature shape: 6400 -> 4400 K minimum at 500 km, rise to a
    7000-10000 K plateau, tanh jump to 5e4 K at 2000 km (width 10 km)."""
    T = np.empty_like(z)
    z0 = z.min()
    lo = z <= 500.0
    T[lo] = 6400.0 + (4400.0 - 6400.0) * (z[lo] - z0) / (500.0 - z0)
    mid = (z > 500.0) & (z <= 1000.0)
    T[mid] = 4400.0 + (7000.0 - 4400.0) * (z[mid] - 500.0) / 500.0
    hi = z > 1000.0
    T[hi] = 7000.0 + (10000.0 - 7000.0) * np.clip((z[hi] - 1000.0) / 980.0, 0.0, 1.0)
    jump = 0.5 * (1.0 + np.tanh((z - 2000.0) / 10.0))
    return T * (1.0 - jump) + 5.0e4 * jump


def _chromosphere(name: str, atom: Atom, x: np.ndarray, n_mu: int, n_chi: int,
                  n_z: int, seed: int, a_range=(1e-3, 5e-2),
                  B_range=(1.0, 100.0), v_amp=5.0) -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    z = np.linspace(-100.0, 2219.43, n_z)
    T = _chromosphere_T(z)
    tau = np.logspace(2.0, -6.0, n_z)
    a = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), n_z))
    # "Saha-like" destruction probability, chi = 5 eV, clipped to [1e-6, 0.5]
    chi_over_k = 5.0 * 11604.518
    eps = 1e-4 * (T / 6000.0) ** 1.5 * np.exp(chi_over_k * (1.0 / 6000.0 - 1.0 / T))
    eps = np.clip(eps, 1e-6, 0.5)
    # Wien function normalised to 1 at the bottom node
    hnu_over_k = 1.438776877e8 / atom.lambda0_A   # h c / (k lambda) in K, lambda in A
    W_T = np.exp(-hnu_over_k / T) / np.exp(-hnu_over_k / T[0])
    Bmag = np.exp(rng.uniform(np.log(B_range[0]), np.log(B_range[1]), n_z))
    thB = np.arccos(rng.uniform(-1.0, 1.0, n_z))
    chB = rng.uniform(0.0, 2.0 * np.pi, n_z)
    phase = rng.uniform(0.0, 2.0 * np.pi)
    vz = v_amp * np.sin(2.0 * np.pi * (z - z[0]) / (z[-1] - z[0]) + phase)
    v = np.zeros((n_z, 3))
    v[:, 2] = vz
    return Problem(name=name, atom=atom, x=np.asarray(x, float), n_mu=n_mu, n_chi=n_chi,
                   tau_line=tau, T=T, xi=np.zeros(n_z), a=a, eps=eps, W_T=W_T, v=v,
                   B=np.stack([Bmag, thB, chB], axis=1), z_km=z,
                   meta={"seed": seed})


def cfg1() -> Problem:
    """Two-level J 0->1, isothermal slab, N_z=40, N_nu=31 on [-8,8], 2+2 mu x 4 chi,
    a=1e-3, eps=1e-4, horizontal 20 G field, static."""
    n_z = 40
    return Problem(name="cfg1_two_level_slab", atom=two_level_atom(),
                   x=np.linspace(-8.0, 8.0, 31), n_mu=4, n_chi=4,
                   tau_line=np.logspace(2.0, -6.0, n_z), T=np.full(n_z, 6000.0),
                   xi=np.zeros(n_z), a=np.full(n_z, 1e-3), eps=np.full(n_z, 1e-4),
                   W_T=np.ones(n_z), v=np.zeros((n_z, 3)),
                   B=np.tile([20.0, np.pi / 2, 0.0], (n_z, 1)), tol=1e-8)


def cfg2(seed: int = 2) -> Problem:
    """Two-level, seeded chromosphere-like column, N_z=70, N_nu=101 on [-12,12],
    4+4 mu x 8 chi, a log-uniform in [1e-3,5e-2], |B| log-uniform 1-100 G,
    vertical 5 km/s sinusoidal velocity."""
    return _chromosphere("cfg2_two_level_chromosphere", two_level_atom(),
                         np.linspace(-12.0, 12.0, 101), 8, 8, 70, seed)


def _cfg3_grid() -> np.ndarray:
    core = []
    for xc in (-10.0, 10.0):
        core.append(np.linspace(xc - 7.0, xc + 7.0, 71))
    gap = np.linspace(-3.0, 3.0, 7)[1:-1]
    wing_r = 17.0 + (50.0 - 17.0) * (np.logspace(0.0, 1.0, 27)[1:] - 1.0) / 9.0
    x = np.concatenate([-wing_r[::-1], core[0], gap, core[1], wing_r])
    x = np.unique(np.round(x, 12))
    if x.size < 200:   # one extra far-wing node to reach 200
        x = np.sort(np.append(x, 0.5 * (x[-1] + x[-2])))
    return x[:200] if x.size > 200 else x


def cfg3(seed: int = 3, n_z: int = 80) -> Problem:
    """Two-term Mg II h&k-like doublet, components at x=+-10, N_z=80, N_nu=200,
    6+6 mu x 8 chi.  n_z < 80 gives the same generator on fewer heights."""
    atom = two_term_atom(2800.0, 24.305, 20.0)
    return _chromosphere("cfg3_two_term_doublet", atom, _cfg3_grid(), 12, 8, n_z, seed)


def cfg4(seed: int = 4, n_z: int = 100) -> Problem:
    """Two-term H I Ly-alpha-like line (fine structure 0.3 Doppler widths), wide
    damping, N_z=100, N_nu=301 on a sinh grid to +-1000, 8+8 mu x 8 chi.
    n_z < 100 gives the same generator on fewer heights."""
    atom = two_term_atom(1215.67, 1.008, 0.3)
    s = np.linspace(-1.0, 1.0, 301)
    x = 1000.0 * np.sinh(6.0 * s) / np.sinh(6.0)
    return _chromosphere("cfg4_two_term_wide_wings", atom, x, 16, 8, n_z, seed,
                         a_range=(1e-2, 1e-1), B_range=(1.0, 300.0))


def tiny(n_z: int = 6, n_nu: int = 13, x_max: float = 6.0, n_mu: int = 2, n_chi: int = 4,
         atom: Optional[Atom] = None, B=(20.0, np.pi / 2, 0.0), v_z: float = 0.0,
         a: float = 1e-2, eps: float = 1e-2, tau_top: float = 1e-3, tau_bot: float = 1e2,
         seed: Optional[int] = None, T: float = 6000.0, cont: Optional[tuple] = None,
         los_mu=None) -> Problem:
    """Small problems for oracle pins and GPU parity.  With ``seed`` set, the
    damping, destruction probability, field and velocity vary with height.
    ``cont = (kappa, sigma)`` adds a continuum whose coefficients (relative to
    the line-centre absorption) change linearly by 25 % across the grid
    (kappa rising to the red end, sigma to the blue end) and vary with height.
    ``los_mu`` adds off-grid lines of sight (rings of zero weight)."""
    atom = atom or two_level_atom()
    tau = np.logspace(np.log10(tau_bot), np.log10(tau_top), n_z)
    Tz = np.full(n_z, float(T))
    az = np.full(n_z, float(a))
    epsz = np.full(n_z, float(eps))
    Bz = np.tile(np.asarray(B, float), (n_z, 1))
    v = np.zeros((n_z, 3))
    v[:, 2] = v_z
    W_T = np.ones(n_z)
    if seed is not None:
        rng = np.random.Generator(np.random.PCG64(seed))
        Tz = T * np.exp(rng.uniform(-0.3, 0.3, n_z))
        az = a * np.exp(rng.uniform(-1.0, 1.0, n_z))
        epsz = eps * np.exp(rng.uniform(-1.0, 1.0, n_z))
        Bz = np.stack([B[0] * np.exp(rng.uniform(-1.0, 1.0, n_z)),
                       np.arccos(rng.uniform(-1.0, 1.0, n_z)),
                       rng.uniform(0.0, 2.0 * np.pi, n_z)], axis=1)
        v[:, 2] = v_z * np.sin(np.linspace(0.0, 2.0 * np.pi, n_z) + rng.uniform(0, 6.28))
        W_T = np.exp(rng.uniform(-0.2, 0.2, n_z))
        W_T /= W_T[0]
    kc = sc = None
    if cont is not None:
        x = np.linspace(-x_max, x_max, n_nu)
        tilt = 1.0 + 0.25 * (x - x[0]) / (x[-1] - x[0])
        hz = np.exp(np.linspace(-0.3, 0.3, n_z)) if seed is None else np.exp(
            np.random.Generator(np.random.PCG64(seed + 1)).uniform(-0.5, 0.5, n_z))
        kc = cont[0] * hz[:, None] * tilt[None, :]
        sc = cont[1] * hz[::-1, None] * tilt[None, ::-1]
    return Problem(name=f"tiny_{atom.kind}", atom=atom,
                   x=np.linspace(-x_max, x_max, n_nu), n_mu=n_mu, n_chi=n_chi,
                   tau_line=tau, T=Tz, xi=np.zeros(n_z), a=az, eps=epsz, W_T=W_T,
                   v=v, B=Bz, kappa_c=kc, sigma_c=sc,
                   los_mu=None if los_mu is None else np.asarray(los_mu, float), meta={"seed": seed})


def serving_stream(n_requests: int = 1024, seed: int = 5, rate_hz: float = 10.0,
                   n_z_range=(40, 100), nu_choices=None, angle_sets=None):
    """Request stream: each request picks one of the four configurations'
    generators with its own seed and resized grids; arrivals are Poisson.
    Defaults span N_z 40-100, N_nu 31-301 and N_dir 16-128; the ranges can be
    narrowed (a bounded stream for short runs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n_requests))
    if angle_sets is None:
        angle_sets = [(4, 4), (8, 4), (8, 8), (12, 8), (16, 8)]
    if nu_choices is None:
        nu_choices = np.arange(31, 302, 30)
    reqs = []
    for i in range(n_requests):
        kind = int(rng.integers(0, 4))
        n_z = int(rng.integers(n_z_range[0], n_z_range[1] + 1))
        n_nu = int(rng.choice(np.asarray(nu_choices)))
        n_mu, n_chi = angle_sets[int(rng.integers(0, len(angle_sets)))]
        s = 5000 + i
        if kind <= 1:
            p = _chromosphere(f"req{i}", two_level_atom(), np.linspace(-12, 12, n_nu),
                              n_mu, n_chi, n_z, s)
        elif kind == 2:
            p = _chromosphere(f"req{i}", two_term_atom(2800.0, 24.305, 20.0),
                              np.linspace(-50, 50, n_nu), n_mu, n_chi, n_z, s)
        else:
            sg = np.linspace(-1.0, 1.0, n_nu)
            p = _chromosphere(f"req{i}", two_term_atom(1215.67, 1.008, 0.3),
                              1000.0 * np.sinh(6.0 * sg) / np.sinh(6.0), n_mu, n_chi, n_z, s,
                              a_range=(1e-2, 1e-1), B_range=(1.0, 300.0))
        reqs.append((float(t[i]), p))
    return reqs
