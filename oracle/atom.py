"""Atomic model for the oracle: states, energies and dipole vectors.

Sect. 2.2: a two-term atom (L-S coupling, terms (L_l, S) and (L_u, S)) with
the two-level atom as the S = 0 case.  In a magnetic field the upper term is
treated in the Paschen-Back regime (states labelled j, Sect. 2.2) and the
lower level/term is infinitely sharp and unpolarised (Sect. 2.2).

States are built in the uncoupled basis |L M_L>|S M_S> with quantisation
axis along B.  Hamiltonian (in Hz):
    upper:  zeta (L.S + c) + nu_L (g_L M_L + g_S M_S)
    lower:  nu_L (g_L M_L + g_S M_S)
with nu_L = mu_B B / h, c centring the two J levels on nu0, g_L = 1 and
g_S = 2.  For the two-level atom (S = 0) the Lande factors of the
configuration are used directly.  Eigenstates of the upper term are
obtained by a dense Hermitian eigensolver (numpy.linalg.eigh).

Dipole matrix elements follow from the Wigner-Eckart theorem on the orbital
part; the electric dipole does not act on spin:
    <L_u M_Lu, S M_Su | D_q | L_l M_Ll, S M_Sl>
        = delta(M_Su, M_Sl) sqrt(3) (-1)^(L_u - M_Lu) (L_u 1 L_l; -M_Lu q M_Ll).
The cartesian dipole vector is d = sum_q <u|D_q|l> e_q^*, with the spherical
unit vectors e_{+-1} = -+(e_x +- i e_y)/sqrt(2), e_0 = e_z, expressed in the
atmospheric frame by rotating the magnetic frame (z_B along B).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from sympy import Rational
from sympy.physics.wigner import wigner_3j

NU_LARMOR_PER_G = 1.39962449361e6      # mu_B / h in Hz per gauss


def _r(x: float):
    return Rational(int(round(2 * x)), 2)


def w3j(j1, j2, j3, m1, m2, m3) -> float:
    return float(wigner_3j(_r(j1), _r(j2), _r(j3), _r(m1), _r(m2), _r(m3)))


def _mvals(j: float):
    n = int(round(2 * j)) + 1
    return np.array([-j + k for k in range(n)])


@dataclass
class AtomModel:
    """Sublevel structure at one height.

    E_u, E_l: energies of upper/lower states in Hz, relative to nu0 (so the
      transition frequency nu_{u,l} - nu0 = E_u - E_l).
    d: [n_u, n_l, 3] complex dipole vectors in the atmospheric frame.
    c_abs, c_sc: normalisations (absorption profile integrates to 1 at B=0;
      generalised Kirchhoff law for the emission, App. E).
    """
    E_u: np.ndarray
    E_l: np.ndarray
    d: np.ndarray
    c_abs: float
    c_sc: float


def _term_states(L: float, S: float):
    return [(ml, ms) for ml in _mvals(L) for ms in _mvals(S)]


def _term_hamiltonian(L, S, zeta, shift, nu_L, gL, gS):
    st = _term_states(L, S)
    n = len(st)
    H = np.zeros((n, n))
    for a, (ml, ms) in enumerate(st):
        H[a, a] = zeta * (ml * ms + shift) + nu_L * (gL * ml + gS * ms)
        for b, (ml2, ms2) in enumerate(st):
            # (L+ S- + L- S+)/2 couples (ml, ms) -> (ml+-1, ms-+1)
            if ml2 == ml + 1 and ms2 == ms - 1:
                v = np.sqrt(L * (L + 1) - ml * (ml + 1)) * np.sqrt(S * (S + 1) - ms * (ms - 1))
                H[b, a] += 0.5 * zeta * v
            if ml2 == ml - 1 and ms2 == ms + 1:
                v = np.sqrt(L * (L + 1) - ml * (ml - 1)) * np.sqrt(S * (S + 1) - ms * (ms + 1))
                H[b, a] += 0.5 * zeta * v
    return st, H


def magnetic_frame(theta_B: float, chi_B: float):
    """Columns: x_B, y_B, z_B unit vectors in the atmospheric frame."""
    st, ct = np.sin(theta_B), np.cos(theta_B)
    sc, cc = np.sin(chi_B), np.cos(chi_B)
    zB = np.array([st * cc, st * sc, ct])
    xB = np.array([ct * cc, ct * sc, -st])
    yB = np.array([-sc, cc, 0.0])
    return np.stack([xB, yB, zB], axis=1)


def build_atom(atom, B_gauss: float, theta_B: float, chi_B: float,
               dnuD_ref_hz: float) -> AtomModel:
    """Sublevels, energies (Hz, relative to nu0) and atmospheric-frame dipoles.

    ``atom`` is a workloads.Atom.  For the two-term atom the fine-structure
    constant zeta is set so that E(J=L+S) - E(J=L-S) equals
    fs_split_x * dnu_D_ref and the two J levels sit symmetrically about nu0.
    """
    nu_L = NU_LARMOR_PER_G * B_gauss
    if atom.kind == "two_level":
        Lu, Ll, S = atom.J_u, atom.J_l, 0.0
        zeta, shift = 0.0, 0.0
        gLu, gSu, gLl, gSl = atom.g_u, 0.0, atom.g_l, 0.0
    elif atom.kind == "two_term":
        Lu, Ll, S = float(atom.L_u), float(atom.L_l), float(atom.S)
        # L.S eigenvalue for J: [J(J+1) - L(L+1) - S(S+1)]/2
        def ls(J):
            return 0.5 * (J * (J + 1) - Lu * (Lu + 1) - S * (S + 1))
        Jhi, Jlo = Lu + S, abs(Lu - S)
        gap = ls(Jhi) - ls(Jlo)
        zeta = atom.fs_split_x * dnuD_ref_hz / gap if gap != 0 else 0.0
        shift = -0.5 * (ls(Jhi) + ls(Jlo))
        gLu, gSu, gLl, gSl = 1.0, 2.0, 1.0, 2.0
    else:
        raise ValueError(f"unknown atom kind {atom.kind}")
    st_u, Hu = _term_hamiltonian(Lu, S, zeta, shift, nu_L, gLu, gSu)
    st_l, Hl = _term_hamiltonian(Ll, S, 0.0, 0.0, nu_L, gLl, gSl)
    Eu, Vu = np.linalg.eigh(Hu)
    El, Vl = np.linalg.eigh(Hl)
    # spherical dipole components in the uncoupled basis, B frame
    nu_, nl_ = len(st_u), len(st_l)
    Dq = np.zeros((3, nu_, nl_))               # q = -1, 0, +1
    for a, (mlu, msu) in enumerate(st_u):
        for b, (mll, msl) in enumerate(st_l):
            if abs(msu - msl) > 1e-9:
                continue
            for iq, q in enumerate((-1, 0, 1)):
                if abs(-mlu + q + mll) > 1e-9:
                    continue
                Dq[iq, a, b] = np.sqrt(3.0) * (-1.0) ** int(round(Lu - mlu)) * w3j(Lu, 1, Ll, -mlu, q, mll)
    # to eigenstates: <u_k| D |l_m> = sum V_u[a,k]^* Dq[a,b] V_l[b,m]
    Dq = np.einsum("ak,qab,bm->qkm", Vu.conj(), Dq, Vl)
    # cartesian in B frame: d = sum_q D_q e_q^*
    ex, ey, ez = np.eye(3)
    e_sph = {-1: (ex - 1j * ey) / np.sqrt(2.0), 0: ez + 0j, 1: -(ex + 1j * ey) / np.sqrt(2.0)}
    dB = np.zeros((nu_, nl_, 3), complex)
    for iq, q in enumerate((-1, 0, 1)):
        dB += Dq[iq][:, :, None] * np.conj(e_sph[q])[None, None, :]
    R = magnetic_frame(theta_B, chi_B)
    d = np.einsum("ij,ulj->uli", R, dB)
    tot = np.sum(np.abs(d) ** 2)
    c_abs = 3.0 / tot
    Du = np.sum(np.abs(d) ** 2, axis=(1, 2))
    if not np.allclose(Du, Du[0], rtol=1e-10):
        raise RuntimeError("upper-state dipole sums differ; L-S structure broken")
    c_sc = 3.0 * c_abs / (2.0 * Du[0])
    return AtomModel(E_u=Eu, E_l=El, d=d, c_abs=c_abs, c_sc=c_sc)
