"""Plain, slow FP64 CPU oracle for the linearised polarised PRD transfer problem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; only the seeded problem descriptions in ``workloads`` serve both.

It follows Riva et al., "A numerical approach for modelling the polarisation
signals of strong resonance lines with partial frequency redistribution":

* the linear system (Id - Lambda Sigma) I = Lambda eps_th + t  (Sect. 2.7,
  Eq. linear_system), solved by dense LU on tiny grids or FP64 GMRES;
* Sigma: the scattering integral (Eq. eps_sc_l) with R = R_II + R_III
  (Eqs. RQIIKKp, G, RIIIQKKp), evaluated in the comoving frame (Sect. 4.1,
  Eq. eps_sc_bar) through the frequency-integrated intermediate W
  (App. D, Eqs. Wkukl and eps_sc_II_exp), with the angular quadrature of
  Sect. 4.2, product integration over frequency (Sect. 4.3), and the
  generalised-Kirchhoff normalisation of App. E;
* Lambda: DELO-linear ray sweeps with trapezoidal optical depth (Sect. 3).

The paper cites, without printing, the coefficients that carry the atomic
structure (the A/B tables of App. B and the scattering phase matrix).  This
oracle writes the redistribution matrix from the second-order scattering
amplitude with explicit dipole vectors between the magnetic sublevels (or
Paschen-Back eigenstates), the branching ratios alpha and beta of App. B,
and the partial-fraction split of the product of two resonance denominators
that produces the [G(k_u') + G(k_u)*] pairing of Eq. RQIIKKp.  That regroups
exactly into the paper's multipole form; the pins in ``tests/`` check it
against closed forms that do not go through the dipole vectors.

Where the paper leaves a point open, the reading taken is stated beside the
function that implements it.
"""
from .grids import angular_grid, theta_table, SplineBasis
from .atom import AtomModel, build_atom
from .redistribution import faddeeva, F_function, kernel_matrix, kernel_matrix_aa, r3_weights
from .transfer import (OracleProblem, setup, sigma_apply, formal_solve, apply_operator, solve, emergent,
                       los_emergent, fixed_point_map, solve_aar)

__all__ = ["angular_grid", "theta_table", "SplineBasis", "AtomModel", "build_atom",
           "faddeeva", "F_function", "kernel_matrix", "kernel_matrix_aa", "r3_weights",
           "OracleProblem", "setup", "sigma_apply", "formal_solve", "apply_operator", "solve", "emergent",
           "los_emergent", "fixed_point_map", "solve_aar"]
