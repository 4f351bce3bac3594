"""Compliant-mechanism objective of Sec. 4.1 (the force inverter): Eq. (1)
with z the unit vector of the output DOF, so J = z^T u = u_out.

Test infrastructure only (see the package docstring).

The adjoint of J: with K u = f and K symmetric, dJ/drho = -lambda^T (dK/drho) u
with K lambda = z, i.e. lambda is the displacement under a unit load at the
output DOF.  K = sum_e P_e^T (sum_s E(rho_s) K_s) P_e plus the ground springs
(which do not depend on rho), so
dJ/drho_{e,s} = -E'(rho_{e,s}) lambda_e^T K_s u_e.
"""

import numpy as np

from .fem import simp_modulus_derivative, subcell_stiffness
from .solve import cell_offsets, element_dofs_global, oracle_solve, rigid_free
from .space import build_space


def bilinear_sensitivity(nelx, nely, p, d, rho, u, lam, E0=1.0, Emin=1e-9, q=3.0, nu=0.3):
    """-E'(rho_{e,s}) lam_e^T K_s u_e for every cell, global vectors u, lam
    [n_dof] (with lam = u it is the compliance sensitivity).  Both element
    vectors have their rigid motions removed first (K_s annihilates them;
    see rigid_free in solve.py)."""
    p = np.asarray(p, dtype=np.int64).ravel()
    d = np.asarray(d, dtype=np.int64).ravel()
    rho = np.asarray(rho, dtype=np.float64).ravel()
    space = build_space(nelx, nely, p)
    off = cell_offsets(d)
    dE = simp_modulus_derivative(rho, E0, Emin, q)
    out = np.zeros(rho.size)
    cache = {}
    for e in range(nelx * nely):
        key = (int(p[e]), int(d[e]))
        if key not in cache:
            cache[key] = subcell_stiffness(key[0], key[1], nu)
        G = element_dofs_global(space, e)
        ue = rigid_free(np.where(G >= 0, u[np.maximum(G, 0)], 0.0), key[0])
        le = rigid_free(np.where(G >= 0, lam[np.maximum(G, 0)], 0.0), key[0])
        out[off[e]:off[e + 1]] = -dE[off[e]:off[e + 1]] * np.einsum("i,sij,j->s", le, cache[key], ue)
    return out


def global_dof(nelx, vx, vy, comp):
    return 2 * (vy * (nelx + 1) + vx) + comp


def mechanism(pr):
    """J = u_out and dJ/drho for a Problem whose load case 0 is the input
    force and load case 1 the unit load at the output DOF (pr.out_dof)."""
    o = oracle_solve(**pr.oracle_args())
    u, lam = o["u"][0], o["u"][1]
    J = float(u[global_dof(pr.nelx, *pr.out_dof)])
    g = bilinear_sensitivity(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, u, lam, pr.E0, pr.Emin, pr.q, pr.nu)
    return J, g, o
