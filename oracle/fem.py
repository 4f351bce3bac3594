"""Element-level pieces of the oracle: 1D basis, plane-stress D0, SIMP, and
the per-density-cell stiffness matrices K_s.

Test infrastructure only (see the package docstring).

Geometry reading: element (ex, ey) is the unit square [ex, ex+1] x [ey, ey+1]
(the paper uses square elements of edge h, Sec. 4.1; 2D elasticity stiffness
is independent of h).  Reference coordinates xi, eta in [-1, 1] with
x = ex + (xi + 1)/2, so d/dx = 2 d/dxi and dx dy = dxi deta / 4.
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def basis_1d(p, xi):
    """Hierarchic 1D shape functions of order p and their xi-derivatives.

    The paper does not name its basis (it uses the FE library of its
    acknowledgements); any basis of the same polynomial space gives the same
    discrete field, compliance and sensitivities.  The reading used here:
    index 0 is (1 - xi)/2 (left vertex), index 1 is (1 + xi)/2 (right vertex),
    and index k = 2..p is the integrated Legendre polynomial
    L_k(xi) = integral_{-1}^{xi} P_{k-1}(t) dt, which vanishes at both ends.

    Returns (phi, dphi), each of shape [p+1, len(xi)].
    """
    xi = np.asarray(xi, dtype=np.float64)
    phi = np.empty((p + 1, xi.size))
    dphi = np.empty((p + 1, xi.size))
    phi[0] = 0.5 * (1.0 - xi)
    phi[1] = 0.5 * (1.0 + xi)
    dphi[0] = -0.5
    dphi[1] = 0.5
    for k in range(2, p + 1):
        pk1 = npleg.Legendre.basis(k - 1)
        lk = pk1.integ(lbnd=-1.0)  # antiderivative that is zero at xi = -1
        phi[k] = lk(xi)
        dphi[k] = pk1(xi)
    return phi, dphi


def constitutive_plane_stress(nu):
    """D0 of Sec. 2.2 (constitutive matrix normalised by Young's modulus),
    plane stress, Voigt order (eps_xx, eps_yy, gamma_xy), unit thickness.
    Plane stress is the reading for the paper's '2D' problems."""
    return (1.0 / (1.0 - nu * nu)) * np.array(
        [[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]]
    )


def simp_modulus(rho, E0, Emin, q):
    """Modified SIMP interpolation of Sec. 2.2: E = Emin + rho^q (E0 - Emin)."""
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho**q * (E0 - Emin)


def simp_modulus_derivative(rho, E0, Emin, q):
    """dE/drho of the modified SIMP law of Sec. 2.2: q rho^(q-1) (E0 - Emin)."""
    rho = np.asarray(rho, dtype=np.float64)
    return q * rho ** (q - 1.0) * (E0 - Emin)


def local_index(p, i, j, comp):
    """Local DOF number of component comp of the tensor-product function
    phi_i(xi) phi_j(eta): scalar index a = j (p+1) + i, DOF 2a + comp."""
    return 2 * (j * (p + 1) + i) + comp


def subcell_stiffness(p, d, nu):
    """Composite per-density-cell stiffness matrices (Appendix B).

    For density cell s = sy*d + sx, which covers
    [sx/d, (sx+1)/d] x [sy/d, (sy+1)/d] of the unit element, returns
    K_s = integral over the cell of B^T D0 B (Sec. 2.2), evaluated with a
    (p+1) x (p+1) Gauss-Legendre rule mapped to the cell.  The integrand is a
    polynomial of degree at most 2p in each direction, so the rule is exact.

    Returns an array [d*d, n_e, n_e] with n_e = 2 (p+1)^2.
    """
    n1 = p + 1
    ne = 2 * n1 * n1
    D0 = constitutive_plane_stress(nu)
    g, w = npleg.leggauss(n1)
    Ks = np.zeros((d * d, ne, ne))
    h = 2.0 / d  # cell width in reference coordinates
    for sy in range(d):
        for sx in range(d):
            s = sy * d + sx
            xq = -1.0 + h * sx + 0.5 * h * (g + 1.0)
            yq = -1.0 + h * sy + 0.5 * h * (g + 1.0)
            wq = 0.5 * h * w
            px, dpx = basis_1d(p, xq)
            py, dpy = basis_1d(p, yq)
            for qy in range(n1):
                for qx in range(n1):
                    # physical derivatives: d/dx = 2 d/dxi, d/dy = 2 d/deta
                    B = np.zeros((3, ne))
                    for j in range(n1):
                        for i in range(n1):
                            Nx = 2.0 * dpx[i, qx] * py[j, qy]
                            Ny = 2.0 * px[i, qx] * dpy[j, qy]
                            ax = local_index(p, i, j, 0)
                            ay = local_index(p, i, j, 1)
                            B[0, ax] = Nx
                            B[1, ay] = Ny
                            B[2, ax] = Ny
                            B[2, ay] = Nx
                    # physical area element: dx dy = dxi deta / 4
                    Ks[s] += (wq[qx] * wq[qy] * 0.25) * (B.T @ D0 @ B)
    return Ks
