"""QR-error indicator of Sec. 3.2.3 (Eq. (9)): for every element, the change
of its strain energy when its shape functions are raised from order p to
p + 1 under the same element load.

Test infrastructure only (see the package docstring).

For element k with order p and displacements u^(p) (its local DOFs taken
from the global solution):
  * K^(p) = sum_s E(rho_s) K_s^(p), K^(p+1) = sum_s E(rho_s) K_s^(p+1)
    (composite integration over the element's density cells);
  * the internal load vector f^(p) = K^(p) u^(p) and J^(p) = 1/2 u^(p)T K^(p) u^(p);
  * f^(p+1): the paper forms it by integrating the interpolated order-p load
    field against the refined shape functions.  Reading: the load field is
    the field f_h of the order-p space whose integrals against the order-p
    functions are the entries of f^(p) (M^(p) c = f^(p), M the element's mass
    matrix, f_h = sum_a c_a N_a); f^(p+1)_b is the integral of f_h N_b over
    the element for every order-(p+1) function N_b.  On the order-p functions
    (which are order-(p+1) functions too) this returns f^(p); the new
    functions get the moments of f_h.  The reading is dimensionally
    consistent and does not depend on the basis;
  * u^(p+1) solves K^(p+1) u = f^(p+1) with 3 DOFs (as many as the rigid
    motions in 2D) copied from u^(p).  Reading: the x and y DOFs of the
    vertex at (0, 0) and the y DOF of the vertex at (1, 0) of the element;
  * J^(p+1) = 1/2 u^(p+1)T K^(p+1) u^(p+1) and eps = 1 - J^(p) / J^(p+1).
    Where J^(p+1) = 0 (a rigid motion) eps is 0.

The load is self-equilibrated (rigid motions lie in the order-p space and
K^(p) annihilates them), so the reactions at the 3 pinned DOFs vanish and the
result does not depend on which 3 DOFs are pinned or on their values; both
energies are unchanged by adding a rigid motion to u^(p).
"""

import numpy as np
from numpy.polynomial import legendre as npleg

from .fem import basis_1d, simp_modulus, subcell_stiffness
from .solve import cell_offsets, element_dofs_global
from .space import build_space

PINNED = (0, 1, 3)  # local DOFs: vertex (0,0) x and y, vertex (1,0) y (2a + c with a = i for j = 0)


def embed_index(p):
    """Local DOF of the order-(p+1) element that carries order-p local DOF
    2 a + c, a = j (p+1) + i: the same tensor-product function, index
    a' = j (p+2) + i."""
    n1 = p + 1
    out = np.empty(2 * n1 * n1, dtype=np.int64)
    for j in range(n1):
        for i in range(n1):
            for c in range(2):
                out[2 * (j * n1 + i) + c] = 2 * (j * (n1 + 1) + i) + c
    return out


def mass_matrix(p):
    """Mass matrix of the order-p element (unit square, vector DOFs 2a + c):
    M[2a + c, 2b + c] = integral of N_a N_b over the element, from the 1D
    mass matrix of basis_1d by a (p + 2)-point Gauss rule (exact)."""
    g, w = npleg.leggauss(p + 2)
    phi, _ = basis_1d(p, g)
    m = 0.5 * (phi * w) @ phi.T  # dx = dxi / 2 on the unit interval
    n1 = p + 1
    scalar = np.einsum("jl,ik->jilk", m, m).reshape(n1 * n1, n1 * n1)  # a = j n1 + i, b = l n1 + k
    M = np.zeros((2 * n1 * n1, 2 * n1 * n1))
    M[0::2, 0::2] = scalar
    M[1::2, 1::2] = scalar
    return M


def refined_load(f, p):
    """The order-(p+1) element load of the order-p load f^(p) (Sec. 3.2.3):
    the load field's coefficients c from M^(p) c = f^(p), then the integrals
    of that field against every order-(p+1) function, M^(p+1)[:, emb] c (the
    order-p functions are the embedded order-(p+1) ones)."""
    Mq = mass_matrix(p + 1)
    emb = embed_index(p)
    c = np.linalg.solve(Mq[np.ix_(emb, emb)], np.asarray(f, dtype=np.float64))
    return Mq[:, emb] @ c


def _quad(K, u):
    """u^T K u with the products accumulated in numpy.longdouble."""
    ul = np.asarray(u, dtype=np.longdouble)
    return ul @ (np.asarray(K, dtype=np.longdouble) @ ul)


def rigid_through(ue, p, pinned):
    """The rigid motion (a - th y, b + th x) of the order-p element that takes
    the values of ue at the 3 pinned local DOFs (vertex DOFs of the order-p
    numbering), as order-p element DOFs (only the vertex functions carry it)."""
    n1 = p + 1
    rows, rhs = [], []
    for k in pinned:
        a = k // 2
        i, j = a % n1, a // n1
        assert i <= 1 and j <= 1, "pinned DOFs must be vertex DOFs"
        rows.append([1.0, 0.0, -float(j)] if k % 2 == 0 else [0.0, 1.0, float(i)])
        rhs.append(ue[k])
    a, b, th = np.linalg.solve(np.array(rows), np.array(rhs))
    r = np.zeros_like(ue)
    for j in range(2):
        for i in range(2):
            k = j * n1 + i
            r[2 * k] = a - th * j
            r[2 * k + 1] = b + th * i
    return r


def element_qr_error(Ks_p, Ks_p1, E, ue, p, pinned=PINNED, rounds=3):
    """eps of Eq. (9) for one element: Ks_p [S, n_e, n_e] and Ks_p1
    [S, n_e', n_e'] the cell matrices at orders p and p+1, E [S] the cell
    moduli, ue [n_e] the element's order-p displacements.

    Both energies are unchanged by adding a rigid motion to u^(p) (K^(p)
    and K^(p+1) annihilate it, the load f^(p) does not see it, and the
    copied values move u^(p+1) by the same motion), so the rigid motion
    through the 3 pinned values is subtracted first and the pinned values
    become zero.  In exact arithmetic this changes nothing; with the cell
    matrices rounded to FP64 the literal u^T K u of an element that moves
    almost rigidly (|u| >> |u - rigid|) would carry an error of relative size
    eps_mach (|u| / |u - rigid|)^2.  The energies are accumulated in
    numpy.longdouble and the element solve is refined against a longdouble
    residual (as the global solve of this package is)."""
    Kp = np.einsum("s,sij->ij", E, Ks_p)
    Kq = np.einsum("s,sij->ij", E, Ks_p1)
    ud = ue - rigid_through(ue, p, pinned)
    f = (np.asarray(Kp, dtype=np.longdouble) @ np.asarray(ud, dtype=np.longdouble)).astype(np.float64)
    Jp = 0.5 * _quad(Kp, ud)
    emb = embed_index(p)
    nq = Kq.shape[0]
    fq = refined_load(f, p)
    pin = np.array([emb[k] for k in pinned])
    free = np.setdiff1d(np.arange(nq), pin)
    uq = np.zeros(nq)  # the pinned values of u - rigid are zero
    Kff = Kq[np.ix_(free, free)]
    for _ in range(rounds):
        r = (np.asarray(fq[free], dtype=np.longdouble)
             - np.asarray(Kq[free], dtype=np.longdouble) @ np.asarray(uq, dtype=np.longdouble))
        uq[free] += np.linalg.solve(Kff, r.astype(np.float64))
    Jq = 0.5 * _quad(Kq, uq)
    return 0.0 if Jq <= 0.0 else float(1.0 - Jp / Jq)


def qr_error(nelx, nely, p, d, rho, u, E0=1.0, Emin=1e-9, q=3.0, nu=0.3):
    """eps [L, nel] for every load case of the global displacements u
    [L, n_dof] (the oracle solve's layout)."""
    p = np.asarray(p, dtype=np.int64).ravel()
    d = np.asarray(d, dtype=np.int64).ravel()
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    space = build_space(nelx, nely, p)
    off = cell_offsets(d)
    E = simp_modulus(np.asarray(rho, dtype=np.float64), E0, Emin, q)
    cache = {}
    out = np.zeros((u.shape[0], nelx * nely))
    for e in range(nelx * nely):
        pe, de = int(p[e]), int(d[e])
        for key in ((pe, de), (pe + 1, de)):
            if key not in cache:
                cache[key] = subcell_stiffness(key[0], key[1], nu)
        G = element_dofs_global(space, e)
        Ee = E[off[e]:off[e + 1]]
        for lc in range(u.shape[0]):
            ue = np.where(G >= 0, u[lc][np.maximum(G, 0)], 0.0)
            out[lc, e] = element_qr_error(cache[(pe, de)], cache[(pe + 1, de)], Ee, ue, pe)
    return out
