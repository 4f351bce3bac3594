"""Pins of the oracle's QR-error indicator (Sec. 3.2.3, Eq. (9)) to facts
that do not come from the oracle itself: the hierarchic nesting of the
order-p space in the order-(p+1) space, the variational bound of the
refined energy, invariances of the element problem, and an independent
route to the refined energy through the pseudo-inverse.  (The paper prints
no numerical values of the indicator, only a colour map.)"""

import numpy as np
import pytest

from oracle import oracle_solve, simp_modulus, subcell_stiffness
from oracle.qr import PINNED, element_qr_error, embed_index, qr_error
from paper_1811_09821_amd import problems as P


def rigid(p, a, b, theta):
    """Order-p element DOFs of the rigid motion (a - theta y, b + theta x):
    only the four vertex functions carry it (the hierarchic modes vanish at
    the vertices and a linear field is reproduced by the vertex functions)."""
    u = np.zeros(2 * (p + 1) ** 2)
    for j in range(2):
        for i in range(2):
            aa = j * (p + 1) + i
            u[2 * aa] = a - theta * j
            u[2 * aa + 1] = b + theta * i
    return u


def random_case(p, d, seed, contrast=True):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, d * d)
    if contrast:
        rho[rng.random(d * d) < 0.3] = 0.0
    E = simp_modulus(rho, 1.0, 1e-9, 3.0)
    ue = rng.standard_normal(2 * (p + 1) ** 2)
    return subcell_stiffness(p, d, 0.3), subcell_stiffness(p + 1, d, 0.3), E, ue


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_order_p_block_of_refined_cells_is_order_p_matrix(p, d):
    """Hierarchic basis: K_s^(p+1) restricted to the embedded order-p DOFs is
    K_s^(p) (same functions, both integrated exactly).  Pins embed_index."""
    emb = embed_index(p)
    Kp, Kq = subcell_stiffness(p, d, 0.3), subcell_stiffness(p + 1, d, 0.3)
    sub = Kq[:, emb][:, :, emb]
    assert np.abs(sub - Kp).max() < 1e-13 * np.abs(Kp).max()


@pytest.mark.parametrize("p,d,seed", [(1, 2, 1), (2, 2, 2), (3, 4, 3), (4, 5, 4), (2, 1, 5)])
def test_refined_energy_bounds_and_range(p, d, seed):
    """Variational bound: under the same self-equilibrated load the richer
    space is softer, J^(p+1) >= J^(p), so 0 <= eps < 1."""
    Ksp, Ksq, E, ue = random_case(p, d, seed)
    eps = element_qr_error(Ksp, Ksq, E, ue, p)
    assert -1e-9 <= eps < 1.0, eps


@pytest.mark.parametrize("p,d,seed", [(1, 2, 11), (2, 3, 12), (3, 4, 13), (4, 2, 14)])
def test_independent_of_which_dofs_are_pinned(p, d, seed):
    """The reactions vanish (equilibrated load), so pinning vertex (1,0) x, y
    and vertex (0,1) x instead gives the same eps."""
    Ksp, Ksq, E, ue = random_case(p, d, seed, contrast=False)
    alt = (2, 3, 2 * (p + 1))
    e1 = element_qr_error(Ksp, Ksq, E, ue, p, PINNED)
    e2 = element_qr_error(Ksp, Ksq, E, ue, p, alt)
    assert abs(e1 - e2) < 1e-10, (e1, e2)


@pytest.mark.parametrize("p,d,seed", [(1, 1, 21), (2, 2, 22), (3, 4, 23)])
def test_refined_energy_by_pseudo_inverse(p, d, seed):
    """J^(p+1) = 1/2 f'^T K'^+ f' for the equilibrated load f' (no pinning at
    all): an independent route to eps."""
    Ksp, Ksq, E, ue = random_case(p, d, seed, contrast=False)
    Kp = np.einsum("s,sij->ij", E, Ksp)
    Kq = np.einsum("s,sij->ij", E, Ksq)
    fq = np.zeros(Kq.shape[0])
    fq[embed_index(p)] = Kp @ ue
    Jq = 0.5 * fq @ np.linalg.pinv(Kq, rcond=1e-12) @ fq
    Jp = 0.5 * ue @ Kp @ ue
    assert abs(element_qr_error(Ksp, Ksq, E, ue, p) - (1.0 - Jp / Jq)) < 1e-9


@pytest.mark.parametrize("p,d,seed", [(2, 2, 41), (3, 4, 42)])
def test_invariances(p, d, seed):
    """eps depends neither on the scale of u or E nor on an added rigid
    motion."""
    Ksp, Ksq, E, ue = random_case(p, d, seed, contrast=False)
    e0 = element_qr_error(Ksp, Ksq, E, ue, p)
    assert abs(element_qr_error(Ksp, Ksq, 7.5 * E, -3.0 * ue, p) - e0) < 1e-11
    assert abs(element_qr_error(Ksp, Ksq, E, ue + rigid(p, 5.0, -2.0, 0.4), p) - e0) < 1e-9


def test_uniform_element_constant_strain():
    """A uniform element in a constant-strain state.  The order-(p+1) load
    keeps the order-p nodal load and is zero on the new functions; the
    consistent load of the state on a new edge function L_{p+1} is the
    edge integral of the constant traction against it, which vanishes for
    p + 1 >= 3 (L_k = (P_k - P_{k-2}) / (2k - 1) has zero mean for k >= 3) and
    not for p + 1 = 2; new interior functions get no load (div sigma = 0).
    So eps = 0 for p >= 2 and eps > 0 for p = 1 (nonzero indicator values in
    uniform regions come from the low orders, Sec. 3.2.3)."""
    vals = []
    for p in (1, 2, 3, 4):
        n1 = p + 1
        ue = np.zeros(2 * n1 * n1)
        for j in range(2):
            for i in range(2):
                a = j * n1 + i
                ue[2 * a], ue[2 * a + 1] = 1e-3 * i + 0.4e-3 * j, -0.3e-3 * j
        E = np.ones(4)
        vals.append(element_qr_error(subcell_stiffness(p, 2, 0.3), subcell_stiffness(p + 1, 2, 0.3), E, ue, p))
    assert vals[0] > 0.1, vals
    assert all(abs(v) < 1e-12 for v in vals[1:]), vals


def test_global_layout_and_solution():
    """qr_error on a solved mixed mesh: shape [L, nel] and every value in
    (0, 1) (no element of a loaded mixed mesh is in a state the refined
    functions reproduce exactly)."""
    pr = P.small_mixed(6, 3, seed=51, n_loads=2)
    o = oracle_solve(**pr.oracle_args())
    eps = qr_error(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, o["u"])
    assert eps.shape == (2, pr.nel)
    assert np.all(eps >= -1e-9) and np.all(eps < 1.0)
    assert np.all(eps > 0.0)
