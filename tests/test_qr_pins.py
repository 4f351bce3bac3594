"""Pins of the oracle's QR-error indicator (Sec. 3.2.3, Eq. (9)) to facts
that do not come from the oracle itself: the hierarchic nesting of the
order-p space in the order-(p+1) space, the variational bound of the
refined energy, invariances of the element problem, and independent routes
to the refined load and energy: a known polynomial load field whose
integrals against the order-p and order-(p+1) functions are taken exactly
(the paper forms the refined load by integrating the interpolated load
field against the refined shape functions), with exact rational solves for
p = 1, 2 and pseudo-inverse energies for p = 3, 4, and an exact rational
evaluation of a near-rigid element that does not subtract its rigid
motion.  (The paper prints no numerical values of the indicator, only a
colour map and the range 0.3-0.5 of fully solid or void Q2 elements.)"""

from fractions import Fraction as F

import numpy as np
import pytest

from oracle import oracle_solve, simp_modulus, subcell_stiffness
from oracle.qr import PINNED, element_qr_error, embed_index, qr_error, refined_load
from paper_1811_09821_amd import problems as P
from tests.exact_rational import (mass_1d_exact, moments_exact, pinned_solve_exact, solve_exact,
                                  subcell_stiffness_exact)


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


@pytest.mark.parametrize("p,d,seed", [(2, 2, 41), (3, 4, 42)])
def test_invariances(p, d, seed):
    """eps depends neither on the scale of u or E nor on an added rigid
    motion."""
    Ksp, Ksq, E, ue = random_case(p, d, seed, contrast=False)
    e0 = element_qr_error(Ksp, Ksq, E, ue, p)
    assert abs(element_qr_error(Ksp, Ksq, 7.5 * E, -3.0 * ue, p) - e0) < 1e-11
    assert abs(element_qr_error(Ksp, Ksq, E, ue + rigid(p, 5.0, -2.0, 0.4), p) - e0) < 1e-9


def equilibrated_field(p, seed):
    """Random rational coefficients beta[c][i][j] of a load field b in Q_p
    (b_c = sum beta xi^i eta^j, reference coordinates), adjusted so that its
    net force and its moment about the element centre vanish (a load the
    element can carry without supports)."""
    rng = np.random.default_rng(seed)
    n1 = p + 1
    beta = [[[F(int(rng.integers(-9, 10)), int(rng.integers(1, 5))) for _ in range(n1)] for _ in range(n1)]
            for _ in range(2)]
    mu = [F(1, m + 1) if m % 2 == 0 else F(0) for m in range(n1 + 2)]  # mean of xi^m over [-1, 1]
    for c in range(2):  # net force: the constant coefficient absorbs it
        tot = sum(beta[c][i][j] * mu[i] * mu[j] for i in range(n1) for j in range(n1))
        beta[c][0][0] -= tot
    # moment about the centre ~ mean of xi b_y - eta b_x: the xi coefficient of b_y absorbs it
    mom = (sum(beta[1][i][j] * mu[i + 1] * mu[j] for i in range(n1) for j in range(n1))
           - sum(beta[0][i][j] * mu[i] * mu[j + 1] for i in range(n1) for j in range(n1)))
    beta[1][1][0] -= mom / mu[2]
    return beta


def exact_moduli(d, seed):
    rng = np.random.default_rng(seed)
    rho = [F(int(rng.integers(0, 11)), 10) for _ in range(d * d)]
    emin = F(1, 10 ** 9)
    return [emin + r ** 3 * (1 - emin) for r in rho]


def exact_matrix(E, Ks):
    n = len(Ks[0])
    return [[sum(E[s] * Ks[s][i][j] for s in range(len(E))) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_refined_load_of_a_known_field(p):
    """The refined load is the integral of the load field against the refined
    functions: for f^(p) = the exact integrals of a known field b in Q_p
    against the order-p functions, the oracle's transfer returns the exact
    integrals of b against the order-(p+1) functions.  The new functions get
    nonzero loads, so a transfer that puts zero there fails."""
    beta = equilibrated_field(p, 100 + p)
    f = np.array([float(v) for v in moments_exact(beta, p)])
    fq = np.array([float(v) for v in moments_exact(beta, p + 1)])
    got = refined_load(f, p)
    assert np.abs(got - fq).max() < 1e-13 * np.abs(fq).max()
    new = np.setdiff1d(np.arange(fq.size), embed_index(p))
    assert np.abs(fq[new]).max() > 1e-3 * np.abs(fq).max()


@pytest.mark.parametrize("p,d,seed", [(1, 2, 31), (2, 2, 32)])
def test_qr_error_exact_rational_known_field(p, d, seed):
    """End to end in exact rational arithmetic: an equilibrated known load
    field, u^(p) from the exactly solved order-p element problem (three DOFs
    pinned, no reactions), u^(p+1) from the order-(p+1) problem under the
    field's exact refined integrals, eps = 1 - J^(p) / J^(p+1) exactly; the
    oracle, given the same moduli and u^(p), agrees to 1e-10."""
    beta = equilibrated_field(p, seed)
    E = exact_moduli(d, seed)
    Kp = exact_matrix(E, subcell_stiffness_exact(p, d))
    Kq = exact_matrix(E, subcell_stiffness_exact(p + 1, d))
    f = moments_exact(beta, p)
    fq = moments_exact(beta, p + 1)
    ue = pinned_solve_exact(Kp, f, list(PINNED), [F(0)] * 3)
    # equilibrated load: the pinned rows need no reaction
    assert all(sum(Kp[k][j] * ue[j] for j in range(len(ue))) == f[k] for k in PINNED)
    emb = embed_index(p)
    uq = pinned_solve_exact(Kq, fq, [int(emb[k]) for k in PINNED], [F(0)] * 3)
    Jp = sum(a * b for a, b in zip(ue, f)) / 2
    Jq = sum(a * b for a, b in zip(uq, fq)) / 2
    eps_exact = 1 - Jp / Jq
    got = element_qr_error(subcell_stiffness(p, d, 0.3), subcell_stiffness(p + 1, d, 0.3),
                           np.array([float(e) for e in E]), np.array([float(v) for v in ue]), p)
    assert abs(got - float(eps_exact)) < 1e-10, (got, float(eps_exact))
    assert 0.0 < float(eps_exact) < 1.0


@pytest.mark.parametrize("p,d,seed", [(3, 2, 41), (4, 3, 42)])
def test_qr_error_known_field_pseudo_inverse(p, d, seed):
    """The same for p = 3, 4 in floating point by another route: exact load
    integrals of the known field, u^(p) = K^(p)+ f^(p) and J^(p+1) =
    f'^T K^(p+1)+ f' / 2 by pseudo-inverses (no pinning, no mass matrix)."""
    beta = equilibrated_field(p, seed)
    E = simp_modulus(np.random.default_rng(seed).uniform(0.0, 1.0, d * d), 1.0, 1e-9, 3.0)
    Ksp, Ksq = subcell_stiffness(p, d, 0.3), subcell_stiffness(p + 1, d, 0.3)
    Kp = np.einsum("s,sij->ij", E, Ksp)
    Kq = np.einsum("s,sij->ij", E, Ksq)
    f = np.array([float(v) for v in moments_exact(beta, p)])
    fq = np.array([float(v) for v in moments_exact(beta, p + 1)])
    ue = np.linalg.pinv(Kp, rcond=1e-13) @ f
    Jp = 0.5 * f @ ue
    Jq = 0.5 * fq @ np.linalg.pinv(Kq, rcond=1e-13) @ fq
    got = element_qr_error(Ksp, Ksq, E, ue, p)
    assert abs(got - (1.0 - Jp / Jq)) < 1e-8, (got, 1.0 - Jp / Jq)


def test_near_rigid_element_exact_rational():
    """A p = 1 element moving almost rigidly (rigid part 1e6, deformation of
    order 1), evaluated exactly in rationals on the very same FP64 values of
    u, with the paper's literal procedure: f = K u, the refined load by the
    exact mass matrices, the 3 pinned values copied, no rigid motion
    subtracted.  The oracle (which subtracts it in floating point) agrees to
    1e-8, while a plain FP64 evaluation of u^T K u is off by far more."""
    p, d, seed = 1, 2, 51
    rng = np.random.default_rng(seed)
    E = exact_moduli(d, seed)
    Ksp_e, Ksq_e = subcell_stiffness_exact(p, d), subcell_stiffness_exact(p + 1, d)
    Kp, Kq = exact_matrix(E, Ksp_e), exact_matrix(E, Ksq_e)
    n1 = p + 1
    ue_f = rng.standard_normal(2 * n1 * n1)
    for j in range(2):
        for i in range(2):  # rigid motion (a - th y, b + th x) scaled by 1e6
            a = j * n1 + i
            ue_f[2 * a] += 1e6 * (0.3 - 0.25 * j)
            ue_f[2 * a + 1] += 1e6 * (-0.7 + 0.25 * i)
    ue = [F(v) for v in ue_f]  # the same numbers, exactly
    f = [sum(Kp[i][j] * ue[j] for j in range(len(ue))) for i in range(len(ue))]
    Jp = sum(a * b for a, b in zip(ue, f)) / 2
    # refined load: coefficients of the load field (M^(p) c = f), integrated against the order-(p+1) functions
    m1, m2 = mass_1d_exact(p), mass_1d_exact(p + 1)

    def vec_mass(m, n):
        M = [[F(0)] * (2 * n * n) for _ in range(2 * n * n)]
        for j in range(n):
            for i in range(n):
                for l in range(n):
                    for k in range(n):
                        for c in range(2):
                            M[2 * (j * n + i) + c][2 * (l * n + k) + c] = m[i][k] * m[j][l]
        return M

    Mp, Mq = vec_mass(m1, n1), vec_mass(m2, n1 + 1)
    emb = [int(v) for v in embed_index(p)]
    coef = solve_exact(Mp, f)
    fq = [sum(Mq[r][emb[a]] * coef[a] for a in range(len(emb))) for r in range(len(Mq))]
    pins = [emb[k] for k in PINNED]
    uq = pinned_solve_exact(Kq, fq, pins, [ue[k] for k in PINNED])
    Jq = sum(uq[i] * sum(Kq[i][j] * uq[j] for j in range(len(uq))) for i in range(len(uq))) / 2
    eps_exact = float(1 - Jp / Jq)
    Ef = np.array([float(e) for e in E])
    got = element_qr_error(subcell_stiffness(p, d, 0.3), subcell_stiffness(p + 1, d, 0.3), Ef, ue_f, p)
    assert abs(got - eps_exact) < 1e-8, (got, eps_exact)
    naive = 0.5 * ue_f @ np.einsum("s,sij->ij", Ef, subcell_stiffness(p, d, 0.3)) @ ue_f
    assert abs(naive - float(Jp)) > 1e-9 * float(Jp)  # the subtraction is what makes the oracle exact here


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
