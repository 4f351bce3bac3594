"""Pins of the oracle's compliant-mechanism path (Sec. 4.1, force inverter:
Eq. (1) with z = e_out, ground springs k_in and k_out): the spring
assembly against the Sherman-Morrison rank-one update, Maxwell-Betti
reciprocity between the input and the adjoint load case, the adjoint
sensitivity against central differences of J, and the reduction of the
bilinear sensitivity to the compliance sensitivity."""

import numpy as np
import pytest

from oracle import oracle_solve
from oracle.mechanism import bilinear_sensitivity, global_dof, mechanism
from paper_1811_09821_amd import problems as P


def small_inverter(seed=7):
    return P.force_inverter(6, 3, p=2, d=2, volfrac=0.5, seed=seed, sigma=1.5)


def test_spring_is_a_rank_one_update():
    """u with a ground spring k at DOF i equals u - k u_i / (1 + k G_ii) G e_i,
    with G the inverse of K without the spring (Sherman-Morrison); on a
    clamped cantilever, where K alone is well conditioned."""
    pr = P.small_mixed(6, 3, seed=52)
    vx, vy = pr.nelx, 1
    i_dof = global_dof(pr.nelx, vx, vy, 0)
    base = dict(pr.oracle_args(), loads=[pr.loads[0], (vx, vy, 1.0, 0.0, 1)], n_load_cases=2)
    o = oracle_solve(**base)
    u, Gi = o["u"][0], o["u"][1]  # Gi = K^-1 e_i (unit load at DOF i)
    k = 0.37
    withk = oracle_solve(**dict(base, springs=[(vx, vy, 0, k)]))
    ref = u - k * u[i_dof] / (1.0 + k * Gi[i_dof]) * Gi
    assert np.abs(withk["u"][0] - ref).max() < 1e-10 * np.abs(ref).max()


def test_reciprocity_of_input_and_adjoint_cases():
    """Maxwell-Betti: the output displacement under f_in equals f_in times the
    input displacement under the unit output load."""
    pr = small_inverter()
    o = oracle_solve(**pr.oracle_args())
    f_in = pr.loads[0][2]
    u_out = o["u"][0][global_dof(pr.nelx, *pr.out_dof)]
    lam_in = o["u"][1][global_dof(pr.nelx, *pr.in_dof)]
    assert abs(u_out - f_in * lam_in) < 1e-12 * abs(u_out)


@pytest.mark.parametrize("seed", [7, 8])
def test_adjoint_sensitivity_matches_central_differences(seed):
    pr = small_inverter(seed)
    J, g, _ = mechanism(pr)
    rng = np.random.default_rng(seed)
    h = 1e-6
    for k in rng.choice(pr.n_cells, size=6, replace=False):
        rp, rm = pr.rho.copy(), pr.rho.copy()
        rp[k] += h
        rm[k] -= h
        prp, prm = small_inverter(seed), small_inverter(seed)
        prp.rho, prm.rho = rp, rm
        fd = (mechanism(prp)[0] - mechanism(prm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g).max(), 1e-12), (k, fd, g[k])


def test_bilinear_with_equal_vectors_is_the_compliance_sensitivity():
    pr = P.small_mixed(6, 3, seed=51)
    o = oracle_solve(**pr.oracle_args())
    u = o["u"][0]
    g = bilinear_sensitivity(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, u, u)
    assert np.abs(g - o["g"][0]).max() <= 1e-12 * np.abs(o["g"][0]).max()


def test_spring_on_a_supported_dof_is_rejected():
    pr = small_inverter()
    with pytest.raises(ValueError):
        oracle_solve(**dict(pr.oracle_args(), springs=[(0, pr.nely, 0, 1.0)]))
