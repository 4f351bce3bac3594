"""GPU parity of the compliant-mechanism path (Sec. 4.1, force inverter:
J = z^T u with z = e_out, ground springs k_in = 1 and k_out = 0.001) against
the oracle.

Tolerances (written here): u and c within 1e-8 relative (as for the
compliance step), J within 1e-8 relative, dJ/drho within 1e-7 (norm-wise);
the solves run to a relative residual of 1e-13, since the soft output spring
(k_out = 0.001) on a random design conditions the inverter worse than the
compliance configurations (at 1e-11 the 80 x 40 case reaches 2.2e-8 in u);
the spring-augmented product K x and the bilinear sensitivity for the same
inputs within 1e-12 (one FP64 evaluation in a different summation order).
"""

import numpy as np
import pytest
import torch

from oracle import oracle_solve
from oracle.mechanism import bilinear_sensitivity, global_dof, mechanism
from oracle.solve import assemble, spring_matrix
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

CASES = {
    "small_p2d2": lambda: P.force_inverter(6, 3, p=2, d=2, volfrac=0.5, seed=7, sigma=1.5),
    "paper_40x20_p2d4": lambda: P.force_inverter(40, 20, p=2, d=4, volfrac=0.45, seed=7),
    "p3d4_80x40": lambda: P.force_inverter(80, 40, p=3, d=4, volfrac=0.45, seed=8, sigma=6.0),
}


def mto():
    from paper_1811_09821_amd import mto as m

    return m


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("key", ["small_p2d2", "paper_40x20_p2d4"])
def test_spring_product(cuda, key):
    """y = (K + springs) x on the free DOFs against the assembled oracle."""
    pr = CASES[key]()
    plan = mto().Plan(pr)
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    K = (K + spring_matrix(space, pr.springs)).tocsr()
    o = oracle_solve(**pr.oracle_args())
    free = o["free"]
    x = np.random.default_rng(3).standard_normal((pr.n_load_cases, space.n_dof))
    x[:, ~free] = 0.0
    y = plan.apply_stiffness(torch.tensor(pr.rho, device=cuda), torch.tensor(x.ravel(), device=cuda))
    y = y.cpu().numpy().reshape(pr.n_load_cases, space.n_dof)
    for lc in range(pr.n_load_cases):
        ref = K @ x[lc]
        ref[~free] = 0.0
        assert rel(y[lc], ref) < 1e-12


@pytest.mark.parametrize("key", sorted(CASES))
def test_mechanism_solve_and_adjoint(cuda, key):
    """Both load cases (input force and adjoint unit load), J = u_out, and
    dJ/drho = -E' lam_e^T K_s u_e, each side from its own solve."""
    pr = CASES[key]()
    m = mto()
    plan = m.Plan(pr, rtol=1e-13)
    rho = torch.tensor(pr.rho, device=cuda)
    u, c, _, st = plan.solve(rho, sensitivities=False)
    J_ref, g_ref, o = mechanism(pr)
    uu = plan.split_u(u)[0].cpu().numpy()
    for lc in range(2):
        assert rel(uu[lc], o["u"][lc]) < 1e-8, (key, lc, rel(uu[lc], o["u"][lc]))
    cc = c.cpu().numpy()
    assert np.all(np.abs(cc - o["c"]) <= 1e-8 * np.abs(o["c"]))
    out = global_dof(pr.nelx, *pr.out_dof)
    J = float(uu[0][out])
    assert abs(J - J_ref) <= 1e-8 * abs(J_ref)
    n = plan.instances[0]["n_dof"]
    lam = torch.cat([u[n:2 * n], u[:n]])
    g = plan.adjoint_sensitivity(rho, u, lam)[:pr.n_cells].cpu().numpy()
    assert rel(g, g_ref) < 1e-7, (key, rel(g, g_ref))
    print(f"\n{key}: J = {J:.10g}, iterations {st['iterations']}", flush=True)


def test_adjoint_sensitivity_same_inputs(cuda):
    """The bilinear kernel on the oracle's u and lam."""
    pr = CASES["paper_40x20_p2d4"]()
    o = oracle_solve(**pr.oracle_args())
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    u = torch.tensor(o["u"].ravel(), device=cuda)
    lam = torch.tensor(o["u"][::-1].copy().ravel(), device=cuda)
    g = plan.adjoint_sensitivity(rho, u, lam).cpu().numpy().reshape(2, pr.n_cells)
    for lc in range(2):
        ref = bilinear_sensitivity(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, o["u"][lc], o["u"][1 - lc])
        assert np.abs(g[lc] - ref).max() <= 1e-12 * np.abs(ref).max()
    # with lam = u it is the compliance sensitivity
    gc = plan.adjoint_sensitivity(rho, u, u).cpu().numpy().reshape(2, pr.n_cells)
    assert np.abs(gc - plan.sensitivity(rho, u).cpu().numpy().reshape(2, pr.n_cells)).max() == 0.0


def test_mechanism_autograd(cuda):
    """MTOMechanism: forward J and backward dJ/drho against the oracle."""
    from paper_1811_09821_amd.autograd import MTOMechanism

    pr = CASES["paper_40x20_p2d4"]()
    plan = mto().Plan(pr, rtol=1e-13)
    rho = torch.tensor(pr.rho, device=cuda, requires_grad=True)
    out = global_dof(pr.nelx, *pr.out_dof)
    J = MTOMechanism.apply(rho, plan, out)
    J.backward()
    J_ref, g_ref, _ = mechanism(pr)
    assert abs(J.item() - J_ref) <= 1e-8 * abs(J_ref)
    assert rel(rho.grad.cpu().numpy(), g_ref) < 1e-7
