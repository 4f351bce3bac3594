"""GPU: the torch.autograd.Function (densities -> compliances, hand-written
adjoint) and the batched plan over uneven designs."""

import numpy as np
import pytest
import torch

from oracle import oracle_solve, simp_modulus, subcell_stiffness
from oracle.solve import element_dofs_global, rigid_free
from oracle.space import build_space
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_gradcheck_small_mixed(cuda):
    """torch.autograd.gradcheck (central differences, eps 1e-6) of the sum of
    two load cases' compliances on a small mixed mesh."""
    from paper_1811_09821_amd import mto
    from paper_1811_09821_amd.autograd import MTOCompliance

    pr = P.small_mixed(5, 3, seed=61, n_loads=2, sigma=1.5)
    plan = mto.Plan(pr, rtol=1e-13)
    # densities inside (0, 1): the central differences step by 1e-6 both ways
    rho = torch.tensor(np.clip(pr.rho, 0.01, 0.99), device=cuda, requires_grad=True)
    assert torch.autograd.gradcheck(lambda r: MTOCompliance.apply(r, plan), (rho,), eps=1e-6, atol=1e-7,
                                    rtol=1e-5, check_undefined_grad=False)


def test_backward_equals_oracle_gradient(cuda):
    """d(sum of compliances)/drho from backward() against the oracle's
    adjoint gradient, three load cases."""
    from paper_1811_09821_amd import mto
    from paper_1811_09821_amd.autograd import total_compliance

    pr = P.small_mixed(14, 7, seed=62, n_loads=3)
    plan = mto.Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda, requires_grad=True)
    J = total_compliance(rho, plan)
    J.backward()
    o = oracle_solve(**pr.oracle_args())
    assert abs(J.item() - o["c"].sum()) < 1e-8 * o["c"].sum()
    gref = o["g"].sum(axis=0)
    assert rel(rho.grad.cpu().numpy(), gref) < 1e-7


def _identity_difference(pr, u_minus, u_plus, k, h):
    """Cancellation-free central difference of c_l at cell k:
    c(rho+) - c(rho-) = -(E(rho_k + h) - E(rho_k - h)) u-_e^T K_s u+_e, with
    each element vector's rigid motion removed first (K_s annihilates it; in
    FP64 the product would otherwise see the rounding of K_s times the
    ~1e9-times-larger rigid motion of regions hanging on void material)."""
    off = pr.cell_offsets()
    e = int(np.searchsorted(off, k, side="right") - 1)
    s = int(k - off[e])
    space = build_space(pr.nelx, pr.nely, pr.p)
    G = element_dofs_global(space, e)
    Ks = subcell_stiffness(int(pr.p[e]), int(pr.d[e]), pr.nu)[s]
    dE = float(simp_modulus(pr.rho[k] + h, pr.E0, pr.Emin, pr.q) - simp_modulus(pr.rho[k] - h, pr.E0, pr.Emin, pr.q))
    out = []
    for lc in range(u_minus.shape[0]):
        um = rigid_free(np.where(G >= 0, u_minus[lc][np.maximum(G, 0)], 0.0), int(pr.p[e]))
        up = rigid_free(np.where(G >= 0, u_plus[lc][np.maximum(G, 0)], 0.0), int(pr.p[e]))
        out.append(-dE * float(um @ Ks @ up) / (2 * h))
    return np.array(out)


@pytest.fixture(scope="module")
def config5(cuda):
    """The 400 x 200 mixed mesh, volume fraction 0.2, three right-edge loads:
    sum of compliances and its backward gradient (Schwarz-multigrid PCG), and
    the per-load-case u, c and dc/drho of a plain solve of the same plan."""
    from paper_1811_09821_amd import mto
    from paper_1811_09821_amd.autograd import total_compliance

    pr = P.config(5)
    plan = mto.Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda, requires_grad=True)
    J = total_compliance(rho, plan)
    J.backward()
    u, c, g, st = plan.solve(rho.detach())
    print(f"\nconfig 5: {pr.nel} elements, {pr.n_cells} cells, J = {J.item():.12g}, iterations "
          f"{st['iterations']}, restarts {st['restarts']}, true residuals {st['true_rel_residual']}", flush=True)
    per_load = (plan.split_u(u)[0].cpu().numpy(), c.cpu().numpy(), plan.split_g(g)[0].cpu().numpy(), st)
    return pr, plan, J.item(), rho.grad.cpu().numpy(), per_load


def test_autograd_config5_fd_cells(cuda, config5):
    """Backward gradient of the summed compliance against central finite
    differences (step 1e-6) on the 32 cells drawn by default_rng(55), each
    from two GPU solves to the full tolerance (warm-started from the
    unperturbed solution) and the cancellation-free identity."""
    from paper_1811_09821_amd import mto

    pr, plan, J, grad, _ = config5
    rho_np = pr.rho.copy()
    u0, _, _, _ = plan.solve(torch.tensor(rho_np, device=cuda), sensitivities=False)
    cells = np.random.default_rng(55).choice(pr.n_cells, size=32, replace=False)
    h = 1e-6
    plan_fd = mto.Plan(pr)
    for k in cells:
        a = rho_np.copy()
        b = rho_np.copy()
        a[k] += h
        b[k] -= h
        up, _, _, sp = plan_fd.solve(torch.tensor(a, device=cuda), u0=u0, sensitivities=False)
        um, _, _, sm = plan_fd.solve(torch.tensor(b, device=cuda), u0=u0, sensitivities=False)
        assert max(sp["true_rel_residual"]) <= 1e-11 and max(sm["true_rel_residual"]) <= 1e-11
        up = plan_fd.split_u(up)[0].cpu().numpy()
        um = plan_fd.split_u(um)[0].cpu().numpy()
        fd = _identity_difference(pr, um, up, int(k), h).sum()
        print(f"cell {int(k)}: backward {grad[k]:.10e} central difference {fd:.10e}", flush=True)
        # 1e-7 relative to the cell's own derivative, plus the error of the two
        # solves (relative 1e-9 of u) on the largest derivative
        assert abs(fd - grad[k]) <= 1e-7 * abs(grad[k]) + 1e-9 * np.abs(grad).max(), (int(k), fd, grad[k])


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_autograd_config5_oracle_gradient(cuda, config5):
    """The same backward gradient and objective against the oracle's direct
    solve of the 400 x 200 design (about a minute of CPU time), and each load
    case's u (2-norm and max-norm), c and dc/drho (2-norm and max-norm)."""
    pr, plan, J, grad, (u, c, g, st) = config5
    print("\noracle solve of config 5 ...", flush=True)
    o = oracle_solve(**pr.oracle_args())
    print(f"oracle: J = {o['c'].sum():.12g}, c = {o['c']}", flush=True)
    assert abs(J - o["c"].sum()) < 1e-8 * o["c"].sum()
    gref = o["g"].sum(axis=0)
    assert rel(grad, gref) < 1e-7
    assert rel_max(grad, gref) < 1e-7
    assert max(st["true_rel_residual"]) <= 1e-11
    for lc in range(pr.n_load_cases):
        e = (rel(u[lc], o["u"][lc]), rel_max(u[lc], o["u"][lc]), rel(g[lc], o["g"][lc]), rel_max(g[lc], o["g"][lc]))
        print(f"load case {lc}: c {c[lc]:.12g} (oracle {o['c'][lc]:.12g}); u {e[0]:.2e} / {e[1]:.2e}, "
              f"g {e[2]:.2e} / {e[3]:.2e} (2-norm / max-norm)", flush=True)
        assert abs(c[lc] - o["c"][lc]) < 1e-8 * abs(o["c"][lc]), lc
        assert e[0] < 1e-8 and e[1] < 1e-8, (lc, e)
        assert e[2] < 1e-7 and e[3] < 1e-7, (lc, e)


def test_batch_equals_single_instance_plans(cuda):
    """A batch of uneven designs gives, instance by instance, the same bits as
    plans of the single instances (no cross-instance coupling in tiles,
    chunks or reductions), and matches the oracle on the smallest ones."""
    from paper_1811_09821_amd import mto

    prs = P.batch_instances(n=8, first_seed=100, lo=20, hi=80)
    # Jacobi: the multigrid hierarchy of a batch is as deep as its largest
    # instance needs, so a small instance alone gets a shallower (different)
    # preconditioner; the test below covers the multigrid batch.
    plan = mto.Plan(prs, precond=mto.PRECOND_JACOBI)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    us, cs, gs = plan.split_u(u), plan.split_c(c), plan.split_g(g)
    for i, pr in enumerate(prs):
        single = mto.Plan(pr, precond=mto.PRECOND_JACOBI)
        u1, c1, g1, st1 = single.solve(torch.tensor(pr.rho, device=cuda))
        assert torch.equal(us[i].reshape(-1), u1) and torch.equal(cs[i], c1) and torch.equal(gs[i].reshape(-1), g1), i
    order = np.argsort([p.nel for p in prs])[:3]
    for i in order:
        o = oracle_solve(**prs[i].oracle_args())
        assert rel(us[i].cpu().numpy(), o["u"]) < 1e-8
        assert np.all(np.abs(cs[i].cpu().numpy() - o["c"]) <= 1e-8 * np.abs(o["c"]))
        assert rel(gs[i].cpu().numpy(), o["g"]) < 1e-7


def test_batch_multigrid_matches_oracle(cuda):
    """The Schwarz-multigrid batch over the same uneven designs: every
    instance against single-instance plans (to the solve tolerance) and the
    three smallest against the oracle."""
    from paper_1811_09821_amd import mto

    prs = P.batch_instances(n=8, first_seed=100, lo=20, hi=80)
    plan = mto.Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    assert max(st["true_rel_residual"]) <= 1e-11
    us, cs, gs = plan.split_u(u), plan.split_c(c), plan.split_g(g)
    for i, pr in enumerate(prs):
        u1, c1, g1, _ = mto.Plan(pr).solve(torch.tensor(pr.rho, device=cuda))
        assert rel(us[i].reshape(-1).cpu().numpy(), u1.cpu().numpy()) < 1e-9, i
        assert np.all(np.abs(cs[i].cpu().numpy() - c1.cpu().numpy()) <= 1e-9 * np.abs(c1.cpu().numpy())), i
    order = np.argsort([p.nel for p in prs])[:3]
    for i in order:
        o = oracle_solve(**prs[i].oracle_args())
        assert rel(us[i].cpu().numpy(), o["u"]) < 1e-8
        assert np.all(np.abs(cs[i].cpu().numpy() - o["c"]) <= 1e-8 * np.abs(o["c"]))
        assert rel(gs[i].cpu().numpy(), o["g"]) < 1e-7
