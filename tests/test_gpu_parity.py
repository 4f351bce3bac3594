"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.

Tolerances (relative, norm-wise, written here): u and c within 1e-8 (u in
both the 2-norm and the max-norm ratios), dc/drho within 1e-7 (both ratios),
with PCG run to a relative residual of 1e-11.  The element contraction itself (no solve) is
compared at 1e-13: it is one FP64 product with a different summation order.
"""

import numpy as np
import pytest
import torch

from oracle import oracle_solve, simp_modulus_derivative, subcell_stiffness
from oracle.solve import assemble, element_dofs_global, free_mask
from oracle.space import build_space
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

U_TOL, C_TOL, G_TOL = 1e-8, 1e-8, 1e-7


def mto():
    from paper_1811_09821_amd import mto as m

    return m


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def rel_max(a, b):
    mb = np.abs(b).max()
    return float(np.abs(a - b).max() / mb) if mb > 0 else float(np.abs(a).max())


def oracle_sens_given_u(pr, u_full):
    """Oracle formula g = -E'(rho) u_e^T K_s u_e for given displacements."""
    space = build_space(pr.nelx, pr.nely, pr.p)
    off = pr.cell_offsets()
    dE = simp_modulus_derivative(pr.rho, pr.E0, pr.Emin, pr.q)
    L = u_full.shape[0]
    g = np.zeros((L, pr.n_cells))
    cache = {}
    for e in range(pr.nel):
        key = (int(pr.p[e]), int(pr.d[e]))
        if key not in cache:
            cache[key] = subcell_stiffness(key[0], key[1], pr.nu)
        Ks = cache[key]
        G = element_dofs_global(space, e)
        for lc in range(L):
            ue = np.where(G >= 0, u_full[lc][np.maximum(G, 0)], 0.0)
            g[lc, off[e]:off[e + 1]] = -dE[off[e]:off[e + 1]] * np.einsum("i,sij,j->s", ue, Ks, ue)
    return g


def check_solution(plan, prs, u, c, g, stats):
    us, cs, gs = plan.split_u(u), plan.split_c(c), plan.split_g(g)
    for i, pr in enumerate(prs):
        o = oracle_solve(**pr.oracle_args())
        uu = us[i].cpu().numpy()
        assert rel(uu, o["u"]) < U_TOL, (pr.name, rel(uu, o["u"]))
        for lc in range(pr.n_load_cases):  # small edge and interior modes must not hide errors
            assert rel_max(uu[lc], o["u"][lc]) < U_TOL, (pr.name, lc, rel_max(uu[lc], o["u"][lc]))
        cc = cs[i].cpu().numpy()
        assert np.all(np.abs(cc - o["c"]) <= C_TOL * np.abs(o["c"])), (pr.name, cc, o["c"])
        gg = gs[i].cpu().numpy()
        for lc in range(pr.n_load_cases):
            assert rel(gg[lc], o["g"][lc]) < G_TOL, (pr.name, lc, rel(gg[lc], o["g"][lc]))
            assert rel_max(gg[lc], o["g"][lc]) < G_TOL, (pr.name, lc, rel_max(gg[lc], o["g"][lc]))
    assert stats["status"] == 0, stats


GROUPS = [(p, d) for p in (1, 2, 3, 4) for d in range(1, 9)]  # every (p, d) the library accepts


@pytest.mark.parametrize("p,d", GROUPS)
def test_matvec_every_group(cuda, p, d):
    """y = K x (element contraction + slot assembly) for all 32 (p, d) groups,
    on a 7 x 5 mesh (35 elements: several 16-column tiles and a ragged tail)
    with several tile widths and density-cell splits across waves, and for
    p >= 3 the LDS-staged contraction (ks = 0: one 64- or 128-column tile,
    ragged); ks = -1 is the fused one-launch product."""
    pr = P.uniform_random(7, 5, p, d, seed=100 + 10 * p + d)
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    free = free_mask(space, pr.supports)
    x = np.random.default_rng(p * d).standard_normal(space.n_dof)
    x[~free] = 0.0
    yref = K @ x
    yref[~free] = 0.0
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    xt = torch.tensor(x, device=cuda)
    shapes = [(1, 1), (2, 2), (1, 4), (4, 1), (1, 8), (1, -1)] + ([(1, 0), (2, 0)] if p >= 3 else [])
    for ncol, ks in shapes:
        plan.set_tile(ncol, ks)
        y = plan.apply_stiffness(rho, xt).cpu().numpy()
        assert rel(y, yref) < 1e-13, (p, d, ncol, ks, rel(y, yref))


@pytest.mark.parametrize("path", [0, 1])
def test_matvec_mixed_and_diag(cuda, path):
    """Mixed mesh (minimum-rule edges, all four groups of the dp rule) and the
    Jacobi diagonal, MFMA and plain comparison paths."""
    pr = P.small_mixed(13, 7, seed=5)
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    free = free_mask(space, pr.supports)
    x = np.random.default_rng(1).standard_normal(space.n_dof)
    x[~free] = 0.0
    yref = K @ x
    yref[~free] = 0.0
    plan = mto().Plan(pr, kernel_path=path)
    rho = torch.tensor(pr.rho, device=cuda)
    y = plan.apply_stiffness(rho, torch.tensor(x, device=cuda)).cpu().numpy()
    assert rel(y, yref) < 1e-13
    dg = plan.jacobi_diagonal(rho).cpu().numpy()
    dref = K.diagonal().copy()
    dref[~free] = 0.0
    assert rel(dg, dref) < 1e-14


def random_orders_mesh():
    """8 x 5 mesh with p in 1..4 and d in 1..8 drawn per element, unsmoothed:
    order jumps of 3 across edges and 26 (p, d) groups of one to four
    elements each (every element tile ragged)."""
    rng = np.random.default_rng(61)
    return P.uniform_random(8, 5, rng.integers(1, 5, 40), rng.integers(1, 9, 40), 61)


@pytest.mark.parametrize("path,fused", [(0, False), (0, True), (1, False)])
def test_matvec_random_orders(cuda, path, fused):
    """26 (p, d) groups of one to four elements: per-group launches, the fused
    one-launch product (tiles of all groups in one grid) and the plain path."""
    pr = random_orders_mesh()
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    free = free_mask(space, pr.supports)
    x = np.random.default_rng(2).standard_normal(space.n_dof)
    x[~free] = 0.0
    yref = K @ x
    yref[~free] = 0.0
    plan = mto().Plan(pr, kernel_path=path)
    if fused:
        plan.set_tile(1, -1)
    y = plan.apply_stiffness(torch.tensor(pr.rho, device=cuda), torch.tensor(x, device=cuda)).cpu().numpy()
    assert rel(y, yref) < 1e-13


@pytest.mark.parametrize("precond", [0, 2])
def test_solve_random_orders(cuda, precond):
    """The unsmoothed mesh above solved with both preconditioners."""
    prs = [random_orders_mesh()]
    plan = mto().Plan(prs, precond=precond)
    u, c, g, st = plan.solve(torch.tensor(prs[0].rho, device=cuda))
    check_solution(plan, prs, u, c, g, st)


def test_sensitivity_kernel_given_u(cuda):
    """g = -E' u_e^T K_s u_e from given (random) displacements, mixed mesh,
    two load cases."""
    pr = P.small_mixed(11, 6, seed=8, n_loads=2)
    space = build_space(pr.nelx, pr.nely, pr.p)
    free = free_mask(space, pr.supports)
    u = np.random.default_rng(2).standard_normal((2, space.n_dof))
    u[:, ~free] = 0.0
    gref = oracle_sens_given_u(pr, u)
    plan = mto().Plan(pr)
    for ncol in (1, 2, 4):
        plan.set_tile(ncol)
        g = plan.sensitivity(torch.tensor(pr.rho, device=cuda), torch.tensor(u.ravel(), device=cuda))
        g = g.cpu().numpy().reshape(2, -1)
        assert rel(g, gref) < 1e-12
        assert rel_max(g, gref) < 1e-12


CASES = {
    "mbb20x10": lambda: [P.mbb_20x10()],
    "uniform_p1d3": lambda: [P.uniform_random(9, 4, 1, 3, 1)],
    "uniform_p2d2": lambda: [P.uniform_random(9, 4, 2, 2, 2)],
    "uniform_p3d4": lambda: [P.uniform_random(8, 4, 3, 4, 3)],
    "uniform_p4d5": lambda: [P.uniform_random(6, 3, 4, 5, 4)],
    "mixed16x8": lambda: [P.small_mixed(16, 8, seed=3)],
    "mixed_3loads": lambda: [P.small_mixed(14, 7, seed=4, n_loads=3)],
    "cantilever_field": lambda: [P.cantilever_uniform(24, 12, 3, 4, sigma=3.0, volfrac=0.4, seed=2)],
    "uniform_p4d8_max": lambda: [P.uniform_random(6, 3, 4, 8, 17)],
}


@pytest.mark.parametrize("precond", [0, 2])
@pytest.mark.parametrize("name", sorted(CASES))
def test_solve_parity(cuda, name, precond):
    """u, c and dc/drho against the oracle (direct solve), Jacobi (0) and
    Schwarz-multigrid (2) preconditioned."""
    prs = CASES[name]()
    plan = mto().Plan(prs, precond=precond)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


@pytest.mark.parametrize("precond", [1, 2])
@pytest.mark.parametrize("name", ["mbb20x10", "mixed_3loads", "uniform_p4d5", "cantilever_field"])
def test_solve_parity_multigrid(cuda, name, precond):
    """The multigrid-preconditioned PCG (l1-Jacobi or element-block Schwarz
    smoothing on the hierarchic level) reaches the same solution."""
    prs = CASES[name]()
    plan = mto().Plan(prs, precond=precond)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_schwarz_multigrid_cuts_iterations(cuda):
    """On a p = 3, d = 4 cantilever with a smoothed density field the
    element-block Schwarz V-cycle needs a small fraction of the Jacobi
    iterations, and both reach the same solution."""
    m = mto()
    pr = P.cantilever_uniform(40, 20, 3, 4, sigma=2.0, volfrac=0.4, seed=7)
    rho = torch.tensor(pr.rho, device=cuda)
    uj, cj, gj, sj = m.Plan(pr, precond=m.PRECOND_JACOBI).solve(rho)
    us, cs, gs, ss = m.Plan(pr, precond=m.PRECOND_MG_ASM).solve(rho)
    print(f"\niterations: Jacobi {sj['iterations']}, Schwarz multigrid {ss['iterations']}", flush=True)
    assert max(ss["iterations"]) * 8 < max(sj["iterations"])
    assert rel(us.cpu().numpy(), uj.cpu().numpy()) < 1e-9
    assert abs(cs.item() - cj.item()) <= 1e-9 * abs(cj.item())


@pytest.mark.parametrize("coarse_max", [0, 200])
def test_widest_coarse_band_and_deeper_hierarchy(cuda, coarse_max):
    """A 74 x 74 mesh coarsens to a 37 x 37 grid whose band width, 79, is the
    widest the coarsest-level Cholesky takes (its LDS window then exceeds
    64 KB); with mg_coarse_max = 200 the hierarchy coarsens three levels
    further.  Both Schwarz-multigrid solves match the Jacobi-preconditioned
    solve of the same system."""
    m = mto()
    pr = P.uniform_random(74, 74, 1, 1, seed=31)
    rho = torch.tensor(pr.rho, device=cuda)
    uj, cj, gj, sj = m.Plan(pr, precond=m.PRECOND_JACOBI).solve(rho)
    us, cs, gs, ss = m.Plan(pr, precond=m.PRECOND_MG_ASM, mg_coarse_max=coarse_max).solve(rho)
    print(f"\niterations: Jacobi {sj['iterations']}, Schwarz multigrid {ss['iterations']}", flush=True)
    assert ss["status"] == 0 and sj["status"] == 0
    assert max(ss["iterations"]) < max(sj["iterations"])
    assert rel(us.cpu().numpy(), uj.cpu().numpy()) < 1e-9
    assert abs(cs.item() - cj.item()) <= 1e-9 * abs(cj.item())
    assert rel(gs.cpu().numpy(), gj.cpu().numpy()) < 1e-8


def test_solve_parity_plain_path(cuda):
    prs = [P.small_mixed(12, 6, seed=6, n_loads=2)]
    plan = mto().Plan(prs, kernel_path=1)
    rho = torch.tensor(prs[0].rho, device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_batch_parity_uneven_instances(cuda):
    """Several independent designs of uneven size, order mix and load count in
    one plan: each instance against its own oracle solve."""
    prs = [P.small_mixed(10, 5, seed=21, n_loads=1), P.mbb_20x10(),
           P.small_mixed(18, 9, seed=22, n_loads=3), P.uniform_random(5, 3, 4, 5, 23),
           P.small_mixed(8, 4, seed=24, n_loads=2)]
    plan = mto().Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


DEGENERATE = {
    "single_p1": lambda: [P.uniform_random(1, 1, 1, 3, 21)],
    "single_p4": lambda: [P.uniform_random(1, 1, 4, 3, 24)],
    "strip12x1_p4": lambda: [P.uniform_random(12, 1, 4, 2, 31)],
    "column1x9_p3": lambda: [P.uniform_random(1, 9, 3, 2, 32, loads=[(1, 9, 0.0, -1.0, 0)])],
}


@pytest.mark.parametrize("precond", [0, 2])
@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_degenerate_meshes(cuda, name, precond):
    """Meshes one element wide or high: a single element (4 free DOFs at
    p = 1, one element tile of 16 rows, an 8-DOF coarsest grid whose band is
    wider than the grid), a 12 x 1 strip and a 1 x 9 column, against the
    oracle with both preconditioners."""
    prs = DEGENERATE[name]()
    plan = mto().Plan(prs, precond=precond)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_zero_load_cases(cuda):
    """A load case with no loads (f = 0) meets the stop test before its first
    iteration and returns u = 0, c = 0 and dc/drho = 0, while the loaded
    systems of the same plan (a second case of the same instance, another
    instance) converge as usual; likewise an instance with no loads at all."""
    prs = [P.uniform_random(6, 3, 2, 3, 11, loads=[(6, 1, 0.0, -1.0, 0)], n_load_cases=2),
           P.uniform_random(5, 2, 3, 2, 12, loads=[]),
           P.small_mixed(8, 4, seed=13)]
    plan = mto().Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)
    its = st["iterations"]  # systems: instance 0 cases 0 and 1, instance 1, instance 2
    assert its[1] == 0 and its[2] == 0 and its[0] > 0 and its[3] > 0, its
    us, cs, gs = plan.split_u(u), plan.split_c(c), plan.split_g(g)
    assert not us[0][1].any() and not us[1].any()
    assert cs[0][1].item() == 0.0 and not cs[1].any()
    assert not gs[0][1].any() and not gs[1].any()


def test_capture_replay_matches_eager(cuda):
    """hipGraph capture of the whole step, replayed several times with eager
    work and synchronisation in between and densities changed in place: every
    replay equals the eager solve of the same densities."""
    prs = [P.small_mixed(12, 6, seed=31, n_loads=2), P.mbb_20x10()]
    plan = mto().Plan(prs)
    rho0 = np.concatenate([p.rho for p in prs])
    rho = torch.tensor(rho0, device=cuda)
    ub, cb, gb = plan.capture(rho)
    eager = mto().Plan(prs)
    for k in range(3):
        scale = 1.0 - 0.1 * k
        rho.copy_(torch.tensor(np.clip(rho0 * scale, 1e-3, 1.0), device=cuda))
        st = plan.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=cuda, dtype=torch.float64).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        u, c, g, st2 = eager.solve(rho)
        assert torch.equal(ub, u) and torch.equal(cb, c) and torch.equal(gb, g), k


def test_warm_start(cuda):
    """u0 = the solution: PCG stops at once with the same outputs."""
    pr = P.small_mixed(12, 6, seed=41)
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    u, c, g, st = plan.solve(rho)
    u2, c2, g2, st2 = plan.solve(rho, u0=u)
    assert st2["max_iterations"] <= 2
    assert rel(u2.cpu().numpy(), u.cpu().numpy()) < 1e-10
    assert abs(c2.item() - c.item()) <= 1e-10 * abs(c.item())


def test_noconv_reported(cuda):
    """max_iter too small: MTO_ENOCONV, outputs still written."""
    m = mto()
    pr = P.small_mixed(12, 6, seed=42)
    plan = m.Plan(pr, max_iter=4, iters_per_launch=2, max_restarts=0, precond=m.PRECOND_JACOBI)
    rho = torch.tensor(pr.rho, device=cuda)
    with pytest.raises(m.MtoError) as ei:
        plan.solve(rho)
    assert ei.value.code == m.MTO_ENOCONV
    u, c, g, st = plan.solve(rho, allow_noconv=True)
    assert st["status"] == m.MTO_ENOCONV and torch.isfinite(u).all()


def test_repeat_solve_is_deterministic(cuda):
    """No atomics: two solves give bit-identical outputs."""
    pr = P.small_mixed(16, 8, seed=51, n_loads=2)
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    a = plan.solve(rho)
    b = plan.solve(rho)
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_time_contraction_modes_leave_solve_exact(cuda):
    """Both timing modes of the contraction report a positive duration, reject
    bad arguments, and a later solve of the same plan is bit-identical to one
    made before them (timing only overwrites the PCG state)."""
    m = mto()
    pr = P.small_mixed(16, 8, seed=52, n_loads=2)
    plan = m.Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    a = plan.solve(rho)
    assert plan.time_contraction(rho, reps=5) > 0.0
    assert plan.time_contraction(rho, reps=40, in_loop=True) > 0.0
    with pytest.raises(m.MtoError):
        plan.time_contraction(rho, reps=0)
    b = plan.solve(rho)
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_stalled_true_residual_is_noconv(cuda):
    """A true residual that misses rtol is MTO_ENOCONV, with finite outputs
    written: rtol 1e-40 (below what the double-double residual resolves) with
    no restarts and with three (the in-cycle residual replacements and then
    the restarts stall).  The same plan at the default tolerance is MTO_OK,
    and at rtol 1e-20 it converges within one cycle: the residual
    replacements carry it past the FP64 floor without a restart."""
    m = mto()
    pr = P.small_mixed(10, 5, seed=43)
    rho = torch.tensor(pr.rho, device=cuda)
    u, c, g, st = m.Plan(pr, rtol=1e-20, max_restarts=0, max_iter=3000).solve(rho)
    assert st["status"] == m.MTO_OK and st["restarts"] == 0 and max(st["true_rel_residual"]) <= 1e-20, st
    for rtol, restarts in ((1e-40, 0), (1e-40, 3)):
        plan = m.Plan(pr, rtol=rtol, max_restarts=restarts, max_iter=3000)
        with pytest.raises(m.MtoError) as ei:
            plan.solve(rho)
        assert ei.value.code == m.MTO_ENOCONV
        u, c, g, st = plan.solve(rho, allow_noconv=True)
        assert st["status"] == m.MTO_ENOCONV and torch.isfinite(u).all() and torch.isfinite(g).all()
        assert max(st["true_rel_residual"]) > rtol
        plan.capture(rho)
        with pytest.raises(m.MtoError) as ei:
            plan.replay()
        assert ei.value.code == m.MTO_ENOCONV
    u, c, g, st = m.Plan(pr).solve(rho)
    assert st["status"] == m.MTO_OK and max(st["true_rel_residual"]) <= 1e-11


@pytest.mark.parametrize("bad", [float("nan"), -0.25, 1.5, float("inf")])
def test_invalid_density_rejected(cuda, bad):
    """A density that is not finite or outside [0, 1] (Eq. (1) bounds it to
    [0, 1]): mto_solve and the graph replay return MTO_EINVAL without
    iterating, and the next solve of the same plan with valid densities is
    bit-identical to a fresh plan's."""
    m = mto()
    pr = P.small_mixed(9, 5, seed=44, n_loads=2)
    plan = m.Plan(pr)
    good = torch.tensor(pr.rho, device=cuda)
    rho = good.clone()
    rho[pr.n_cells // 3] = bad
    with pytest.raises(m.MtoError) as ei:
        plan.solve(rho)
    assert ei.value.code == m.MTO_EINVAL and "density" in str(ei.value)
    ub, cb, gb = plan.capture(rho)
    with pytest.raises(m.MtoError) as ei:
        plan.replay()
    assert ei.value.code == m.MTO_EINVAL
    rho.copy_(good)
    st = plan.replay()
    assert st["status"] == m.MTO_OK
    u, c, g, st2 = m.Plan(pr).solve(good)
    assert torch.equal(ub, u) and torch.equal(cb, c) and torch.equal(gb, g)
    u2, c2, g2, _ = plan.solve(good)
    assert torch.equal(u2, u) and torch.equal(c2, c)
    # the bounds themselves are valid densities
    edge = good.clone()
    edge[0], edge[1] = 0.0, 1.0
    plan.solve(edge)


def test_autotune_cache(cuda, tmp_path):
    """The tile-shape cache: a first autotune times every group and writes one
    line per (arch, p, d, size class), plus one line (p = 0) for the choice
    between one launch per group and the fused launch; a second plan of the
    same mesh takes every shape and that choice from the file without timing
    and solves to the same bits as the first; a malformed file is
    MTO_EINVAL."""
    m = mto()
    pr = P.small_mixed(16, 8, seed=45)
    rho = torch.tensor(pr.rho, device=cuda)
    path = tmp_path / "tiles.txt"
    a = m.Plan(pr)
    rep_a = a.autotune(rho, cache=str(path))
    lines = [ln for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert len(lines) == a.info["n_groups"] + 1, (lines, rep_a)
    assert sum(ln.split()[1] == "0" for ln in lines) == 1
    assert "cached" not in rep_a
    product = [ln for ln in rep_a.splitlines() if ln.startswith("product:")]
    b = m.Plan(pr)
    rep_b = b.autotune(rho, cache=str(path))
    assert rep_b.count("cached") == a.info["n_groups"], rep_b
    assert sorted(l for l in rep_a.splitlines() if l.endswith("chosen")) == \
        sorted(l for l in rep_b.splitlines() if l.endswith("chosen"))
    assert product == [ln for ln in rep_b.splitlines() if ln.startswith("product:")]
    ua, ca, ga, _ = a.solve(rho)
    ub, cb, gb, _ = b.solve(rho)
    assert torch.equal(ua, ub) and torch.equal(ca, cb) and torch.equal(ga, gb)
    # a stored-matrix choice (ks = -2) in the file is taken as well
    st_path = tmp_path / "stored.txt"
    fields = [ln.split() for ln in path.read_text().splitlines() if not ln.startswith("#")]
    for f in fields:
        if f[1] == "4":
            f[4], f[5] = "1", "-2"
        if f[1] == "0":  # one launch per group, so the stored choice is used
            f[4] = "2"
    st_path.write_text("".join(" ".join(f) + "\n" for f in fields))
    c = m.Plan(pr, stored_matrices=1)
    rep_c = c.autotune(rho, cache=str(st_path))
    assert "p=4 d=5 ncol=1 ks=-2: chosen" in rep_c, rep_c
    uc, cc, gc, stc = c.solve(rho)
    check_solution(c, [pr], uc, cc, gc, stc)
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 3 4 nonsense\n")
    with pytest.raises(m.MtoError) as ei:
        m.Plan(pr).autotune(rho, cache=str(bad))
    assert ei.value.code == m.MTO_EINVAL


@pytest.mark.parametrize("ncol", [1, 2])
@pytest.mark.parametrize("name", ["uniform_p3d4", "uniform_p4d5", "uniform_p4d8_max", "mixed_3loads"])
def test_solve_parity_lds_staged(cuda, name, ncol):
    """Solves with the LDS-staged contraction (cell tables shared by four
    waves through LDS) on every p >= 3 group, against the oracle."""
    prs = CASES[name]()
    plan = mto().Plan(prs)
    plan.set_tile(ncol, 0)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_lds_staged_product_many_tiles(cuda):
    """The LDS-staged product on a 40 x 23 p = 4, d = 5 mesh with two load
    cases (30 tiles of 64 columns, the last ragged; tiles of both systems)
    equals the register-fragment product to 1e-14 and the oracle's K x."""
    pr = P.uniform_random(40, 23, 4, 5, seed=91, loads=[(40, 11, 0.0, -1.0, 0), (40, 3, 1.0, 0.0, 1)], n_load_cases=2)
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    free = free_mask(space, pr.supports)
    x = np.random.default_rng(5).standard_normal((2, space.n_dof))
    x[:, ~free] = 0.0
    yref = (K @ x.T).T
    yref[:, ~free] = 0.0
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    xt = torch.tensor(x.ravel(), device=cuda)
    plan.set_tile(1, 1)
    y1 = plan.apply_stiffness(rho, xt).cpu().numpy()
    for nc in (1, 2):
        plan.set_tile(nc, 0)
        y = plan.apply_stiffness(rho, xt).cpu().numpy()
        assert rel(y, yref.ravel()) < 1e-13, (nc, rel(y, yref.ravel()))
        assert rel(y, y1) < 1e-14


@pytest.mark.parametrize("precond", ["schwarz", "jacobi"])
@pytest.mark.parametrize("name", ["uniform_p1d3", "uniform_p2d2", "uniform_p3d4", "uniform_p4d5", "uniform_p4d8_max",
                                  "mixed16x8", "mixed_3loads"])
def test_solve_parity_stored(cuda, name, precond):
    """Solves with stored element matrices (K_e = sum_s E_s K_s assembled in
    the set-up, each product reading it) on every group, against the oracle."""
    m = mto()
    prs = CASES[name]()
    plan = m.Plan(prs, precond=m.PRECOND_MG_ASM if precond == "schwarz" else m.PRECOND_JACOBI)
    plan.set_tile(1, -2)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_stored_batch_many_loads(cuda):
    """Stored element matrices over a batch of uneven instances, one with six
    load cases (two passes of four systems over each tile), one with one;
    solved twice with different densities (the matrices are reassembled),
    against the oracle."""
    m = mto()
    loads = [(12, k, 0.0, -1.0, k) for k in range(6)]
    prs = [P.uniform_random(12, 6, 4, 5, seed=71, loads=loads, n_load_cases=6), P.small_mixed(10, 5, seed=72)]
    plan = m.Plan(prs)
    plan.set_tile(1, -2, p=4, d=5)
    for seed in (0, 1):
        if seed:
            for pr in prs:
                pr.rho = np.clip(pr.rho * np.random.default_rng(seed).uniform(0.5, 1.0, pr.rho.size), 1e-3, 1.0)
        rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
        u, c, g, st = plan.solve(rho)
        check_solution(plan, prs, u, c, g, st)


def test_stored_product_apply(cuda):
    """mto_apply_stiffness with stored element matrices (assembled from the
    given densities) on a 40 x 23 p = 4, d = 5 mesh with two load cases
    equals the oracle's K x and the contraction to 1e-13."""
    pr = P.uniform_random(40, 23, 4, 5, seed=91, loads=[(40, 11, 0.0, -1.0, 0), (40, 3, 1.0, 0.0, 1)], n_load_cases=2)
    K, space, *_ = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    free = free_mask(space, pr.supports)
    x = np.random.default_rng(6).standard_normal((2, space.n_dof))
    x[:, ~free] = 0.0
    yref = (K @ x.T).T
    yref[:, ~free] = 0.0
    plan = mto().Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    xt = torch.tensor(x.ravel(), device=cuda)
    y1 = plan.apply_stiffness(rho, xt).cpu().numpy()
    plan.set_tile(1, -2)
    y = plan.apply_stiffness(rho, xt).cpu().numpy()
    assert rel(y, yref.ravel()) < 1e-13, rel(y, yref.ravel())
    assert rel(y, y1) < 1e-13


@pytest.mark.parametrize("name", ["mixed16x8", "mixed_3loads", "uniform_p4d5"])
def test_solve_parity_fused_product(cuda, name):
    """Solves with the fused product (one launch over the tiles of every
    (p, d) group and system) against the oracle."""
    prs = CASES[name]()
    plan = mto().Plan(prs)
    plan.set_tile(1, -1)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)


def test_schwarz_persistent_grid(cuda, monkeypatch):
    """The Schwarz smoother's grid capped at 1, 2 and 5 blocks
    (MTO_ASM_GRID): each block then walks many tiles through its load/compute
    pipeline, with 1 block over two 256-tile windows (the 48 x 24 p = 4 mesh
    has 288 tiles of 4 element columns), and a six-load instance takes two
    passes of four systems per tile.  Every capped solve equals the uncapped
    one (one block per tile at this size) bit for bit, and that one equals
    the oracle."""
    m = mto()
    loads = [(48, 4 * k, 0.0, -1.0, k) for k in range(6)]
    prs = [P.uniform_random(48, 24, 4, 5, seed=81, loads=loads, n_load_cases=6),
           P.small_mixed(14, 7, seed=82, n_loads=3)]
    plan = m.Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    monkeypatch.delenv("MTO_ASM_GRID", raising=False)
    u0, c0, g0, st0 = plan.solve(rho)
    check_solution(plan, prs, u0, c0, g0, st0)
    for cap in ("1", "2", "5"):
        monkeypatch.setenv("MTO_ASM_GRID", cap)
        u, c, g, st = plan.solve(rho)
        assert torch.equal(u, u0) and torch.equal(c, c0) and torch.equal(g, g0), cap
        assert st["iterations"] == st0["iterations"], cap


@pytest.mark.parametrize("case", ["mixed", "void_cells"])
def test_true_residual_extended_precision(cuda, case):
    """The true residual a solve reports, |f - K u| / |f| per load case on the
    free DOFs, against the same quantity from the oracle's element operator
    in 80-bit long double (rigid motions removed as on both sides; its error
    is far below the residual).  u comes from a solve to rtol 1e-13 and is
    then given as the initial guess of a solve to rtol 1e-6, which stops at
    iteration 0 and reports the residual of exactly that u.  Near 1e-13 the
    residual through the assembled FP64 matrix differs from it by 2-20 % on
    these meshes (measured with the oracle's solutions); agreement to 2 %
    pins the library's extended-precision product (compensated per-cell
    sums, double-double over the cells)."""
    from oracle.fem import simp_modulus
    from oracle.solve import ElementOperator, load_vectors

    m = mto()
    if case == "mixed":
        pr = P.small_mixed(12, 6, seed=64, n_loads=2)
    else:  # i.i.d. densities down to 1e-3: moduli over nine decades within elements
        pr = P.uniform_random(12, 6, 2, 3, seed=65, lo=1e-3, hi=1.0,
                              loads=[(12, 3, 0.0, -1.0, 0), (12, 6, 1.0, 0.0, 1)], n_load_cases=2)
    rho = torch.tensor(pr.rho, device=cuda)
    u, c, g, st = m.Plan(pr, rtol=1e-13).solve(rho, allow_noconv=True)
    u2, c2, g2, st2 = m.Plan(pr, rtol=1e-6).solve(rho, u0=u)
    assert max(st2["iterations"]) == 0 and torch.equal(u2, u), st2
    uu = u.cpu().numpy().reshape(pr.n_load_cases, -1)
    K, space, edofs, off, ks = assemble(pr.nelx, pr.nely, pr.p, pr.d, pr.rho, pr.E0, pr.Emin, pr.q, pr.nu)
    E = simp_modulus(pr.rho, pr.E0, pr.Emin, pr.q)
    op = ElementOperator(pr.p, pr.d, E, edofs, off, ks, pr.nu, space.n_dof)
    free = free_mask(space, pr.supports)
    f = load_vectors(space, pr.loads, pr.n_load_cases)
    for lc in range(pr.n_load_cases):
        r = f[lc].astype(np.longdouble) - op.apply(uu[lc])
        ref = float(np.sqrt(np.sum(r[free] ** 2)) / np.sqrt(np.sum(f[lc][free].astype(np.longdouble) ** 2)))
        got = st2["true_rel_residual"][lc]
        assert 0.0 < ref < 1e-9 and abs(got - ref) <= 0.02 * ref, (case, lc, got, ref, st["true_rel_residual"])


@pytest.mark.parametrize("ncol", [2, 4])
@pytest.mark.parametrize("name", ["mixed_3loads", "uniform_p4d5", "uniform_p3d4", "uniform_p2d2"])
def test_solve_parity_wide_tiles(cuda, name, ncol):
    """Schwarz-multigrid solves with tiles of 16 ncol columns for every group
    (the PCG product, the product after the pre-smoothing and the vertex
    update on them, ragged last tiles included), against the oracle."""
    prs = CASES[name]()
    plan = mto().Plan(prs)
    plan.set_tile(ncol, 1)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    u, c, g, st = plan.solve(rho)
    check_solution(plan, prs, u, c, g, st)
