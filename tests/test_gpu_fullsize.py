"""Full-size parity: the benchmark workloads in the launch configuration the
benchmark times (autotuned tiles, captured graphs), against the CPU oracle's
direct solve of the same design (it finishes in seconds at these sizes), plus
properties that hold at any size.  The workloads use the plain random density
field of the configurations; config 2 is also run on the eased field with
solid load paths, and the iteration counts of both are printed."""

import functools
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

from oracle import oracle_solve, simp_modulus, simp_modulus_derivative
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

U_TOL, C_TOL, G_TOL = 1e-8, 1e-8, 1e-7


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@functools.lru_cache(maxsize=None)
def _oracle(cfg, solid_paths):
    """Oracle solution of a configuration and the FP64 floor of its true
    residual, eps || |K| |u| || / ||f||."""
    pr = P.config(cfg, solid_paths=solid_paths)
    o = oracle_solve(**pr.oracle_args(), want_K=True)
    K = o.pop("K")
    floor = np.finfo(float).eps * np.linalg.norm(abs(K) @ np.abs(o["u"].ravel())) / np.linalg.norm(o["f"])
    return o, floor


@pytest.mark.parametrize("cfg,solid_paths,precond", [(2, False, 0), (2, False, 2), (2, True, 2), (3, False, 0),
                                                      (3, False, 2)])
def test_fullsize_against_oracle(cuda, cfg, solid_paths, precond):
    """Jacobi (0) and Schwarz-multigrid (2) preconditioned solves; the plain
    field of the configuration, and for config 2 also the eased field."""
    from paper_1811_09821_amd import mto

    pr = P.config(cfg, solid_paths=solid_paths)
    field = "eased (solid load paths)" if solid_paths else "plain"
    print(f"\nfull-size config {cfg}: {pr.name}, {field} field, preconditioner {precond}", flush=True)
    plan = mto.Plan(pr, precond=precond)
    rho = torch.tensor(pr.rho, device=cuda)
    plan.autotune(rho)
    u, c, g = plan.capture(rho)
    st = plan.replay()
    torch.cuda.synchronize()
    print(f"iterations {st['iterations']} restarts {st['restarts']} true residual {st['true_rel_residual']}",
          flush=True)
    o, floor = _oracle(cfg, solid_paths)
    un, cn, gn = u.cpu().numpy(), c.cpu().numpy(), g.cpu().numpy()
    ou, og = o["u"].ravel(), o["g"].ravel()
    print(f"c = {cn[0]:.10g} (oracle {o['c'][0]:.10g}); u rel 2-norm {rel(un, ou):.2e} max-norm "
          f"{rel_max(un, ou):.2e}; g rel 2-norm {rel(gn, og):.2e} max-norm {rel_max(gn, og):.2e}", flush=True)
    assert rel(un, ou) < U_TOL
    assert rel_max(un, ou) < U_TOL
    assert abs(cn[0] - o["c"][0]) < C_TOL * abs(o["c"][0])
    assert rel(gn, og) < G_TOL
    assert rel_max(gn, og) < G_TOL
    # The library checks its true residual in double-double, so it meets
    # 1e-11 even where an FP64 evaluation of f - K u could not resolve it
    # (floor about eps || |K| |u| ||, printed for reference).
    print(f"FP64 residual floor {floor:.3e}", flush=True)
    assert st["true_rel_residual"][0] <= 1e-11

    # properties at full size: c = u^T K u, Euler identity, sign of g
    Ku = plan.apply_stiffness(rho, u).cpu().numpy()
    assert abs(float(un @ Ku) - cn[0]) < 1e-9 * cn[0]
    w = -gn / simp_modulus_derivative(pr.rho, pr.E0, pr.Emin, pr.q)
    lhs = float(np.dot(pr.rho, gn))
    rhs = -pr.q * (cn[0] - pr.Emin * w.sum())
    assert abs(lhs - rhs) < 1e-8 * abs(rhs)
    # g <= 0 up to the rounding of u_e^T K_s u_e (near-rigid void cells)
    assert (gn <= 1e-10 * np.abs(gn).max()).all()
    assert abs(float(np.dot(simp_modulus(pr.rho, pr.E0, pr.Emin, pr.q), w)) - cn[0]) < 1e-8 * cn[0]


def _oracle_of_design(i):
    """Oracle u, c, g of design i of the 64-design batch (run in a worker)."""
    pr = P.batch_instances(n=1, first_seed=100 + i)[0]  # design i alone (seeded per design)
    o = oracle_solve(**pr.oracle_args())
    return i, o["u"], o["c"], o["g"]


@functools.lru_cache(maxsize=None)
def _oracle_batch():
    """The oracle's direct solves of all 64 designs, spread over the host
    cores (forked workers that use only NumPy/SciPy)."""
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_oracle_of_design, range(64), chunksize=1)
    return {i: (u, c, g) for i, u, c, g in out}


def test_fullsize_batch_of_64(cuda):
    """The batch of 64 uneven mixed-order designs (40 x 20 to 314 x 157
    elements, one to three load cases each) in the launch configuration the
    benchmark times: every system meets the 1e-11 true residual; for every
    design and load case c = u^T K u, the Euler identity of the SIMP
    sensitivities and the sign of g hold, and u (2-norm and max-norm), c and
    g (2-norm and max-norm) match the oracle's direct solve."""
    from paper_1811_09821_amd import mto

    prs = P.config(4)
    plan = mto.Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    plan.autotune(rho)
    u, c, g = plan.capture(rho)
    st = plan.replay()
    torch.cuda.synchronize()
    print(f"\nbatch of {len(prs)}: iterations {min(st['iterations'])}-{max(st['iterations'])} "
          f"(mean {np.mean(st['iterations']):.1f}), restarts {st['restarts']}, "
          f"largest true residual {max(st['true_rel_residual']):.2e}", flush=True)
    assert st["status"] == 0 and max(st["true_rel_residual"]) <= 1e-11
    Ku = plan.apply_stiffness(rho, u)
    us, cs, gs, kus = plan.split_u(u), plan.split_c(c), plan.split_g(g), plan.split_u(Ku)
    for i, pr in enumerate(prs):
        ui, ci, gi, kui = (t.cpu().numpy() for t in (us[i], cs[i], gs[i], kus[i]))
        E = simp_modulus(pr.rho, pr.E0, pr.Emin, pr.q)
        dE = simp_modulus_derivative(pr.rho, pr.E0, pr.Emin, pr.q)
        for lc in range(pr.n_load_cases):
            assert abs(float(ui[lc] @ kui[lc]) - ci[lc]) < 1e-9 * ci[lc], (pr.name, lc)
            w = -gi[lc] / dE
            rhs = -pr.q * (ci[lc] - pr.Emin * w.sum())
            assert abs(float(np.dot(pr.rho, gi[lc])) - rhs) < 1e-8 * abs(rhs), (pr.name, lc)
            assert (gi[lc] <= 1e-10 * np.abs(gi[lc]).max()).all(), (pr.name, lc)
            assert abs(float(np.dot(E, w)) - ci[lc]) < 1e-8 * ci[lc], (pr.name, lc)
    print("oracle solves of the 64 designs ...", flush=True)
    ref = _oracle_batch()
    worst = [0.0, 0.0, 0.0, 0.0]
    for i, pr in enumerate(prs):
        ou, oc, og = ref[i]
        ui, ci, gi = us[i].cpu().numpy(), cs[i].cpu().numpy(), gs[i].cpu().numpy()
        for lc in range(pr.n_load_cases):
            e = (rel(ui[lc], ou[lc]), rel_max(ui[lc], ou[lc]), rel(gi[lc], og[lc]), rel_max(gi[lc], og[lc]))
            worst = [max(a, b) for a, b in zip(worst, e)]
            assert e[0] < U_TOL and e[1] < U_TOL, (pr.name, lc, e)
            assert e[2] < G_TOL and e[3] < G_TOL, (pr.name, lc, e)
        assert np.all(np.abs(ci - oc) <= C_TOL * np.abs(oc)), (pr.name, ci, oc)
    print(f"worst over all designs and load cases: u {worst[0]:.2e} / {worst[1]:.2e} (2-norm / max-norm), "
          f"g {worst[2]:.2e} / {worst[3]:.2e}", flush=True)
