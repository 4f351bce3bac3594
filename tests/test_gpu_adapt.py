"""GPU parity of the refinement indicators (Sec. 3.2.1 Kelly, Sec. 3.2.2
density) against the oracle.

Tolerances (written here): the Kelly indicator within 1e-10 of the largest
value (each edge integral is a short Gauss sum of squared gradient jumps; the
jumps are differences of two gradients, so the absolute error scales with
the gradients, not with the jump); the density indicator within 1e-15
(the same few additions in the same order)."""

import numpy as np
import pytest
import torch

from oracle import oracle_solve
from oracle.adapt import density_indicator, kelly_indicator
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

CASES = {
    "mixed_13x7_2loads": lambda: P.small_mixed(13, 7, seed=71, n_loads=2),
    "p1d2": lambda: P.uniform_random(9, 4, 1, 2, 72),
    "p3d4": lambda: P.uniform_random(6, 3, 3, 4, 73),
    "p4d5": lambda: P.uniform_random(5, 3, 4, 5, 74),
    "inverter_40x20": lambda: P.force_inverter(40, 20, p=2, d=4),
}


def mto():
    from paper_1811_09821_amd import mto as m

    return m


@pytest.mark.parametrize("key", sorted(CASES))
def test_kelly_indicator(cuda, key):
    pr = CASES[key]()
    o = oracle_solve(**pr.oracle_args())
    plan = mto().Plan(pr)
    g = plan.kelly_indicator(torch.tensor(o["u"].ravel(), device=cuda)).cpu().numpy()
    ref = kelly_indicator(pr.nelx, pr.nely, pr.p, o["u"]).ravel()
    assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max(), (key, np.abs(g - ref).max(), np.abs(ref).max())


def test_kelly_batch_layout(cuda):
    prs = [CASES[k]() for k in ("mixed_13x7_2loads", "p1d2", "p4d5")]
    us = [oracle_solve(**pr.oracle_args())["u"] for pr in prs]
    plan = mto().Plan(prs)
    ufull = torch.zeros(plan.info["n_u"], dtype=torch.float64, device=cuda)
    for r, u in zip(plan.instances, us):
        ufull[r["u_off"]:r["u_off"] + u.size] = torch.tensor(u.ravel(), device=cuda)
    gs = plan.split_eps(plan.kelly_indicator(ufull))
    for pr, u, g in zip(prs, us, gs):
        ref = kelly_indicator(pr.nelx, pr.nely, pr.p, u)
        assert np.abs(g.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("cycle", [1, 2, 4])
def test_density_indicator(cuda, cycle):
    prs = [P.small_mixed(13, 7, seed=75), P.config(2), P.uniform_random(4, 3, 2, 8, 76, lo=0.0, hi=1.0)]
    plan = mto().Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=cuda)
    g = plan.density_indicator(rho, cycle).cpu().numpy()
    ref = np.concatenate([density_indicator(pr.d, pr.rho, cycle) for pr in prs])
    assert np.abs(g - ref).max() <= 1e-15


def test_indicators_full_size(cuda):
    """The 160 x 80 (p = 3, d = 4) cantilever: the Kelly indicator of every
    element against the oracle's."""
    pr = P.config(2)
    o = oracle_solve(**pr.oracle_args())
    plan = mto().Plan(pr)
    g = plan.kelly_indicator(torch.tensor(o["u"].ravel(), device=cuda)).cpu().numpy()
    ref = kelly_indicator(pr.nelx, pr.nely, pr.p, o["u"]).ravel()
    assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()
