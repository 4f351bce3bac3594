"""Pins of the oracle's refinement indicators and dp update (Sec. 3.2-3.3):
the Kelly estimator vanishes for fields without gradient jumps and has a
closed form for a piecewise-linear kink; the density indicator matches
values worked by hand (tests/golden/density_indicator.json); the dp update
matches a case worked by hand and keeps its invariants."""

import json
import os

import numpy as np
import pytest

from oracle.adapt import density_bounds, density_indicator, dp_update, kelly_indicator, qr_update, smooth_p
from oracle.solve import element_dofs_global
from oracle.space import build_space
from paper_1811_09821_amd import problems as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "density_indicator.json")


def vertex_field(nelx, nely, p, fx, fy):
    """Global DOF vector whose vertex values are (fx, fy)(x, y) and whose
    hierarchic modes are zero: on every element it is the bilinear
    interpolant of the vertex values."""
    space = build_space(nelx, nely, p)
    u = np.zeros(space.n_dof)
    for vy in range(nely + 1):
        for vx in range(nelx + 1):
            s = vy * (nelx + 1) + vx
            u[2 * s], u[2 * s + 1] = fx(vx, vy), fy(vx, vy)
    return u


def test_kelly_zero_for_a_linear_field_on_a_mixed_mesh():
    pr = P.small_mixed(7, 4, seed=61)
    u = vertex_field(pr.nelx, pr.nely, pr.p, lambda x, y: 0.3 * x - 0.2 * y + 1.0, lambda x, y: 0.1 * x + 0.5 * y)
    g = kelly_indicator(pr.nelx, pr.nely, pr.p, u[None])
    assert np.abs(g).max() < 1e-26


@pytest.mark.parametrize("p", [1, 2, 3])
def test_kelly_kink_closed_form(p):
    """u_x = |x - 2| on a uniform order-p mesh: du_x/dx jumps by 2 across
    the vertical edges at x = 2 (and nowhere else), so an element next to
    that line gets c_F * 2^2 * 1 = sqrt(2)/(2p) * 4 and every other element 0;
    u_y = |y - 1| adds the same on the horizontal edges at y = 1."""
    nelx, nely = 5, 3
    pa = np.full(nelx * nely, p)
    u = vertex_field(nelx, nely, pa, lambda x, y: abs(x - 2), lambda x, y: abs(y - 1))
    g = kelly_indicator(nelx, nely, pa, u[None])[0]
    one = np.sqrt(2.0) / (2 * p) * 4.0
    for e in range(nelx * nely):
        ex, ey = e % nelx, e // nelx
        expect = one * ((ex in (1, 2)) + (ey in (0, 1)))
        assert abs(g[e] - expect) < 1e-12, (e, g[e], expect)


def test_density_indicator_golden():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        rho = np.array(c["rho"])
        d = int(round(np.sqrt(rho.size)))
        assert d * d == rho.size
        g = density_indicator([d], rho, c["cycle"])
        assert abs(g[0] - c["expected"]) < 1e-15, (c, g[0])


def test_density_bounds_widen_with_the_cycle():
    """The refinement zone [r_l, r_u] widens and the coarsening zones shrink
    towards 0 and 1 as the cycle index grows (Sec. 3.2.2)."""
    prev = None
    for k in range(1, 6):
        rl, ru, cl, cu, avg = density_bounds(k)
        assert 0.0 <= cl <= rl <= avg <= ru <= cu <= 1.0
        if prev:
            assert rl < prev[0] and ru > prev[1] and cl < prev[2] and cu > prev[3]
        prev = (rl, ru, cl, cu)


def test_dp_update_worked_case():
    """Four elements, p = 2: analysis ranking 0.1 (e0) < 0.2 (e3) < 0.3 (e2) <
    0.4 (e1) with a quarter coarsened and a quarter refined -> e0 down
    (theta -1, p 1), e1 up (theta 1, p 3); density indicator -0.1, 0, 0.2,
    -0.3 -> e3 coarsened to p 1, e0 already at p 1 (theta -2), e2 refined to
    p 3; no smoothing needed (differences 2); design points 1 (theta -2),
    2*16-3 = 29, 29, 2*4-3 = 5; background 36 cells (6^2 >= 29)."""
    p, theta, dp, cells = dp_update(4, 1, [2, 2, 2, 2], [0.1, 0.4, 0.3, 0.2], [-0.1, 0.0, 0.2, -0.3],
                                   frac_a_refine=0.25, frac_a_coarsen=0.25)
    assert list(p) == [1, 3, 3, 1]
    assert list(theta) == [-2, 1, 0, 0]
    assert list(dp) == [1, 29, 29, 5]
    assert cells == 36


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dp_update_invariants(seed):
    rng = np.random.default_rng(seed)
    nelx, nely = 9, 5
    p0 = rng.integers(1, 6, nelx * nely)
    p0 = smooth_p(p0, nelx, nely)
    p, theta, dp, cells = dp_update(nelx, nely, p0, rng.standard_normal(nelx * nely),
                                    rng.standard_normal(nelx * nely))
    P2 = p.reshape(nely, nelx)
    assert np.abs(np.diff(P2, axis=0)).max() <= 2 and np.abs(np.diff(P2, axis=1)).max() <= 2
    assert p.min() >= 1 and p.max() <= 5
    assert dp.max() <= 64 and cells >= dp.max() and int(np.sqrt(cells)) ** 2 == cells


def test_qr_update():
    assert list(qr_update([1, 2, 5, 3], [0.95, 0.2, 0.99, 0.9])) == [2, 2, 5, 3]
