"""Refinement indicators and the dp update of Sec. 3.2-3.3.

Test infrastructure only (see the package docstring).

* Analysis indicator (Sec. 3.2.1, the Kelly estimator): for element i,
  Gamma^a_i = sum over its edges F of c_F * integral over F of |[du/dn]|^2 ds,
  [.] the jump across F, c_F = h_F / (2 p_F), h_F the element diagonal and
  p_F the larger order of the two elements.  Reading: only interior edges
  carry a jump (a boundary edge has no neighbour; the estimator is used for
  ranking only), u is the vector field (both components' jumps squared and
  added), lengths in element edge lengths (h_F = sqrt(2)).
* Density indicator (Sec. 3.2.2): Gamma^d_k summed over the element's cells
  with the cycle-dependent bounds r_l, r_u, c_l, c_u (alpha = 0.2,
  beta = 0.8).  Readings: rho_min, rho_max are the bounds of the density
  (0 and 1); the second refinement case reads "rho_avg < rho <= r_u" (the
  printed condition names r_avg and rho_u).
* dp update (Sec. 3.3), steps 2-4 in the paper's order; see dp_update.
"""

import numpy as np
from numpy.polynomial import legendre as npleg

from .fem import basis_1d
from .solve import element_dofs_global
from .space import build_space


def _grad_normal(ue, p, side, t):
    """d u / d n (outward normal of the element's edge `side`) of the element
    field with local DOFs ue at the edge points with tangential reference
    coordinate t in [-1, 1]; side in 'left', 'right', 'bottom', 'top'.
    Returns [2, len(t)] (both components).  d/dx = 2 d/dxi."""
    n1 = p + 1
    xi_fixed = {"left": -1.0, "right": 1.0, "bottom": -1.0, "top": 1.0}[side]
    phi_t, dphi_t = basis_1d(p, t)
    phi_f, dphi_f = basis_1d(p, np.array([xi_fixed]))
    sign = 1.0 if side in ("right", "top") else -1.0
    out = np.zeros((2, t.size))
    for j in range(n1):
        for i in range(n1):
            a = j * n1 + i
            if side in ("left", "right"):  # normal x: d/dxi at xi fixed, eta = t
                val = 2.0 * dphi_f[i, 0] * phi_t[j]
            else:  # normal y: d/deta at eta fixed, xi = t
                val = 2.0 * phi_t[i] * dphi_f[j, 0]
            for c in range(2):
                out[c] += ue[2 * a + c] * val
    return sign * out


def kelly_indicator(nelx, nely, p, u):
    """Gamma^a [L, nel] for global displacements u [L, n_dof]."""
    p = np.asarray(p, dtype=np.int64).ravel()
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    space = build_space(nelx, nely, p)
    hF = np.sqrt(2.0)
    out = np.zeros((u.shape[0], nelx * nely))
    for lc in range(u.shape[0]):
        ue = []
        for e in range(nelx * nely):
            G = element_dofs_global(space, e)
            ue.append(np.where(G >= 0, u[lc][np.maximum(G, 0)], 0.0))
        for e in range(nelx * nely):
            ex, ey = e % nelx, e // nelx
            for side, (dx, dy), other in (("left", (-1, 0), "right"), ("right", (1, 0), "left"),
                                          ("bottom", (0, -1), "top"), ("top", (0, 1), "bottom")):
                nx_, ny_ = ex + dx, ey + dy
                if not (0 <= nx_ < nelx and 0 <= ny_ < nely):
                    continue
                f = ny_ * nelx + nx_
                pF = max(p[e], p[f])
                t, w = npleg.leggauss(int(pF) + 1)
                # the jump of du/dn with n the outward normal of e: du_e/dn_e + du_f/dn_f
                jump = _grad_normal(ue[e], int(p[e]), side, t) + _grad_normal(ue[f], int(p[f]), other, t)
                # ds = dt / 2 on a unit edge
                integral = float(np.sum(0.5 * w * (jump ** 2).sum(axis=0)))
                out[lc, e] += hF / (2.0 * pF) * integral
    return out


def density_bounds(cycle, alpha=0.2, beta=0.8, rho_min=0.0, rho_max=1.0):
    """(r_l, r_u, c_l, c_u, rho_avg) of Sec. 3.2.2 for adaptive cycle index
    `cycle` (1 for the first)."""
    avg = 0.5 * (rho_max + rho_min)
    s = avg * np.exp(-beta * (cycle - 1))
    return (rho_min + (1 - alpha) * s, rho_max - (1 - alpha) * s, rho_min + alpha * s, rho_max - alpha * s, avg)


def density_indicator(d, rho, cycle, alpha=0.2, beta=0.8, rho_min=0.0, rho_max=1.0):
    """Gamma^d [nel] of Sec. 3.2.2 from the densities of each element's cells
    (element-major, d_e^2 cells each)."""
    d = np.asarray(d, dtype=np.int64).ravel()
    rho = np.asarray(rho, dtype=np.float64).ravel()
    rl, ru, cl, cu, avg = density_bounds(cycle, alpha, beta, rho_min, rho_max)
    out = np.zeros(d.size)
    k0 = 0
    for e in range(d.size):
        n = int(d[e]) ** 2
        g = 0.0
        for r in rho[k0:k0 + n]:
            if rl <= r <= avg:
                g += (r - rl) / n
            if avg < r <= ru:
                g += (ru - r) / n
            if r <= cl:
                g -= (cl - r) / n
            if r >= cu:
                g -= (r - cu) / n
        out[e] = g
        k0 += n
    return out


def smooth_p(p, nelx, nely, max_jump=2):
    """Raise the lower order of neighbouring elements until they differ by at
    most max_jump (Sec. 3.3, step 3c)."""
    p = np.asarray(p, dtype=np.int64).reshape(nely, nelx).copy()
    for _ in range(max(0, int(p.max() - p.min() - max_jump))):
        for ey in range(nely):
            for ex in range(nelx):
                for fx, fy in ((ex + 1, ey), (ex, ey + 1)):
                    if fx < nelx and fy < nely:
                        a, b = p[ey, ex], p[fy, fx]
                        if a < b - max_jump:
                            p[ey, ex] = b - max_jump
                        elif b < a - max_jump:
                            p[fy, fx] = a - max_jump
    return p.ravel()


def dp_update(nelx, nely, p, gamma_a, gamma_d, frac_a_refine=0.10, frac_a_coarsen=0.05,
              frac_d_refine=1.0, frac_d_coarsen=1.0, p_max=5, d_max=64):
    """Steps 2 and 3 of the dp update (Sec. 3.3).  Returns (p_new, theta,
    design_points, cells_per_element).

    Readings: ranking by ascending value, ties by element index; the density
    fractions select among elements with Gamma^d < 0 (coarsening) and > 0
    (refinement) only, which is what the paper's fractions of 1.0 amount to;
    p stays within [1, p_max]; the design points of an element are capped at
    d_max; the background grid has the smallest perfect square of cells not
    below the largest number of design points."""
    p = np.asarray(p, dtype=np.int64).ravel().copy()
    ga = np.asarray(gamma_a, dtype=np.float64).ravel()
    gd = np.asarray(gamma_d, dtype=np.float64).ravel()
    nel = p.size
    theta = np.zeros(nel, dtype=np.int64)
    # step 2: analysis indicator
    order = np.lexsort((np.arange(nel), ga))
    nc, nr = int(np.floor(frac_a_coarsen * nel)), int(np.floor(frac_a_refine * nel))
    theta[order[:nc]] = -1
    theta[order[nel - nr:]] = 1
    p = np.clip(p + theta, 1, p_max)
    # step 3: density indicator
    order = np.lexsort((np.arange(nel), gd))
    neg = [k for k in order if gd[k] < 0]
    pos = [k for k in order if gd[k] > 0]
    for k in neg[:int(np.floor(frac_d_coarsen * len(neg)))]:
        if p[k] == 1:
            theta[k] = -2
        elif theta[k] == 0:
            p[k] -= 1
    for k in pos[len(pos) - int(np.floor(frac_d_refine * len(pos))):]:
        if theta[k] in (0, -1):
            p[k] = min(p[k] + 1, p_max)
    p = smooth_p(p, nelx, nely)
    dp = np.where(theta == -2, 1, np.minimum(2 * (p + 1) ** 2 - 3, d_max))
    side = int(np.ceil(np.sqrt(dp.max()) - 1e-12))
    return p, theta, dp, side * side


def qr_update(p, eps, alpha_qr=0.9, p_max=5):
    """Step 4 of Sec. 3.3: p + 1 where the QR error exceeds alpha_qr (one
    step per cycle), capped at p_max."""
    p = np.asarray(p, dtype=np.int64).ravel()
    return np.minimum(p + (np.asarray(eps).ravel() > alpha_qr), p_max)
