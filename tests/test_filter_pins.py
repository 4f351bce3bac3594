"""Pins of the oracle's density filter (Sec. 2.2, Eqs. (4)-(5)) and of the
chain rule through it: a hand-worked example, a brute-force neighbour search,
partition of unity, the identity limit, linear precision, symmetry of H and
finite differences of a composite function."""

import json
import math
import os

import numpy as np

from oracle.filter import cell_centre_list, filter_apply, filter_grad, filter_matrix, filter_weights

HERE = os.path.dirname(os.path.abspath(__file__))


def test_golden_one_element_d2():
    g = json.load(open(os.path.join(HERE, "golden", "filter_1x1_d2.json")))
    H = filter_weights(g["nelx"], g["nely"], g["d"], g["R"]).toarray()
    W = filter_matrix(g["nelx"], g["nely"], g["d"], g["R"]).toarray()
    assert np.allclose(H, g["H"], atol=1e-15)
    assert np.allclose(W, g["W"], atol=1e-15)


def test_brute_force_neighbours_mixed_mesh():
    """The k-d tree search against a plain double loop over all cell pairs."""
    nelx, nely = 4, 3
    d = [1, 2, 3, 2, 1, 3, 2, 2, 1, 3, 1, 2]
    R = 0.7
    pts = cell_centre_list(nelx, nely, d)
    n = len(pts)
    Hb = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            dist = math.hypot(pts[i][0] - pts[j][0], pts[i][1] - pts[j][1])
            if dist < R:
                Hb[i, j] = R - dist
    H = filter_weights(nelx, nely, d, R).toarray()
    assert np.allclose(H, Hb, rtol=0, atol=1e-14)
    assert np.allclose(H, H.T, atol=1e-15)  # dist is symmetric


def test_cell_centres_by_hand():
    pts = cell_centre_list(2, 1, [1, 2])
    assert np.allclose(pts, [[0.5, 0.5], [1.25, 0.25], [1.75, 0.25], [1.25, 0.75], [1.75, 0.75]])


def test_partition_of_unity_and_constants():
    nelx, nely = 5, 4
    d = np.random.default_rng(1).integers(1, 6, nelx * nely)
    W = filter_matrix(nelx, nely, d, 0.45)
    assert np.allclose(np.asarray(W.sum(axis=1)).ravel(), 1.0, atol=1e-15)
    assert (W.data > 0).all()
    rho = np.full(W.shape[0], 0.37)
    assert np.allclose(W @ rho, 0.37, atol=1e-15)


def test_identity_below_cell_spacing():
    """R below the smallest distance between cell centres (1/d_max = 1/3):
    every cell sees only itself."""
    nelx, nely = 3, 3
    d = [1, 2, 3, 3, 2, 1, 2, 3, 1]
    rho = np.random.default_rng(2).uniform(0, 1, sum(k * k for k in d))
    assert np.array_equal(filter_apply(nelx, nely, d, 0.3, rho), rho)


def test_linear_precision_interior():
    """A symmetric neighbourhood averages a linear field to its centre value:
    exact on cells at least R from the boundary of a uniform-d region."""
    nelx, nely, dd, R = 6, 5, 2, 0.6
    d = [dd] * (nelx * nely)
    pts = cell_centre_list(nelx, nely, d)
    rho = 0.3 + 0.05 * pts[:, 0] - 0.02 * pts[:, 1]
    out = filter_apply(nelx, nely, d, R, rho)
    inner = (pts[:, 0] > R) & (pts[:, 0] < nelx - R) & (pts[:, 1] > R) & (pts[:, 1] < nely - R)
    assert inner.sum() > 20
    assert np.allclose(out[inner], rho[inner], rtol=0, atol=1e-15)
    assert not np.allclose(out[~inner], rho[~inner], atol=1e-6)  # one-sided at the boundary


def test_chain_rule_by_central_differences():
    """F(rho) = sum_i a_i rho~_i^2 + b . rho~: filter_grad(dF/drho~) against
    central differences on every cell of a small mixed mesh."""
    nelx, nely, R = 3, 2, 0.55
    d = [2, 1, 3, 3, 2, 1]
    rng = np.random.default_rng(3)
    n = sum(k * k for k in d)
    rho = rng.uniform(0.1, 0.9, n)
    a, b = rng.uniform(0.5, 2.0, n), rng.standard_normal(n)

    def F(r):
        t = filter_apply(nelx, nely, d, R, r)
        return float(np.sum(a * t * t) + b @ t)

    t = filter_apply(nelx, nely, d, R, rho)
    g = filter_grad(nelx, nely, d, R, 2 * a * t + b)
    h = 1e-6
    fd = np.array([(F(rho + h * np.eye(n)[k]) - F(rho - h * np.eye(n)[k])) / (2 * h) for k in range(n)])
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-9)
