"""Density filter of Sec. 2.2 (Eqs. (4)-(5)) on the density cells, and the
chain rule through it.

Test infrastructure only (see the package docstring).

The paper filters the background densities onto the integration points:
rho~_i = sum_j H_ij rho^_j / sum_j H_ij with H_ij = R - dist(i, j) over the
cells j whose centres lie within R of point i (Eqs. (4)-(5)).  With the
composite integration of Appendix B every density cell is integrated with
one constant modulus, so the point i of a cell is taken to be its centre:
cell i gets rho~_i from the cells of the whole mesh (across element
boundaries) within R of its centre.  Lengths are in element edge lengths
(elements are unit squares, cell s = sy*d + sx of element e = ey*nelx + ex
has its centre at (ex + (sx + 1/2)/d, ey + (sy + 1/2)/d)).

Chain rule: for a function J of the filtered densities,
dJ/drho_j = sum_i (dJ/drho~_i) H_ij / sum_k H_ik, i.e. the transpose of the
row-normalised filter matrix applied to the gradient.
"""

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree


def cell_centre_list(nelx, nely, d):
    """Centres of all density cells, element-major, cell order sy*d + sx."""
    d = np.asarray(d, dtype=np.int64).ravel()
    pts = []
    for e in range(nelx * nely):
        ex, ey, de = e % nelx, e // nelx, int(d[e])
        for s in range(de * de):
            sx, sy = s % de, s // de
            pts.append((ex + (sx + 0.5) / de, ey + (sy + 0.5) / de))
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


def filter_weights(nelx, nely, d, R):
    """The matrix H of Eq. (5): H_ij = R - dist(i, j) where positive
    (CSR, one row per cell, columns in increasing order)."""
    if not R > 0.0:
        raise ValueError("filter radius must be positive")
    pts = cell_centre_list(nelx, nely, d)
    n = len(pts)
    tree = cKDTree(pts)
    D = tree.sparse_distance_matrix(tree, R, output_type="coo_matrix")
    keep = (D.row != D.col) & (D.data < R)
    rows = np.concatenate([D.row[keep], np.arange(n)])
    cols = np.concatenate([D.col[keep], np.arange(n)])
    vals = np.concatenate([R - D.data[keep], np.full(n, float(R))])  # dist(i, i) = 0
    H = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    H.sort_indices()
    return H


def filter_matrix(nelx, nely, d, R):
    """Row-normalised filter W = diag(1 / sum_j H_ij) H (Eq. (4))."""
    H = filter_weights(nelx, nely, d, R)
    rs = np.asarray(H.sum(axis=1)).ravel()
    return sp.diags(1.0 / rs) @ H


def filter_apply(nelx, nely, d, R, rho):
    """rho~ = W rho (Eq. (4))."""
    return filter_matrix(nelx, nely, d, R) @ np.asarray(rho, dtype=np.float64)


def filter_grad(nelx, nely, d, R, g_tilde):
    """dJ/drho = W^T dJ/drho~ (chain rule through Eq. (4))."""
    return filter_matrix(nelx, nely, d, R).T @ np.asarray(g_tilde, dtype=np.float64)
