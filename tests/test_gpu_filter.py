"""GPU parity of the density filter (Sec. 2.2, Eqs. (4)-(5)) and its chain
rule against the oracle's sparse W = diag(1 / rowsum) H.

Tolerance (written here): max-norm relative error 1e-14 for W rho and
W^T g.  Each output is a sum of at most a few hundred positive-weight terms
whose weights are formed in a different order (the library stores H and
1/rowsum; the oracle forms W), so the difference is a few units of rounding.
"""

import numpy as np
import pytest
import torch

from oracle import filter_apply, filter_grad, filter_matrix, oracle_solve
from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu

F_TOL = 1e-14


def mto():
    from paper_1811_09821_amd import mto as m

    return m


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def check_filter(cuda, prs, R, seed):
    m = mto()
    prs = prs if isinstance(prs, list) else [prs]
    F = m.Filter(prs, R)
    n = sum(pr.n_cells for pr in prs)
    assert F.n_cells == n
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    gt = rng.standard_normal(n)
    y = F.apply(torch.tensor(x, device=cuda)).cpu().numpy()
    g = F.grad(torch.tensor(gt, device=cuda)).cpu().numpy()
    yo, go, nnz, off = [], [], 0, 0
    for pr in prs:
        W = filter_matrix(pr.nelx, pr.nely, pr.d, R)
        nnz += W.nnz
        yo.append(W @ x[off:off + pr.n_cells])
        go.append(W.T @ gt[off:off + pr.n_cells])
        off += pr.n_cells
    yo, go = np.concatenate(yo), np.concatenate(go)
    assert F.nnz == nnz
    assert rel_max(y, yo) < F_TOL, rel_max(y, yo)
    assert rel_max(g, go) < F_TOL, rel_max(g, go)
    return F


@pytest.mark.parametrize("R", [0.3, 0.75, 1.0, 1.6, 2.5])
def test_filter_mixed_mesh(cuda, R):
    """Mixed d (the dp rule gives 2 and 5 here) across element boundaries."""
    check_filter(cuda, P.small_mixed(13, 7, seed=71), R, 71)


@pytest.mark.parametrize("d", [1, 3, 5, 8])
def test_filter_uniform_d(cuda, d):
    """Uniform d; 13 x 5 elements so the slices of 64 rows end ragged."""
    check_filter(cuda, P.uniform_random(13, 5, 2, d, 72), 0.9, 72)


def test_filter_batch_keeps_instances_apart(cuda):
    """A batch of uneven instances: no weight couples two instances."""
    prs = [P.small_mixed(9, 4, seed=73), P.uniform_random(1, 1, 1, 1, 74), P.uniform_random(6, 11, 3, 3, 75)]
    check_filter(cuda, prs, 1.3, 76)


def test_filter_single_cell_and_tiny_radius(cuda):
    """Degenerate cases: one cell (W = 1), and R below every cell spacing
    (W = I) on a mesh whose last slice has a single row."""
    check_filter(cuda, P.uniform_random(1, 1, 1, 1, 77), 0.5, 77)
    pr = P.uniform_random(5, 5, 1, 3, 78)  # 225 cells = 3 * 64 + 33
    F = check_filter(cuda, pr, 0.3, 78)
    assert F.nnz == pr.n_cells


@pytest.mark.parametrize("cfg,R", [(2, 0.3), (2, 1.5), (3, 0.3), (5, 0.3)])
def test_filter_full_size(cuda, cfg, R):
    """The full design meshes (160 x 80 uniform d = 4, 200 x 100 and
    400 x 200 mixed) at the paper's radius 0.3 and a wider one."""
    check_filter(cuda, P.config(cfg), R, 79)


def test_filter_is_deterministic_and_rejects_in_place(cuda):
    m = mto()
    pr = P.small_mixed(8, 4, seed=80)
    F = m.Filter(pr, 1.2)
    x = torch.rand(pr.n_cells, dtype=torch.float64, device=cuda)
    assert torch.equal(F.apply(x), F.apply(x))
    assert torch.equal(F.grad(x), F.grad(x))
    with pytest.raises(m.MtoError) as ei:
        m._check(m.lib().mto_filter_apply(F.handle, m._ptr(x), m._ptr(x), m._stream(None)))
    assert ei.value.code == m.MTO_EINVAL
    with pytest.raises(ValueError):
        F.apply(torch.rand(pr.n_cells + 1, dtype=torch.float64, device=cuda))


def test_filter_autograd_gradcheck(cuda):
    """DensityFilter is linear: gradcheck of its backward (W^T) against
    finite differences of its forward."""
    m = mto()
    from paper_1811_09821_amd.autograd import DensityFilter

    pr = P.small_mixed(4, 3, seed=81)
    F = m.Filter(pr, 1.1)
    x = torch.rand(pr.n_cells, dtype=torch.float64, device=cuda, requires_grad=True)
    assert torch.autograd.gradcheck(lambda r: DensityFilter.apply(r, F), (x,), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_filtered_compliance_gradient_matches_oracle(cuda):
    """c(W rho) and its gradient W^T (dc/drho~) against the oracle: the
    filter, the solve at the filtered densities and the chain rule."""
    m = mto()
    from paper_1811_09821_amd.autograd import filtered_total_compliance

    pr = P.small_mixed(14, 7, seed=82, n_loads=2)
    R = 0.6
    plan = m.Plan(pr)
    F = m.Filter(pr, R)
    rho = torch.tensor(pr.rho, device=cuda, requires_grad=True)
    J = filtered_total_compliance(rho, plan, F)
    J.backward()
    rt = filter_apply(pr.nelx, pr.nely, pr.d, R, pr.rho)
    args = pr.oracle_args()
    args["rho"] = rt
    o = oracle_solve(**args)
    assert abs(J.item() - o["c"].sum()) < 1e-8 * o["c"].sum()
    gref = filter_grad(pr.nelx, pr.nely, pr.d, R, o["g"].sum(axis=0))
    gg = rho.grad.cpu().numpy()
    assert np.linalg.norm(gg - gref) < 1e-7 * np.linalg.norm(gref)
