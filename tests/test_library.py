"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/mto.h declares, and rejects bad input before any device
work."""

import os
import re

import numpy as np
import pytest

from paper_1811_09821_amd import mto
from paper_1811_09821_amd import problems as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mto.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(mto_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = mto.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mto.EXPORTED)


def test_version_string():
    assert "gfx950" in mto.version()


def _err(prob, **kw):
    with pytest.raises(mto.MtoError) as ei:
        mto.Plan(prob, **kw)
    return ei.value.code


def test_rejects_order_and_grid_out_of_range():
    assert _err(P.uniform_random(3, 2, 5, 1, 0)) == mto.MTO_EINVAL
    assert _err(P.uniform_random(3, 2, 0, 1, 0)) == mto.MTO_EINVAL
    assert _err(P.uniform_random(3, 2, 2, 9, 0)) == mto.MTO_EINVAL


@pytest.mark.parametrize("sup", [
    [],                                   # nothing fixed
    [(0, 0, 0, 3)],                       # one vertex: rotation free
    [(1, 0, 0, 1)],                       # x only on the left edge: y translation free
    [(0, 0, 0, 1), (0, 3, 0, 2)],         # one x row and one y row: rotation free
    [(3, 0, 0, 2)],                       # y on the bottom edge: x translation free
])
def test_rejects_supports_leaving_rigid_modes(sup):
    pr = P.uniform_random(3, 2, 2, 1, 0, supports=sup, loads=[(3, 1, 0.0, -1.0, 0)])
    assert _err(pr) == mto.MTO_ESINGULAR


@pytest.mark.parametrize("sup", [
    [(0, 0, 0, 3), (0, 3, 0, 2)],         # pin + roller (MBB-like)
    [(1, 0, 0, 1), (0, 3, 0, 2)],         # symmetry edge + roller
    [(0, 0, 0, 1), (0, 0, 2, 1), (0, 3, 0, 2)],
])
def test_accepts_sufficient_supports_until_device_work(sup):
    """Host validation passes; plan creation then fails only for lack of a
    GPU (or succeeds on one)."""
    pr = P.uniform_random(3, 2, 2, 1, 0, supports=sup, loads=[(3, 2, 0.0, -1.0, 0)])
    try:
        plan = mto.Plan(pr)
        plan.close()
    except mto.MtoError as e:
        assert e.code in (mto.MTO_EHIP, mto.MTO_ENOMEM), e


def test_rejects_an_instance_without_free_dofs():
    """Every edge clamped in both directions on a 1 x 1, p = 1 mesh leaves no
    free DOF: nothing to solve, so the plan is refused."""
    sup = [(k, 0, 0, 3) for k in (P.SUP_EDGE_LEFT, P.SUP_EDGE_RIGHT, P.SUP_EDGE_BOTTOM, P.SUP_EDGE_TOP)]
    pr = P.uniform_random(1, 1, 1, 1, 0, supports=sup, loads=[(1, 1, 0.0, -1.0, 0)])
    with pytest.raises(mto.MtoError) as ei:
        mto.Plan(pr)
    assert ei.value.code == mto.MTO_EINVAL
    assert "no free DOFs" in str(ei.value)


def test_rejects_bad_loads_and_supports():
    pr = P.uniform_random(3, 2, 1, 1, 0, loads=[(0, 1, 0.0, -1.0, 0)])  # load on the clamped edge
    assert _err(pr) == mto.MTO_EINVAL
    pr = P.uniform_random(3, 2, 1, 1, 0, loads=[(4, 1, 0.0, -1.0, 0)])  # vertex outside
    assert _err(pr) == mto.MTO_EINVAL
    pr = P.uniform_random(3, 2, 1, 1, 0, loads=[(3, 1, 0.0, -1.0, 1)])  # load case out of range
    assert _err(pr) == mto.MTO_EINVAL
    pr = P.uniform_random(3, 2, 1, 1, 0, supports=[(1, 0, 0, 4)])       # bad component mask
    assert _err(pr) == mto.MTO_EINVAL
    pr = P.uniform_random(3, 2, 1, 1, 0, supports=[(7, 0, 0, 3)])       # unknown kind
    assert _err(pr) == mto.MTO_EINVAL


def test_rejects_bad_params():
    pr = P.uniform_random(3, 2, 1, 1, 0)
    assert _err(pr, rtol=0.0) == mto.MTO_EINVAL
    assert _err(pr, nu=0.5) == mto.MTO_EINVAL
    assert _err(pr, Emin=2.0) == mto.MTO_EINVAL
    assert _err(pr, kernel_path=7) == mto.MTO_EINVAL


def test_binding_type_checks():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        mto._f64_cuda(np.zeros(3), 3, "x")
    with pytest.raises(TypeError):
        mto._f64_cuda(torch.zeros(3, dtype=torch.float32), 3, "x")
    with pytest.raises(TypeError):
        mto._f64_cuda(torch.zeros(3, dtype=torch.float64), 3, "x")  # host tensor


def test_generators_are_seeded_and_shaped():
    a, b = P.config(2), P.config(2)
    assert np.array_equal(a.rho, b.rho)
    assert a.nel == 12800 and a.n_cells == 204800
    assert abs(np.mean(a.rho) - 0.4) < 1e-9 and a.rho.min() >= 1e-3 and a.rho.max() <= 1.0
    m = P.config(3)
    groups = set(zip(m.p.tolist(), m.d.tolist()))
    assert groups <= {(4, 5), (2, 2), (1, 1), (2, 1)} and (4, 5) in groups
    frac = float(np.mean(m.p == 4))
    assert 0.12 < frac < 0.3
    # neighbouring orders differ by at most 2 (smoothing step of Sec. 3.3)
    pp = m.p.reshape(m.nely, m.nelx).astype(int)
    assert np.abs(np.diff(pp, axis=0)).max() <= 2 and np.abs(np.diff(pp, axis=1)).max() <= 2


def test_filter_rejects_bad_radius_and_mesh():
    """mto_filter_create validates R and d on the host before any device work."""
    pr = P.uniform_random(3, 2, 2, 2, 0)
    for R in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(mto.MtoError) as ei:
            mto.Filter(pr, R)
        assert ei.value.code == mto.MTO_EINVAL
    bad = P.uniform_random(3, 2, 2, 2, 0)
    bad.d = bad.d.copy()
    bad.d[1] = 9
    with pytest.raises(mto.MtoError) as ei:
        mto.Filter(bad, 0.5)
    assert ei.value.code == mto.MTO_EINVAL


@pytest.mark.parametrize("spr", [[(3, 0, 0, 1.0), (0, 2, 0, 1.0)],  # second one on the clamped vertex
                                 [(3, 0, 2, 1.0)], [(3, 0, 0, 0.0)], [(9, 0, 0, 1.0)]])
def test_rejects_bad_springs(spr):
    """Ground springs are checked on the host: vertex, component, k > 0, and
    not on a supported DOF."""
    pr = P.force_inverter(3, 2, p=1, d=1)
    pr.springs = spr
    assert _err(pr) == mto.MTO_EINVAL
