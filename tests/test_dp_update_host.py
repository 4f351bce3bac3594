"""The library's dp update (Sec. 3.3, host code behind the C ABI) against
the oracle: integer outputs, so bit-exact."""

import numpy as np
import pytest

from oracle.adapt import dp_update as dp_oracle, qr_update as qr_oracle, smooth_p
from paper_1811_09821_amd import mto


def test_worked_case():
    p, th, dp, cells = mto.dp_update(4, 1, [2, 2, 2, 2], [0.1, 0.4, 0.3, 0.2], [-0.1, 0.0, 0.2, -0.3],
                                     frac_a_refine=0.25, frac_a_coarsen=0.25, p_max=5)
    assert list(p) == [1, 3, 3, 1] and list(th) == [-2, 1, 0, 0] and list(dp) == [1, 29, 29, 5] and cells == 36


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("p_max", [4, 5])
def test_matches_oracle(seed, p_max):
    rng = np.random.default_rng(seed)
    nelx, nely = int(rng.integers(1, 17)), int(rng.integers(1, 9))
    n = nelx * nely
    p0 = smooth_p(rng.integers(1, p_max + 1, n), nelx, nely)
    ga = rng.standard_normal(n)
    gd = rng.standard_normal(n) * (rng.random(n) < 0.7)
    if seed % 2:  # ties in the rankings
        ga = np.round(ga, 1)
        gd = np.round(gd, 1)
    kw = dict(frac_a_refine=[0.1, 0.3][seed % 2], frac_a_coarsen=[0.05, 0.2][seed % 2],
              frac_d_refine=[1.0, 0.5][seed % 2], frac_d_coarsen=[1.0, 0.7][seed % 2], p_max=p_max)
    p, th, dp, cells = mto.dp_update(nelx, nely, p0, ga, gd, **kw)
    po, tho, dpo, cellso = dp_oracle(nelx, nely, p0, ga, gd, **kw)
    assert np.array_equal(p, po) and np.array_equal(th, tho) and np.array_equal(dp, dpo) and cells == cellso


def test_qr_update_matches_oracle():
    rng = np.random.default_rng(9)
    p = rng.integers(1, 5, 50)
    eps = rng.random(50)
    assert np.array_equal(mto.qr_update(p, eps, 0.6, 4), qr_oracle(p, eps, 0.6, 4))


def test_rejects_bad_parameters():
    with pytest.raises(mto.MtoError):
        mto.dp_update(2, 1, [1, 1], [0.0, 0.0], [0.0, 0.0], frac_a_refine=1.5)
    with pytest.raises(mto.MtoError):
        mto.dp_update(2, 1, [0, 1], [0.0, 0.0], [0.0, 0.0])
