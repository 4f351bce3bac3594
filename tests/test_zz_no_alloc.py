"""GPU: the allocation-free stiffness product (mto_apply_stiffness_noalloc)
against the allocating one (mto_apply_stiffness), through the C ABI.

Both run the same kernels on the same inputs, the first with its scratch
(cell moduli, gathered x, element slots) in the library's static device
array, so the results must be bit-identical.  Two calls in a row, the second
on a smaller plan, check that the array's leftover contents from the first
call do not leak into the second (its slots are cleared each call); a plan
whose scratch exceeds the array is rejected with MTO_EINVAL."""

import numpy as np
import pytest
import torch

from paper_1811_09821_amd import problems as P

pytestmark = pytest.mark.gpu


def _case(pr, seed, cuda):
    from paper_1811_09821_amd import mto

    plan = mto.Plan(pr)
    rho = torch.tensor(pr.rho, device=cuda)
    x = torch.tensor(np.random.default_rng(seed).standard_normal(plan.info["n_u"]), device=cuda)
    return plan, rho, x


def test_noalloc_product_matches_allocating_entry_point(cuda):
    from paper_1811_09821_amd import mto

    big = P.cantilever_uniform(48, 24, 3, 4, sigma=4.0, volfrac=0.4, seed=12)
    small = P.small_mixed(9, 5, seed=13, n_loads=2)
    for pr, seed in ((big, 1), (small, 2)):
        print(f"\nno-alloc product: {pr.name}, {pr.nel} elements, {pr.n_load_cases} load case(s)", flush=True)
        plan, rho, x = _case(pr, seed, cuda)
        y_ref = plan.apply_stiffness(rho, x)
        y = torch.full_like(y_ref, float("nan"))
        rc = mto.lib().mto_apply_stiffness_noalloc(plan.handle, mto._ptr(rho), mto._ptr(x), mto._ptr(y),
                                                   mto._stream(None))
        assert rc == mto.MTO_OK, mto.lib().mto_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), float((y - y_ref).abs().max())
        # and once more through the binding, into a reused output buffer
        plan.apply_stiffness_noalloc(rho, x, y)
        assert torch.equal(y, y_ref)


def test_noalloc_rejects_plans_beyond_the_scratch(cuda):
    from paper_1811_09821_amd import mto

    pr = P.config(5)  # three load cases on the 400 x 200 mixed mesh: about 80 MB of scratch
    plan, rho, x = _case(pr, 3, cuda)
    y = torch.empty_like(x)
    rc = mto.lib().mto_apply_stiffness_noalloc(plan.handle, mto._ptr(rho), mto._ptr(x), mto._ptr(y),
                                               mto._stream(None))
    assert rc == mto.MTO_EINVAL
    assert "scratch" in mto.lib().mto_last_error().decode()
