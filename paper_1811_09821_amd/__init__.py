"""MI355X (gfx950) library for the FEA + sensitivity step of dp-adaptive
multiresolution topology optimization (arXiv 1811.09821).

    from paper_1811_09821_amd import mto, problems
    plan = mto.Plan(problems.config(2))
    u, c, g, stats = plan.solve(rho_cuda)

``mto`` is the ctypes binding of libmto.so (include/mto.h); ``autograd``
holds the torch.autograd.Function (densities -> sum of compliances);
``problems`` holds the seeded synthetic input generators.
"""

__all__ = ["mto", "problems", "autograd", "build"]
