"""CPU oracle for the FEA + sensitivity step of dp-adaptive multiresolution
topology optimization (Gupta, van Keulen, Langelaar, arXiv 1811.09821).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (its own basis, quadrature, numbering, assembly and solve), and it
imports nothing from ``paper_1811_09821_amd``.

What it computes, in plain FP64 (longdouble for residual accumulation):

* the element stiffness of Sec. 2.2 (K_e as a sum of B^T D B over quadrature
  points) in the composite per-density-cell form of Appendix B: one matrix
  K_s per density cell, integrated exactly with (p+1)^2 Gauss points;
* the modified SIMP modulus of Sec. 2.2, E(rho) = Emin + rho^q (E0 - Emin);
* the assembled global K, the solve Ku = f (Eq. ``eq_comp_1``) by a sparse
  direct factorisation followed by extended-precision iterative refinement;
* the density filter of Sec. 2.2 (Eqs. (4)-(5)) on the density cells and
  the chain rule through it (``filter.py``);
* the QR-error indicator of Sec. 3.2.3 (Eq. (9)): the element-level
  order-(p+1) problem under the element's own load and the strain-energy
  ratio (``qr.py``);
* the compliant-mechanism objective of Sec. 4.1 (force inverter, z = e_out)
  with ground springs, its adjoint (a unit load at the output DOF) and the
  bilinear sensitivity -E' lambda_e^T K_s u_e (``mechanism.py``);
* the refinement indicators and the dp update of Sec. 3.2-3.3: the Kelly
  gradient-jump estimator, the density-based indicator, the ranking and
  flagging steps and the order smoothing (``adapt.py``);
* compliance c = f^T u (Sec. 4.1, z = f) and the per-cell sensitivity
  dc/drho = -E'(rho) u_e^T K_s u_e (the paper names the sensitivity analysis
  in Sec. 1 and Sec. 2.1 but prints no formula; this is the adjoint result for
  the self-adjoint compliance, lambda = -u).

Every function cites the passage it follows; where the paper leaves a point
open (basis, mixed-p compatibility, layouts) the reading taken is stated
there.  Parity status: every function is pinned by ``-m "not gpu"``
tests in ``tests/test_oracle_pins.py``, ``tests/test_filter_pins.py``,
``tests/test_qr_pins.py``, ``tests/test_mechanism_pins.py`` and
``tests/test_adapt_pins.py``; none is "parity unpinned".
"""

from .fem import (  # noqa: F401
    basis_1d,
    constitutive_plane_stress,
    subcell_stiffness,
    simp_modulus,
    simp_modulus_derivative,
)
from .space import DofSpace, build_space  # noqa: F401
from .solve import oracle_solve, assemble, element_dofs_global  # noqa: F401
from .filter import filter_apply, filter_grad, filter_matrix, filter_weights  # noqa: F401
from .qr import element_qr_error, qr_error  # noqa: F401
from .mechanism import bilinear_sensitivity, mechanism  # noqa: F401
from .adapt import density_indicator, dp_update, kelly_indicator, qr_update  # noqa: F401
