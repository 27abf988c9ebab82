"""FP64 CPU oracle for the curvature phase-field energy F_eps and its gradient.

TEST INFRASTRUCTURE ONLY: it checks the HIP path and is never part of it. Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it. It imports nothing from the product package, and the product
package imports nothing from it.

Modules:
  fe_oracle     the discrete energy, its hand-derived adjoint gradient, the
                mass-projected descent step (eqs. (Meps), (Feps); Sec. 4.1), and
                the H^-1 flow of Algorithm 1 (div A + m0, blur, Adam on A)
  classical     Cahn-Hilliard, Willmore and Helfrich phase fields, the diffuse
                curvatures, each from its own equation (Secs. 2.3, 3.1), and the
                diagnostics built on them (curvature histogram, discrepancy)
  closed_forms  continuum values on tanh-profile spheres, cylinders and planes by
                co-area quadrature (Sec. 3.2)
  params        coefficient vectors: eq. (redundant), Helfrich, inside-out swap
  l2flow        Algorithm 2: replicate boundaries, the blur with replicate padding,
                and L-BFGS (Sec. 4.2)
"""

from .fe_oracle import (XI, double_well, double_well_prime, fd_gradient, fd_hessian,
                        fd_laplacian, feps_coefficients, softplus, logistic, pointwise,
                        energy, energy_abs, adjoint_fields, energy_grad, mass_projected_step,
                        descend, adam_projected_step, descend_adam, energy_grad_batch,
                        fd_divergence, gaussian_weights, gaussian_blur, hminus_energy,
                        hminus_energy_grad, hminus_adam_step, hminus_descend,
                        transpose_stencils)

__all__ = ["XI", "double_well", "double_well_prime", "fd_gradient", "fd_hessian",
           "fd_laplacian", "feps_coefficients", "softplus", "logistic", "pointwise", "energy",
           "energy_abs", "adjoint_fields", "energy_grad", "mass_projected_step", "descend",
           "adam_projected_step", "descend_adam", "energy_grad_batch", "fd_divergence",
           "gaussian_weights", "gaussian_blur", "hminus_energy", "hminus_energy_grad",
           "hminus_adam_step", "hminus_descend", "transpose_stencils"]
