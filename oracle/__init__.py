"""Plain FP64 CPU oracle for the total-Lagrangian vectorial lattice Boltzmann method
(D2Q4 lattice, six-component vector populations) of Feng & Chu, arXiv 2605.26677.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package: only the
test suite, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import or call it.  It shares no code with the HIP library (no kernels, headers,
helpers or constant tables); the only thing both sides use is the seeded input generator
package ``lbm_inputs``, which holds none of the method's arithmetic.

The oracle is whole-array numpy in float64 and follows the paper's equations in the
paper's order and notation.  It deliberately stores the *unshifted* deformation gradient
F (populations carry F itself, not F - I), which is a different numerical formulation
from the library's shifted storage, so agreement between the two is a real test.

Modules
-------
material  hyperelastic closures of Appendix A: P(F), tangent C = dP/dF, energy W.
lbm       one time step of Sec. 3.7: moments (eq:moment-U), equilibrium (eq:feq),
          BGK collision with trapezoidal forcing (eq:collision), streaming
          (eq:streaming), half-way Dirichlet / Neumann rules (eq:boundary-general,
          eq:dirichlet-boundary-rule, eq:neumann-boundary-rule), second-order
          initialisation (eq:init-compact .. eq:init-expanded), displacement
          quadrature (eq:trapezoid-u).
adjoint   hand-written reverse sweep of the same map (gradient of a probe
          displacement loss w.r.t. per-cell mu, lambda, body force and initial velocity).
symbol    24x24 Fourier symbol of the step linearised about the rest state
          (stability and dispersion of the linear lattice dynamics).
mms       the periodic manufactured solution of Sec. 4.1 (eq:periodic-mms-displacement,
          eq:mms-body-force).
"""
