"""Plain FP64 CPU oracle of the matrix-valued quantum lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library and never
imports it.

Representation: every discrete population W_i(x) is held as a complex128 2x2
Hermitian matrix, array shape ``[Q, *grid, 2, 2]`` with grid axes ordered
``(y, x)`` in 2D and ``(z, y, x)`` in 3D (x fastest).  This differs on purpose
from the library's real Pauli-coefficient layout, so that Hermiticity and the
Pauli bookkeeping are checked rather than assumed.

Modules
  constants  cubature weights, lattice constant and polynomial-equilibrium
             coefficients from their closed forms (Sec. 3.1, Appendix), mpmath
  lattice    the D2Q9 / D3Q19 velocity sets (Sec. 3, Fig. 1 caption, Sec. 3.1)
  fermi      complete Fermi-Dirac integrals and their inversion (Sec. 2.2)
  qlbm       moments, polynomial equilibrium, BGK collision, streaming, the
             Fermi-Dirac initial state and global observables (Sec. 3.3)
  eigen      the equilibrium built through the eigen-decomposition of rho and
             the Fermi-Dirac parameters (Prop. 1, Eqs. WeqFD, WeqDiscr)
  adjoint    reverse-mode derivative of the step and of the spin loss
  magnetic   the collision with an external magnetic field (Sec. 5)
  variants   the isothermal equilibrium (Sec. 3.1) and the positivity-limited
             relaxation rate (Sec. 3.3)
  euler      the exact solution of the Riemann problem of the Euler
             equations (Eq. Euler), the reference of the Riemann workload
  pauli      conversion between the matrix form and Pauli coefficients

Parity status: every function here is pinned by a CPU test against values the
paper prints, closed forms, library special functions or invariants.  The
polynomial equilibrium is pinned by its moments (continuum integration gives
the exact Fermi-Dirac moments, Sec. 3.2); its pointwise deviation from the
exact Fermi-Dirac function, which the paper shows only in a figure with no
number and no stated bound, is asserted only in the ordering the text states.
"""
