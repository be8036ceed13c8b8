"""Oracle: a plain, slow, obviously correct CPU (NumPy complex128) implementation of
the time-stepped Schroedinger evolution of Hofmann & Schaller, "Probing nonlinear
adiabatic paths with a universal integrator" (arXiv:1311.3938).

TEST INFRASTRUCTURE ONLY.  This package is imported by the test suite, by the
package's smoke check and by the CPU-baseline leg of the benchmark.  The HIP
library and its Python binding never import, call or link anything here, and
nothing here imports them: the two implementations share no code.

Modules
  * ``sqh``          Pauli-string terms, path schedules and H(t)|psi> (Sec. II.A)
  * ``integrate``    classical RK4 and the one-evaluation 4th-order
                     predictor-corrector (Sec. II.B), fixed and adaptive steps
  * ``observables``  norm, overlap, energy, ground-state fidelity (Sec. III.B)
  * ``subspace``     states and evolution within one Hamming weight (Sec. III.A)
  * ``spectrum``     lowest eigenvalues and the gap of H(t) (Sec. IV.B)
  * ``tsearch``      the successful runtime T_s, E(T_s) = 1/2 (Sec. III.B)
"""
from . import sqh, integrate, observables, subspace, spectrum, tsearch  # noqa: F401
