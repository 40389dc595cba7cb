"""FP64 CPU oracle of the lattice-Boltzmann stream-and-collide step.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg import it; the product path never does.  It shares no code with
the HIP library or its Python binding.

Modules
    lbm       stencils, equilibrium (Eq. 3), moments (Eq. 4), BGK (Eq. 2), streaming
              (Eq. 1), Guo forcing (textbook), the pull-convention step
    storage   stored-population formats and the emulated reduced-precision step
    adjoint   reverse-mode derivatives by torch autograd (Sec. 3.2's route)
    spectrum  shell energy spectrum and the log-spectrum loss

Parity pins: every function is checked in tests/test_oracle_*.py against facts fixed
by the paper or by mathematics (closed forms, invariants, brute force, finite
differences).  No function is left unpinned.
"""
from . import lbm, storage, adjoint, spectrum  # noqa: F401
