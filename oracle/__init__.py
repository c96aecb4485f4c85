"""FP64 CPU oracle of the electron-phonon interpolation and scattering-rate path.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
cpu_baseline leg may import this package; the product library never does, and
this package imports nothing from the product.  It is a plain, slow, NumPy
float64 evaluation of what the paper defines, with LAPACK ``eigh`` for the
Hermitian eigenproblems, written so each step can be checked against the paper
by eye.

Every function cites the passage it follows (section and equation of the
Phoebe paper, arXiv:2111.14999).  Where the paper is silent or inconsistent
the reading taken is stated at the function.

Pins: each module's results are checked in ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force on tiny inputs and library special
cases (NumPy FFT).  Functions without such a pin say "parity unpinned".
"""

from . import constants, mesh, bands, coupling, rates, mlp, linewidth, polar, velocity, phonon3, rng  # noqa: F401
