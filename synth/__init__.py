"""Seeded synthetic inputs for the electron-phonon interpolation path.

This package builds the *inputs* of the method (real-space Hamiltonian H(R),
harmonic force constants Phi(R), atomic masses, real-space coupling
g(Re, Rp), meshes and rate parameters).  It holds none of the method's
arithmetic: no Fourier sums, no eigensolves, no couplings, no rates.  Both the
FP64 oracle (through the tests) and the GPU library consume what it returns.
"""

from .systems import (  # noqa: F401
    System,
    box_vectors,
    make_system,
    config_c1,
    config_c2,
    small_system,
    local_coupling_system,
    cscl_structure,
    perovskite_structure,
    random_structure,
    config_c4_specs,
    config_c4,
    add_polar,
    third_order_constants,
)
