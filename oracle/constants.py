"""Unit conversions used by the oracle (CODATA 2018 SI values).

The paper leaves units implicit.  Reading taken: energies in eV, lengths in
Angstrom, masses in amu, force constants in eV/A^2, couplings g(Re,Rp) in eV/A,
and hbar = 1 in the rate formula so Gamma = hbar/tau is an energy in eV.

* phonon energy (Phonon Properties, eigenvalue equation of D):
  hbar*omega = C_OMEGA * sqrt(lambda) with lambda in eV/(A^2 amu);
* zero-point length of the 1/sqrt(2 m omega) factor (Electron Properties,
  definition of g): l^2 = C_PH / (2 M hbar*omega), l in A when M in amu and
  hbar*omega in eV.
"""

import math

HBAR_SI = 1.054571817e-34       # J s
EV_SI = 1.602176634e-19         # J (exact)
AMU_SI = 1.66053906660e-27      # kg
ANGSTROM_SI = 1.0e-10           # m
KB_SI = 1.380649e-23            # J/K (exact)

#: hbar * sqrt(eV / (A^2 amu)) expressed in eV
C_OMEGA = HBAR_SI * math.sqrt(EV_SI / (ANGSTROM_SI ** 2 * AMU_SI)) / EV_SI
#: hbar^2 / (amu A^2) expressed in eV
C_PH = HBAR_SI ** 2 / (AMU_SI * ANGSTROM_SI ** 2) / EV_SI
#: Boltzmann constant in eV/K
KB_EV = KB_SI / EV_SI


def kT_of(temperature_k: float) -> float:
    return KB_EV * temperature_k

EPS0_SI = 8.8541878128e-12      # F/m
#: e^2 / (4 pi eps0) expressed in eV A (the Coulomb constant of the polar coupling)
E2_4PIEPS0 = EV_SI / (4.0 * math.pi * EPS0_SI * ANGSTROM_SI)
