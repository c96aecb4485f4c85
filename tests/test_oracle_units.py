"""Unit conversions of the oracle pinned against scipy.constants (an independent source).

scipy may ship a newer CODATA set than the 2018 values the oracle uses; the
atomic mass unit moved by ~1e-9 relative between them, hence 1e-8 tolerances.
"""

import math

import scipy.constants as sc

from oracle import constants as oc


def test_c_omega_matches_scipy():
    # hbar * omega for a 1 eV/A^2 spring on a 1 amu mass, in eV
    w = math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass)
    assert abs(oc.C_OMEGA - sc.hbar * w / sc.electron_volt) < 1e-8 * oc.C_OMEGA
    assert abs(oc.C_OMEGA - 0.0646541513) < 1e-9


def test_c_ph_matches_scipy():
    c = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt
    assert abs(oc.C_PH - c) < 1e-8 * c
    assert abs(oc.C_PH - 4.18015928e-3) < 1e-11


def test_kb_matches_scipy():
    assert abs(oc.KB_EV - sc.k / sc.electron_volt) < 1e-15
    assert abs(oc.kT_of(300.0) - 0.025852) < 1e-6
