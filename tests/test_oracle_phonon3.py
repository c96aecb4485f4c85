"""Pins of the three-phonon coupling interpolation V3 (Phonon Properties; Kokkos section).

* the two-stage evaluation (sum over R at fixed q, then over R' per q')
  against explicit loops over (R, R') and direct rotations;
* permutation symmetry: for constants symmetric under every permutation of
  the three displacements, V3(q nu, q' nu', q'' nu'') = V3(q' nu', q nu, q'' nu'')
  exactly, and |V3| is unchanged by the cyclic order (q'', q, q');
* invariance of |V3| under a global Cartesian rotation of the harmonic and
  third-order constants;
* closed form: Einstein phonons (z = 1) and constants at R = R' = 0 only give
  V3 = Phi3[0, 0] l l l at every (q, q').
"""

import copy
import math

import numpy as np
import scipy.constants as sc

import synth
from helpers import random_rotation
from oracle import phonon3

C_OMEGA = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt
C_PH = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt


def _system3(seed=5, nat=2):
    s = synth.small_system(seed, n_wannier=1, n_atoms=nat, r=1)
    r, phi3 = synth.third_order_constants(seed, nat)
    s.r1 = r
    s.r2 = r
    s.phi3 = phi3
    return s


def test_generator_translation_symmetry():
    s = _system3()
    idx = {tuple(int(x) for x in v): i for i, v in enumerate(s.r1)}
    R, Rp = np.array([1, 0, -1]), np.array([0, 1, 1])
    a = s.phi3[idx[tuple(R)], idx[tuple(Rp)]]
    # Phi3(x1 R, x2 R', x3 0) = Phi3(x3 -R', x1 R-R', x2 0)
    b = s.phi3[idx[tuple(-Rp)], idx[tuple(R - Rp)]]
    assert np.max(np.abs(a - np.transpose(b, (1, 2, 0)))) < 1e-15
    assert np.max(np.abs(a)) > 0


def test_two_stage_matches_explicit_loops():
    s = _system3(seed=6, nat=1)
    rng = np.random.default_rng(1)
    q = rng.uniform(-1, 1, size=(2, 3))
    qp = rng.uniform(-1, 1, size=(3, 3))
    out = phonon3.interp_v3(q, qp, s)["v3"]
    ref = phonon3.interp_v3_brute(q, qp, s)
    assert np.max(np.abs(out - ref)) < 1e-11 * np.max(np.abs(ref))


def test_permutation_symmetry():
    s = _system3(seed=7, nat=2)
    rng = np.random.default_rng(2)
    q = rng.uniform(-1, 1, size=(1, 3))
    qp = rng.uniform(-1, 1, size=(1, 3))
    a = phonon3.interp_v3(q, qp, s)["v3"][0, 0]
    b = phonon3.interp_v3(qp, q, s)["v3"][0, 0]
    assert np.max(np.abs(a - np.transpose(b, (1, 0, 2)))) < 1e-11 * np.max(np.abs(a))
    qpp = -q - qp
    c = phonon3.interp_v3(qpp, q, s)["v3"][0, 0]       # (q'' nu'', q nu, q' nu')
    assert np.max(np.abs(np.abs(a) - np.abs(np.transpose(c, (1, 2, 0))))) < 1e-10 * np.max(np.abs(a))


def test_cartesian_rotation_invariance():
    s = _system3(seed=8, nat=2)
    O = random_rotation(np.random.default_rng(3))
    Ob = np.kron(np.eye(2), O)
    s2 = copy.deepcopy(s)
    s2.phi_r = Ob[None] @ s.phi_r @ Ob.T[None]
    s2.phi3 = np.einsum("ai,bj,ck,xyijk->xyabc", Ob, Ob, Ob, s.phi3)
    rng = np.random.default_rng(4)
    q = rng.uniform(-1, 1, size=(2, 3))
    qp = rng.uniform(-1, 1, size=(2, 3))
    a = np.abs(phonon3.interp_v3(q, qp, s)["v3"])
    b = np.abs(phonon3.interp_v3(q, qp, s2)["v3"])
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(a)


def test_einstein_closed_form():
    M = 1.7
    kk = np.array([0.6, 1.1, 1.45])
    R = synth.box_vectors(1)
    phi = np.zeros((27, 3, 3))
    phi[13] = np.diag(kk)
    rng = np.random.default_rng(9)
    p3 = np.zeros((27, 27, 3, 3, 3))
    p3[13, 13] = rng.standard_normal((3, 3, 3))
    s = synth.System(n_wannier=1, n_atoms=1, positions=np.zeros((1, 3)), mass=np.array([M]),
                     rh=R, h_r=np.zeros((27, 1, 1), complex), rd=R, phi_r=phi, re=R, rp=R,
                     g_rr=None)
    s.r1, s.r2, s.phi3 = R, R, p3
    w = C_OMEGA * np.sqrt(kk / M)
    l = np.sqrt(C_PH / (2 * M * w))
    ref = p3[13, 13] * l[:, None, None] * l[None, :, None] * l[None, None, :]
    q = rng.uniform(-1, 1, size=(3, 3))
    qp = rng.uniform(-1, 1, size=(2, 3))
    out = phonon3.interp_v3(q, qp, s)["v3"]
    # z = 1 up to the sign of each column: compare magnitudes
    # (scipy's and the oracle's CODATA revisions differ near 1e-10)
    assert np.max(np.abs(np.abs(out) - np.abs(ref)[None, None])) < 1e-9 * np.max(np.abs(ref))
