"""Pins of the band-structure step (Phonon and Electron Properties).

* Hermiticity of H(k) and D(q) from H(-R) = H(R)^dagger and the
  force-constant symmetry;
* eigen-residuals and orthonormality of the LAPACK eigenpairs;
* acoustic sum rule: exactly three zero modes at q = 0, none elsewhere;
* closed forms: monatomic simple cubic with axis springs (textbook), the
  diatomic chain (textbook), and a single Wannier function (nW = 1).
"""

import math

import numpy as np
import pytest
import scipy.constants as sc

import synth
from oracle import bands, mesh


C_OMEGA_SCIPY = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt


@pytest.mark.parametrize("make", [lambda: synth.config_c1(), lambda: synth.small_system(11, 5, 5, 1)])
def test_hermitian_and_residuals(make):
    s = make()
    rng = np.random.default_rng(0)
    k = rng.uniform(-1, 1, size=(20, 3))
    H = bands.hamiltonian_k(k, s.rh, s.h_r)
    assert np.max(np.abs(H - np.conj(np.swapaxes(H, 1, 2)))) < 1e-14 * np.max(np.abs(H))
    D = bands.dynamical_matrix(k, s.rd, s.phi_r, s.mass)
    assert np.max(np.abs(D - np.conj(np.swapaxes(D, 1, 2)))) < 1e-14 * np.max(np.abs(D))
    eps, U = bands.electron_bands(k, s.rh, s.h_r)
    assert np.all(np.diff(eps, axis=1) >= 0)
    res = H @ U - U * eps[:, None, :]
    assert np.max(np.abs(res)) < 1e-13 * np.max(np.abs(eps))
    I = np.conj(np.swapaxes(U, 1, 2)) @ U
    assert np.max(np.abs(I - np.eye(s.n_wannier))) < 1e-13


@pytest.mark.parametrize("make", [lambda: synth.config_c1(), lambda: synth.small_system(11, 2, 5, 1)])
def test_acoustic_sum_rule(make):
    s = make()
    w, z, lam = bands.phonon_modes(np.zeros((1, 3)), s.rd, s.phi_r, s.mass)
    scale = np.max(np.abs(lam))
    assert np.sum(np.abs(lam[0]) < 1e-12 * scale) == 3
    pts = mesh.mesh_points((4, 4, 4))[1:]
    w, z, lam = bands.phonon_modes(pts, s.rd, s.phi_r, s.mass)
    assert np.min(lam) > 1e-6 * scale


def _axis_spring_phi(k_long, alpha):
    """Monatomic SC, bonds to the six axis neighbours: Phi(+-e_i) = -K_i, Phi(0) = 2 sum K_i."""
    R = synth.box_vectors(1)
    idx = {tuple(r): i for i, r in enumerate(R)}
    phi = np.zeros((R.shape[0], 3, 3))
    for ax in range(3):
        K = alpha * k_long * np.eye(3)
        K[ax, ax] = k_long
        for sgn in (1, -1):
            e = [0, 0, 0]
            e[ax] = sgn
            phi[idx[tuple(e)]] -= K
            phi[idx[(0, 0, 0)]] += K
    return R, phi


def test_monatomic_axis_springs_closed_form():
    k_long, alpha, M = 1.3, 0.25, 2.2
    R, phi = _axis_spring_phi(k_long, alpha)
    rng = np.random.default_rng(3)
    q = rng.uniform(-0.5, 0.5, size=(30, 3))
    w, z, lam = bands.phonon_modes(q, R, phi, np.array([M]))
    c = 1.0 - np.cos(2 * np.pi * q)                     # [nq, 3]
    ref = np.empty((q.shape[0], 3))
    for a in range(3):
        others = [b for b in range(3) if b != a]
        ref[:, a] = (2 * k_long * c[:, a] + 2 * alpha * k_long * c[:, others].sum(axis=1)) / M
    ref.sort(axis=1)
    assert np.max(np.abs(lam - ref)) < 1e-13 * np.max(ref)
    # scipy may carry a newer CODATA amu (relative change ~1e-9)
    assert np.max(np.abs(w / (C_OMEGA_SCIPY * np.sqrt(ref)) - 1.0)) < 1e-8


def test_diatomic_chain_closed_form():
    # atoms at 0 and 1/2 along x, longitudinal springs C to both neighbours
    C, M1, M2 = 0.9, 1.4, 2.7
    R = synth.box_vectors(1)
    idx = {tuple(r): i for i, r in enumerate(R)}
    phi = np.zeros((R.shape[0], 6, 6))
    K = np.zeros((3, 3))
    K[0, 0] = C
    for Rb in [(0, 0, 0), (-1, 0, 0)]:              # atom 0 bonded to atom 1 in cells 0 and -x
        mR = tuple(-x for x in Rb)
        phi[idx[Rb], 0:3, 3:6] -= K
        phi[idx[mR], 3:6, 0:3] -= K
        phi[idx[(0, 0, 0)], 0:3, 0:3] += K
        phi[idx[(0, 0, 0)], 3:6, 3:6] += K
    qx = np.linspace(-0.5, 0.5, 17)
    q = np.stack([qx, 0.3 * np.ones_like(qx), -0.2 * np.ones_like(qx)], axis=1)
    w, z, lam = bands.phonon_modes(q, R, phi, np.array([M1, M2]))
    s = 1.0 / M1 + 1.0 / M2
    root = np.sqrt(s * s - 4.0 * np.sin(np.pi * qx) ** 2 / (M1 * M2))
    hi = C * (s + root)
    lo = C * (s - root)
    # four transverse zero modes + the acoustic and optical longitudinal branches
    assert np.max(np.abs(lam[:, 0:4])) < 1e-13
    assert np.max(np.abs(lam[:, 4] - lo)) < 1e-13
    assert np.max(np.abs(lam[:, 5] - hi)) < 1e-13


def test_single_wannier_function_band_is_fourier_sum():
    rng = np.random.default_rng(8)
    R = synth.box_vectors(1)
    idx = {tuple(r): i for i, r in enumerate(R)}
    h = np.zeros((R.shape[0], 1, 1), dtype=np.complex128)
    for i, r in enumerate(R):
        j = idx[tuple(-x for x in r)]
        if i < j:
            v = rng.standard_normal() + 1j * rng.standard_normal()
            h[i, 0, 0], h[j, 0, 0] = v, np.conj(v)
        elif i == j:
            h[i, 0, 0] = rng.standard_normal()
    k = rng.uniform(-1, 1, size=(10, 3))
    eps, U = bands.electron_bands(k, R, h)
    ref = np.zeros(10)
    for i, r in enumerate(R):
        ref += (h[i, 0, 0] * np.exp(2j * np.pi * (k @ r))).real
    assert np.max(np.abs(eps[:, 0] - ref)) < 1e-13


def test_occupations_closed_values():
    kT = 0.025
    assert abs(bands.fermi_dirac(np.array([0.3]), 0.3, kT)[0] - 0.5) < 1e-15
    x = np.array([-2.0, -0.1, 0.0, 0.05, 1.5])
    f = bands.fermi_dirac(x, 0.0, kT)
    assert np.allclose(f + bands.fermi_dirac(-x, 0.0, kT), 1.0, atol=1e-15)
    assert abs(f[3] - 1.0 / (math.exp(2.0) + 1.0)) < 1e-15
    n = bands.bose_einstein(np.array([0.05]), kT)[0]
    assert abs(n - 1.0 / (math.exp(2.0) - 1.0)) < 1e-14
