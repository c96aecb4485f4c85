"""Electron and phonon band structure by Fourier interpolation (FP64, LAPACK).

* Electrons (Electron Properties): the Wannier-gauge Hamiltonian at any k is
  the back Fourier transform H^W(k) = sum_R e^{i k.R} <0n|H|Rm>, and its
  diagonalisation U_k^dagger H^W(k) U_k = diag(eps_k) gives the band energies
  and the rotation U_k (columns are eigenvectors).
* Phonons (Phonon Properties, dynamical matrix and its eigenvalue equation):
  D(q) = sum_R V2(0|R) e^{i q.R}, D z = (hbar omega)^2 z.

Readings taken where the paper is silent or garbled:
* phases are e^{+i 2 pi k.R} with k, R in crystal coordinates (the paper's
  k.R with a = 1);
* the printed D has no mass weighting although its eigenvalue is (hbar
  omega)^2; the standard mass-weighted form D_{s a, s' b} = sum_R Phi(R)
  e^{i 2 pi q.R} / sqrt(M_s M_s') is used, z is orthonormal, and hbar omega =
  C_OMEGA sqrt(max(lambda, 0));
* eigenvalues ascending, ties in LAPACK's order.
"""

import numpy as np

from .constants import C_OMEGA


def fourier_sum(points, rvecs, mats):
    """sum_R exp(+i 2 pi p.R) M[R] for every point p.

    points [np, 3] crystal coords, rvecs [nR, 3] ints, mats [nR, ...] -> [np, ...].
    """
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    phase = np.exp(2j * np.pi * (points @ np.asarray(rvecs, dtype=np.float64).T))
    flat = np.asarray(mats).reshape(mats.shape[0], -1)
    return (phase @ flat).reshape((points.shape[0],) + mats.shape[1:])


def hamiltonian_k(k, rh, h_r):
    """H^W(k) = sum_R e^{i 2 pi k.R} H(R)   ([nk, nW, nW] complex128)."""
    return fourier_sum(k, rh, h_r)


def electron_bands(k, rh, h_r):
    """(eps [nk, nW] ascending, U [nk, nW, nW] with eigenvectors as columns)."""
    H = hamiltonian_k(k, rh, h_r)
    eps, U = np.linalg.eigh(H)
    return eps, U


def dynamical_matrix(q, rd, phi_r, mass):
    """Mass-weighted D(q) = sum_R Phi(R) e^{i 2 pi q.R} / sqrt(M_s M_s')."""
    D = fourier_sum(q, rd, phi_r.astype(np.complex128))
    m3 = np.repeat(np.asarray(mass, dtype=np.float64), 3)
    w = 1.0 / np.sqrt(np.outer(m3, m3))
    return D * w[None, :, :]


def phonon_modes(q, rd, phi_r, mass):
    """(hbar omega [nq, 3nat] ascending in lambda, z [nq, 3nat, 3nat] columns, lambda)."""
    D = dynamical_matrix(q, rd, phi_r, mass)
    lam, z = np.linalg.eigh(D)
    omega = C_OMEGA * np.sqrt(np.maximum(lam, 0.0))
    return omega, z, lam


def fermi_dirac(eps, mu, kT):
    """Equilibrium electron occupation 1/(exp((eps - mu)/kT) + 1)."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    ex = np.exp(-x[pos])
    out[pos] = ex / (1.0 + ex)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def bose_einstein(omega, kT):
    """Equilibrium phonon occupation 1/(exp(hbar omega/kT) - 1) (omega > 0 only)."""
    return 1.0 / np.expm1(np.asarray(omega, dtype=np.float64) / kT)
