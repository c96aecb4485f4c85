"""Electron velocities and adaptive Gaussian smearing (FP64).

Follows Electron Properties, Velocity (the velocity operator as the k-derivative
of the Wannier-interpolated Hamiltonian rotated to the Bloch basis, with the
degenerate subspaces diagonalised) and the Dirac delta and Smearing section
(adaptive Gaussian smearing).

* v_{alpha k, b b'} = [U_k^dagger (d H^W_k / d k_alpha) U_k]_{b b'}; with the
  Cartesian wavevector 2 pi k / a (a = 1 A) and Cartesian R,
  d H^W_k / d k_alpha = sum_R i R_alpha e^{i 2 pi k.R} H(R)   (eV A);
* the group velocity of a non-degenerate band is the diagonal element; for a
  degenerate group the block of v_alpha on the group is diagonalised and its
  eigenvalues (ascending) are the velocities of the group's bands in order,
  separately for each alpha;
* adaptive smearing of a transition between (k, b) and (k', b'):
  sigma = (A / sqrt 12) sqrt( sum_beta ( sum_alpha (v_alpha(k b) - v_alpha(k' b'))
                                         C_{alpha beta} / N_beta )^2 ).

Readings taken where the paper is silent or garbled:
* the derivative is taken analytically (the paper's central difference is the
  approximation of the same derivative; it serves as a pin);
* the printed adaptive sigma has no square inside the sum over beta; the sum
  of squares (the norm of the velocity difference projected on the mesh
  steps) is the reading, and A = 1;
* C_{alpha beta}: for sigma to be an energy the velocity difference (eV A) is
  projected on the reciprocal-lattice vectors b_beta (1/A) divided by the mesh
  size, i.e. C_{alpha beta} = (b_beta)_alpha = 2 pi / a delta_{alpha beta} for
  the simple-cubic cell; sigma is then the standard deviation of the energy
  difference over one mesh cell of displacements (uniform distribution);
* sigma is floored at a given sigma_min, so that transitions with equal
  velocities keep a finite delta;
* degenerate groups: |eps_b - eps_b'| < 1e-6 eV.
"""

import numpy as np

from .bands import electron_bands  # noqa: F401 (re-exported for the pins)


def hamiltonian_derivative(k, rh, h_r):
    """d H^W / d k_alpha = sum_R i R_alpha e^{i 2 pi k.R} H(R)   ([nk, 3, nW, nW], eV A)."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    R = np.asarray(rh, dtype=np.float64)
    phase = np.exp(2j * np.pi * (k @ R.T))                          # [nk, nR]
    flat = np.asarray(h_r).reshape(R.shape[0], -1)
    out = np.empty((k.shape[0], 3) + h_r.shape[1:], dtype=np.complex128)
    for a in range(3):
        out[:, a] = ((phase * (1j * R[:, a])[None, :]) @ flat).reshape((k.shape[0],) + h_r.shape[1:])
    return out


def velocity_matrix(k, rh, h_r):
    """(eps [nk, nW], U [nk, nW, nW], V [nk, 3, nW, nW]) with V_alpha = U^dagger dH/dk_alpha U."""
    eps, U = electron_bands(k, rh, h_r)
    dH = hamiltonian_derivative(k, rh, h_r)
    Uh = np.conj(np.swapaxes(U, -1, -2))
    V = Uh[:, None] @ dH @ U[:, None]
    return eps, U, V


def group_velocities(k, rh, h_r, deg_tol=1e-6):
    """(eps [nk, nW], v [nk, nW, 3]) with degenerate subspaces diagonalised per direction."""
    eps, U, V = velocity_matrix(k, rh, h_r)
    nk, nW = eps.shape
    v = np.empty((nk, nW, 3))
    for i in range(nk):
        b = 0
        while b < nW:
            e = b + 1
            while e < nW and abs(eps[i, e] - eps[i, e - 1]) < deg_tol:
                e += 1
            for a in range(3):
                blk = V[i, a, b:e, b:e]
                if e - b == 1:
                    v[i, b, a] = blk[0, 0].real
                else:
                    v[i, b:e, a] = np.linalg.eigvalsh(blk)
            b = e
    return eps, v


def adaptive_sigma(v_from, v_to, mesh, sigma_min, prefactor=1.0):
    """sigma of transitions with velocities v_from -> v_to ([..., 3] eV A each), floored at sigma_min."""
    dv = np.asarray(v_from, dtype=np.float64) - np.asarray(v_to, dtype=np.float64)
    steps = 2.0 * np.pi / np.asarray(mesh, dtype=np.float64)           # |b_beta| / N_beta
    s = prefactor / np.sqrt(12.0) * np.sqrt(np.sum((dv * steps) ** 2, axis=-1))
    return np.maximum(s, sigma_min)
