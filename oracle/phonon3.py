"""Interpolation of the three-phonon coupling V^(3)(q nu, q' nu', q'' nu'') (FP64).

Follows Phonon Properties (the Fourier transform of the third derivative of
the energy that gives the 3-phonon coupling) and the Kokkos (Interaction)
section (the generic coupling contraction, computed with the sum over the
first lattice vector precomputed at fixed q, then the sum over the second at
each q').

  V3(q nu, q' nu', q'' nu'') =
      sum_{R, R'} sum_{s a, s' b, s'' c} Phi3(s a R, s' b R', s'' c 0)
          e^{-i 2 pi (q.R + q'.R')}
          z*_{s a, nu}(q) l_{s, q nu}  z*_{s' b, nu'}(q') l_{s', q' nu'}
          z*_{s'' c, nu''}(q'') l_{s'', q'' nu''},

with q'' = -q - q' (momentum conservation up to a reciprocal-lattice vector)
and l_{s, q nu} = sqrt(C_PH / (2 M_s hbar omega_{q nu})) the phonon length of
the el-ph coupling, so that V3 is in eV for Phi3 in eV/A^3.

Readings taken where the paper is garbled or silent:
* the printed prefactor (2/hbar)^{3/2} sqrt(m m' m'' / (omega omega' omega''))
  is dimensionally inconsistent; it is read as the usual product of the three
  zero-point lengths, (hbar/2)^{3/2} / sqrt(m m' m'' omega omega' omega''),
  i.e. the product of the three l factors above;
* the prefactor 1/N0^3 is taken as 1 (the synthetic Phi3 carries its own
  scale), every lattice vector with weight 1;
* the third displacement sits in the reference cell, as printed, and the
  third wavevector is fixed by the other two: q'' = -q - q';
* modes with hbar omega < omega_min get l = 0.
"""

import numpy as np

from .bands import fourier_sum, phonon_modes
from .coupling import phonon_length


def _phase_sum(points, rvecs, mats):
    """sum_R e^{-i 2 pi p.R} M[R] for every point p."""
    return fourier_sum(-np.asarray(points, dtype=np.float64).reshape(-1, 3), rvecs, mats)


def v3_fixed_q(q, r1, phi3, zl_q):
    """The precomputation at fixed q (Kokkos section):
    T[i, R', nu, s'b, s''c] = sum_{R, sa} e^{-i 2 pi q_i.R} Phi3[R, R', sa, s'b, s''c] z*l[sa, nu]."""
    S = _phase_sum(q, r1, phi3.astype(np.complex128))        # [nq, nR', sa, s'b, s''c]
    return np.einsum("irabc,iav->irvbc", S, np.conj(zl_q))


def interp_v3(q, qp, system3, omega_min=1e-4):
    """V3 for every pair of a q list and a q' list (q'' = -q - q').

    system3: an object with rd, phi_r, mass (harmonic part), r1, r2 (int [n, 3]
    lattice vectors of the first and second displacement) and phi3
    [n_r1, n_r2, 3nat, 3nat, 3nat] (eV/A^3).
    Returns dict(v3 [nq, nqp, nModes, nModes, nModes] (nu, nu', nu''),
    omega_q, omega_qp [nq, nqp... see keys], omega_qpp [nq, nqp, nModes]).
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    qp = np.asarray(qp, dtype=np.float64).reshape(-1, 3)
    nq, nqp = q.shape[0], qp.shape[0]
    s = system3
    w1, z1, _ = phonon_modes(q, s.rd, s.phi_r, s.mass)
    w2, z2, _ = phonon_modes(qp, s.rd, s.phi_r, s.mass)
    qpp = -(q[:, None, :] + qp[None, :, :]).reshape(-1, 3)
    w3, z3, _ = phonon_modes(qpp, s.rd, s.phi_r, s.mass)
    nm = z1.shape[-1]
    zl1 = z1 * np.repeat(phonon_length(w1, s.mass, omega_min), 3, axis=1)
    zl2 = z2 * np.repeat(phonon_length(w2, s.mass, omega_min), 3, axis=1)
    zl3 = (z3 * np.repeat(phonon_length(w3, s.mass, omega_min), 3, axis=1)).reshape(nq, nqp, nm, nm)
    T = v3_fixed_q(q, s.r1, s.phi3, zl1)                      # [nq, nR', nu, s'b, s''c]
    out = np.empty((nq, nqp, nm, nm, nm), dtype=np.complex128)
    for i in range(nq):
        X = _phase_sum(qp, s.r2, T[i])                          # [nqp, nu, s'b, s''c]
        out[i] = np.einsum("jvbc,jbw,jcx->jvwx", X, np.conj(zl2), np.conj(zl3[i]))
    return dict(v3=out, omega_q=w1, omega_qp=w2, omega_qpp=w3.reshape(nq, nqp, nm))


def interp_v3_brute(q, qp, system3, omega_min=1e-4):
    """The same double sum with explicit loops over (R, R') and the direct rotations (tiny inputs)."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    qp = np.asarray(qp, dtype=np.float64).reshape(-1, 3)
    s = system3
    nm = 3 * s.mass.shape[0]
    out = np.zeros((q.shape[0], qp.shape[0], nm, nm, nm), dtype=np.complex128)
    for i in range(q.shape[0]):
        for j in range(qp.shape[0]):
            pts = np.stack([q[i], qp[j], -q[i] - qp[j]])
            w, z, _ = phonon_modes(pts, s.rd, s.phi_r, s.mass)
            zl = z * np.repeat(phonon_length(w, s.mass, omega_min), 3, axis=1)
            F = np.zeros((nm, nm, nm), dtype=np.complex128)
            for a, R in enumerate(s.r1):
                for b, Rp in enumerate(s.r2):
                    ph = np.exp(-2j * np.pi * (q[i] @ R + qp[j] @ Rp))
                    F += ph * s.phi3[a, b]
            for v1 in range(nm):
                for v2 in range(nm):
                    for v3 in range(nm):
                        out[i, j, v1, v2, v3] = np.einsum(
                            "abc,a,b,c->", F, np.conj(zl[0][:, v1]), np.conj(zl[1][:, v2]),
                            np.conj(zl[2][:, v3]))
    return out
