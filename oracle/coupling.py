"""Wannier-to-Bloch interpolation of the electron-phonon coupling (FP64).

Follows Electron Properties (definition of g with the (1/2 m omega)^{1/2}
factor; interpolation of g^0 from g^0(Re, Rp)) and the Kokkos (Interaction)
section (the generic coupling contraction and its precomputation at fixed k).

Readings taken:
* the printed interpolation writes U_{k+q} g U_k^dagger z while the coarse
  transform writes U_{k+q}^dagger g U_k and the generic contraction has no
  conjugates; with U_k holding eigenvectors as columns the form used is
      g_{n m nu}(k, q) = sum_{s alpha} [U_k^dagger G_{s alpha}(k, q) U_{k+q}]_{n m}
                                         z_{s alpha, nu}(q) l_{s, q nu},
  n a band at k and m a band at k+q, where
      G_{s alpha}(k, q) = sum_{Re, Rp} e^{i 2 pi (k.Re + q.Rp)} g(Re, Rp)_{s alpha}
  and the first Wannier index of g(Re, Rp) pairs with k;
* the prefactor 1/N_e is taken as 1 (the synthetic g(Re, Rp) carries its own
  scale) and every lattice vector has weight 1;
* the single mass m of the definition is the mass M_s of the displaced atom,
  inside the s sum: l_{s, q nu} = sqrt(C_PH / (2 M_s hbar omega_{q nu})) in A;
* modes with hbar omega < omega_min (acoustic modes at q = 0, where the factor
  diverges) get l = 0.
"""

import numpy as np

from .bands import electron_bands, fourier_sum, phonon_modes
from .constants import C_PH


def coupling_k_rp(k, re, g_rr):
    """First phase sum at fixed k: sum_Re e^{i 2 pi k.Re} g(Re, Rp).

    This is the quantity the paper precomputes at fixed k before the inner
    loop over k' (Kokkos section).  [nk, n_rp, 3nat, nW, nW].
    """
    return fourier_sum(k, re, g_rr)


def coupling_wannier_gauge(k, q, re, rp, g_rr):
    """G(k, q) = sum_{Re, Rp} e^{i 2 pi (k.Re + q.Rp)} g(Re, Rp)  ([nk, nq, 3nat, nW, nW]).

    Evaluated as the paper's two sums: first over Re at fixed k, then over Rp.
    """
    f = coupling_k_rp(k, re, g_rr)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    out = np.empty((f.shape[0], q.shape[0]) + f.shape[2:], dtype=np.complex128)
    for i in range(f.shape[0]):
        out[i] = fourier_sum(q, rp, f[i])
    return out


def coupling_wannier_gauge_brute(k, q, re, rp, g_rr):
    """The same double sum written as explicit loops over (Re, Rp) (tiny inputs only)."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((k.shape[0], q.shape[0]) + g_rr.shape[2:], dtype=np.complex128)
    for i in range(k.shape[0]):
        for j in range(q.shape[0]):
            acc = np.zeros(g_rr.shape[2:], dtype=np.complex128)
            for a in range(re.shape[0]):
                for b in range(rp.shape[0]):
                    ph = 2.0 * np.pi * (k[i] @ re[a] + q[j] @ rp[b])
                    acc += np.exp(1j * ph) * g_rr[a, b]
            out[i, j] = acc
    return out


def phonon_length(omega, mass, omega_min):
    """l_{s, q nu} = sqrt(C_PH / (2 M_s hbar omega_{q nu})), 0 for omega < omega_min.

    omega [nq, nModes] -> [nq, nat, nModes].
    """
    omega = np.asarray(omega, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    ok = omega >= omega_min
    safe = np.where(ok, omega, 1.0)
    l = np.sqrt(C_PH / (2.0 * mass[None, :, None] * safe[:, None, :]))
    return np.where(ok[:, None, :], l, 0.0)


def rotate_to_bloch(G, U_k, U_kq, z, l):
    """g_{n m nu} = sum_{s alpha} [U_k^dagger G_{s alpha} U_kq]_{n m} z_{s alpha, nu} l_{s, nu}.

    G [..., nModes, nW, nW], U_k [..., nW, nW], U_kq [..., nW, nW],
    z [..., nModes, nModes], l [..., nat, nModes]; leading dims broadcast.
    Returns [..., nModes(nu), nW(n), nW(m)].
    """
    Uh = np.conj(np.swapaxes(U_k, -1, -2))                       # [..., n, a]
    Y = Uh[..., None, :, :] @ G @ U_kq[..., None, :, :]          # [..., sa, n, m]
    lsa = np.repeat(l, 3, axis=-2)                               # [..., sa, nu]
    w = z * lsa                                                  # [..., sa, nu]
    return np.einsum("...snm,...sv->...vnm", Y, w)


def polar_params(system):
    """(born, eps_inf, alpha, g_max) of a polar system, or None (no long-range term)."""
    born = getattr(system, "born", None)
    if born is None:
        return None
    return born, system.eps_inf, system.ewald_alpha, system.g_max


def coupling(k, q, system, omega_min=1e-4):
    """Interpolated el-ph coupling g(k, q) for every pair of the k and q lists.

    For a polar system (one carrying Born charges) g is the sum of the
    interpolated short-range part and the long-range part of ``oracle.polar``.
    Returns dict with g [nk, nq, nModes, nW, nW] (index order nu, n at k, m at
    k+q), eps_k [nk, nW], eps_kq [nk, nq, nW], omega_q [nq, nModes].
    """
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    nk, nq, nW = k.shape[0], q.shape[0], system.n_wannier
    eps_k, U_k = electron_bands(k, system.rh, system.h_r)
    kq = (k[:, None, :] + q[None, :, :]).reshape(-1, 3)
    eps_kq, U_kq = electron_bands(kq, system.rh, system.h_r)
    eps_kq = eps_kq.reshape(nk, nq, nW)
    U_kq = U_kq.reshape(nk, nq, nW, nW)
    omega, z, _ = phonon_modes(q, system.rd, system.phi_r, system.mass)
    l = phonon_length(omega, system.mass, omega_min)
    G = coupling_wannier_gauge(k, q, system.re, system.rp, system.g_rr)
    g = rotate_to_bloch(G, U_k[:, None], U_kq, z[None], l[None])
    pp = polar_params(system)
    if pp is not None:
        from .polar import polar_coupling, polar_factor
        L = polar_factor(q, z, l, *pp)                                # [nq, nu]
        g = g + polar_coupling(U_k[:, None], U_kq, L[None])
    return dict(g=g, eps_k=eps_k, eps_kq=eps_kq, omega_q=omega)
