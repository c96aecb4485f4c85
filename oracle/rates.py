"""Electron-phonon scattering rates Gamma_nk = hbar/tau_nk (FP64).

Follows Transport Methods, electron BTE (the lifetime 1/tau_kb as a sum over
k', b', q, nu of |g|^2 times occupation factors and energy-conserving deltas),
the Dirac delta and Smearing section (Gaussian smearing), the Band structure
classes section (energy window, ragged kept states) and the Points class
(mesh ordering, k + q on the mesh).

With momentum conservation k' = k + q on a uniform mesh the rate of state
(k, n) reads

  Gamma_nk = 2 pi sum_q w_q sum_m sum_nu |g_{n m nu}(k, q)|^2
             [ (n_{q nu} + 1 - f_{m,k+q}) delta(eps_nk - eps_{m,k+q} - hbar omega_{q nu})
             + (n_{q nu} + f_{m,k+q})     delta(eps_nk - eps_{m,k+q} + hbar omega_{q nu}) ]

with w_q = 1/N_q on the full q mesh (or caller weights for explicit q lists),
delta(x) = exp(-x^2/sigma^2)/(sqrt(pi) sigma), f Fermi-Dirac at (mu, kT), n
Bose-Einstein at kT.

Readings taken:
* the prefactor 2 pi/(N_k V) becomes 2 pi/N_q with hbar = 1 (Gamma in eV);
  V = 1 A^3 for the unit cube and N_k = N_q on one mesh;
* f in the rate is the equilibrium Fermi-Dirac occupation of the final state;
* sigma is used literally (the Gaussian's standard deviation is sigma/sqrt 2);
* modes with hbar omega < omega_min are left out of the sum;
* energy window: state (k, n) is kept iff win_lo < eps_nk < win_hi; a k point
  is kept iff it has a kept state; n runs over kept states only, m over all
  bands;
* the coupling is the fixed-k precomputation of the Kokkos section with the
  k-side rotation folded in, f~(k, Rp) = sum_Re e^{i 2 pi k.Re} U_k^dagger
  g(Re, Rp), then the sum over Rp at each q and the k+q-side and phonon
  rotations (see ``oracle.coupling`` for the conventions).
"""

import numpy as np

from .bands import (bose_einstein, electron_bands, fermi_dirac,
                    phonon_modes)
from .coupling import coupling_k_rp, phonon_length, polar_params
from .mesh import mesh_points, sum_index_table
from .polar import polar_factor
from .velocity import adaptive_sigma, group_velocities


def gaussian_delta(x, sigma):
    """delta(x) ~ exp(-x^2/sigma^2) / (sqrt(pi) sigma)   (Gaussian smearing)."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-(x * x) / (sigma * sigma)) / (np.sqrt(np.pi) * sigma)


def window_mask(eps, win_lo, win_hi):
    """1 where win_lo < eps < win_hi (energy-cutoff window), as uint8."""
    eps = np.asarray(eps)
    return ((eps > win_lo) & (eps < win_hi)).astype(np.uint8)


def kept_points(mask):
    """Indices (ascending) of points with at least one state in the window."""
    return np.nonzero(np.asarray(mask).any(axis=1))[0].astype(np.int64)


def mesh_tables(system, mesh):
    """Band energies/rotations and phonon modes at every point of a uniform mesh."""
    pts = mesh_points(mesh)
    eps, U = electron_bands(pts, system.rh, system.h_r)
    omega, z, lam = phonon_modes(pts, system.rd, system.phi_r, system.mass)
    return dict(points=pts, eps=eps, U=U, omega=omega, z=z, lam=lam)


def rate_terms(g2, eps_n, eps_m, f_m, omega, n_b, sigma, active):
    """sum over (m, nu) of |g|^2 times the emission and absorption factors.

    g2 [..., nu, m]; eps_n scalar; eps_m, f_m [..., m]; omega, n_b, active
    [..., nu].  Returns [...].
    """
    x = eps_n - eps_m[..., None, :]                 # [..., 1, m]
    w = omega[..., :, None]                         # [..., nu, 1]
    nb = n_b[..., :, None]
    fm = f_m[..., None, :]
    emis = (nb + 1.0 - fm) * gaussian_delta(x - w, sigma)
    absn = (nb + fm) * gaussian_delta(x + w, sigma)
    term = g2 * (emis + absn) * active[..., :, None]
    return term.sum(axis=(-1, -2))


def transition_sigma(sigma, adaptive, v_all, ik, n, kq, mesh):
    """Smearing width of the transitions (k, n) -> (k+q, m): the fixed sigma, or
    with ``adaptive`` = dict(sigma_min=..., prefactor=...) the adaptive width of
    ``oracle.velocity`` from the group velocities ([q, 1, m], broadcast over nu)."""
    if adaptive is None:
        return sigma
    s = adaptive_sigma(v_all[ik, n][None, None, :], v_all[kq], mesh, adaptive["sigma_min"],
                       adaptive.get("prefactor", 1.0))
    return s[:, None, :]


def scattering_rates(system, mesh, mu, kT, sigma, win_lo, win_hi, omega_min=1e-4,
                     k_idx=None, q_lists=None, tables=None, q_chunk=4096, k_batch=8,
                     adaptive=None):
    """Gamma_nk for kept states of the k mesh (full q mesh or weighted q lists).

    adaptive: None (Gaussian smearing of width sigma) or dict(sigma_min=...,
      prefactor=1.0): adaptive Gaussian smearing (Dirac delta and Smearing), a
      width per transition from the group velocities at k and k+q.

    mesh: (N0, N1, N2), the same mesh for k and q.
    k_idx: mesh linear indices of the k points to evaluate; None = every k with
      a state in the window.
    q_lists: None (all mesh q, weight 1/N_q) or (q_off [nk+1], q_idx, q_w) with
      q_idx mesh linear indices and q_w the weights of each listed q.
    Returns dict(gamma [nk, nW] (0 outside the window), band_mask [nk, nW],
      k_idx [nk], tables).
    """
    if tables is None:
        tables = mesh_tables(system, mesh)
    eps, U, omega, z = tables["eps"], tables["U"], tables["omega"], tables["z"]
    pts = tables["points"]
    nq_mesh = pts.shape[0]
    mask_all = window_mask(eps, win_lo, win_hi)
    if k_idx is None:
        k_idx = kept_points(mask_all)
    k_idx = np.asarray(k_idx, dtype=np.int64)
    nk, nW = k_idx.shape[0], system.n_wannier
    nm = system.n_modes
    f_all = fermi_dirac(eps, mu, kT)
    active_all = omega >= omega_min
    nb_all = np.where(active_all, bose_einstein(np.where(active_all, omega, 1.0), kT), 0.0)
    l_all = phonon_length(omega, system.mass, omega_min)              # [N, nat, nu]
    zl_all = z * np.repeat(l_all, 3, axis=1)                          # [N, sa, nu]
    rp = np.asarray(system.rp, dtype=np.float64)
    # polar systems: g = g^S + i L(q, nu) [U_k^dagger U_{k+q}]_{n m} (oracle.polar)
    pp = polar_params(system)
    L_all = polar_factor(pts, z, l_all, *pp) if pp is not None else None   # [N, nu]
    v_all = group_velocities(pts, system.rh, system.h_r)[1] if adaptive is not None else None

    gamma = np.zeros((nk, nW))
    band_mask = mask_all[k_idx]
    for b0 in range(0, nk, k_batch):
        kb = k_idx[b0:b0 + k_batch]
        f1 = coupling_k_rp(pts[kb], system.re, system.g_rr)          # [b, Rp, sa, a, b]
        for t, ik in enumerate(kb):
            a_row = b0 + t
            nlist = np.nonzero(band_mask[a_row])[0]
            if nlist.size == 0:
                continue
            Uh = np.conj(U[ik][:, nlist]).T                             # [n, a]
            ft = np.einsum("na,rsab->rsnb", Uh, f1[t])                 # f~(k, Rp)
            ftf = ft.reshape(ft.shape[0], -1)
            if q_lists is None:
                qsel = np.arange(nq_mesh)
                wq = np.full(nq_mesh, 1.0 / nq_mesh)
            else:
                q_off, q_idx, q_w = q_lists
                qsel = np.asarray(q_idx[q_off[a_row]:q_off[a_row + 1]], dtype=np.int64)
                wq = np.asarray(q_w[q_off[a_row]:q_off[a_row + 1]], dtype=np.float64)
            kq_all = sum_index_table([ik], mesh)[0]
            acc = np.zeros(nlist.size)
            for c0 in range(0, qsel.size, q_chunk):
                qs = qsel[c0:c0 + q_chunk]
                ph = np.exp(2j * np.pi * (pts[qs] @ rp.T))             # [q, Rp]
                X = (ph @ ftf).reshape((qs.size,) + ft.shape[1:])      # [q, sa, n, b]
                kq = kq_all[qs]
                Y = X @ U[kq][:, None, :, :]                            # [q, sa, n, m]
                g = np.einsum("qsnm,qsv->qnvm", Y, zl_all[qs])          # [q, n, nu, m]
                if L_all is not None:
                    O = Uh[None] @ U[kq]                                # [q, n, m]
                    g = g + 1j * L_all[qs][:, None, :, None] * O[:, :, None, :]
                g2 = (g * np.conj(g)).real
                for j, n in enumerate(nlist):
                    sig = transition_sigma(sigma, adaptive, v_all, ik, n, kq, mesh)
                    terms = rate_terms(g2[:, j], eps[ik, n], eps[kq], f_all[kq],
                                       omega[qs], nb_all[qs], sig, active_all[qs])
                    acc[j] += np.sum(wq[c0:c0 + q_chunk] * terms)
            gamma[a_row, nlist] = 2.0 * np.pi * acc
    return dict(gamma=gamma, band_mask=band_mask, k_idx=k_idx, tables=tables)
