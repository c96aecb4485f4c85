"""Phonon scattering rate from the electron-phonon interaction, P^{el-ph}_{q nu} (FP64).

Follows Transport Methods, phonon BTE: the el-ph term on the diagonal of the
rescaled phonon scattering matrix A,

  P_{q nu} = -(2 pi / (N_k hbar)) n_{q nu} (n_{q nu} + 1)
             sum_{k b b'} |g_{b b' nu}(k, q)|^2 (f_{k b} - f_{k+q, b'})
             delta(eps_{k b} - eps_{k+q, b'} - hbar omega_{q nu}),

with the paper's replacement f_{k b} - f_{k+q, b'} ~ (df/d eps)_{k b} hbar omega_{q nu}.
Since -df/d eps = f (1 - f) / kT this is

  P_{q nu} = (2 pi / N_k) n (n + 1) hbar omega_{q nu}
             sum_{k, b, b'} |g_{b b' nu}(k, q)|^2 f_{k b} (1 - f_{k b}) / kT
             delta(eps_{k b} - eps_{k+q, b'} - hbar omega_{q nu}).

Readings taken (besides those of ``oracle.rates`` and ``oracle.coupling``):
* hbar = 1: P is an energy in eV, like Gamma;
* the sum over k runs over every point of the k mesh, N_k its size; b runs over
  the states inside the energy window (the electronic states the calculation
  keeps), b' over all bands, as m does in the electron lifetime;
* g_{b b' nu}(k, q) has b at k and b' at k + q, the index order of the
  electron lifetime's coupling;
* modes with hbar omega < omega_min are left out (P = 0 there);
* delta is the Gaussian of the Dirac delta and Smearing section with the given
  sigma.
"""

import numpy as np

from .bands import bose_einstein, fermi_dirac
from .coupling import coupling_k_rp, phonon_length, polar_params
from .mesh import mesh_triples, sum_index_table
from .polar import polar_factor
from .rates import gaussian_delta, kept_points, mesh_tables, transition_sigma, window_mask
from .velocity import group_velocities


def phonon_linewidth(system, mesh, mu, kT, sigma, win_lo, win_hi, omega_min=1e-4, tables=None,
                     q_chunk=4096, k_batch=8, adaptive=None):
    """P^{el-ph}_{q nu} at every q of the mesh (the k and the q mesh are the same mesh).

    adaptive: as in ``oracle.rates.scattering_rates`` (a smearing width per transition).

    Returns dict(P [N_q, nModes] eV, k_idx (the kept k summed over), tables).
    """
    if tables is None:
        tables = mesh_tables(system, mesh)
    eps, U, omega, z = tables["eps"], tables["U"], tables["omega"], tables["z"]
    pts = tables["points"]
    N = pts.shape[0]
    nm = system.n_modes
    mask_all = window_mask(eps, win_lo, win_hi)
    k_idx = kept_points(mask_all)
    f_all = fermi_dirac(eps, mu, kT)
    mdf = f_all * (1.0 - f_all) / kT                                  # -df/d eps
    active = omega >= omega_min
    l_all = phonon_length(omega, system.mass, omega_min)
    zl_all = z * np.repeat(l_all, 3, axis=1)                          # [N, sa, nu]
    rp = np.asarray(system.rp, dtype=np.float64)
    # polar systems: g = g^S + i L(q, nu) [U_k^dagger U_{k+q}]_{n m} (oracle.polar)
    pp = polar_params(system)
    L_all = polar_factor(pts, z, l_all, *pp) if pp is not None else None   # [N, nu]
    v_all = group_velocities(pts, system.rh, system.h_r)[1] if adaptive is not None else None

    # S[q, nu] = sum over kept (k, b) and all b' of |g|^2 (-f'_{k b}) delta(...)
    S = np.zeros((N, nm))
    for b0 in range(0, k_idx.size, k_batch):
        kb = k_idx[b0:b0 + k_batch]
        f1 = coupling_k_rp(pts[kb], system.re, system.g_rr)          # [b, Rp, sa, a, b]
        for t, ik in enumerate(kb):
            nlist = np.nonzero(mask_all[ik])[0]
            Uh = np.conj(U[ik][:, nlist]).T                             # [n, a]
            ft = np.einsum("na,rsab->rsnb", Uh, f1[t])
            ftf = ft.reshape(ft.shape[0], -1)
            kq_all = sum_index_table([ik], mesh)[0]
            for c0 in range(0, N, q_chunk):
                qs = np.arange(c0, min(N, c0 + q_chunk))
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
                    x = eps[ik, n] - eps[kq][:, None, :] - omega[qs][:, :, None]   # [q, nu, m]
                    sig = transition_sigma(sigma, adaptive, v_all, ik, n, kq, mesh)
                    S[qs] += mdf[ik, n] * np.sum(g2[:, j] * gaussian_delta(x, sig), axis=-1)
    nb = np.where(active, bose_einstein(np.where(active, omega, 1.0), kT), 0.0)
    P = np.where(active, (2.0 * np.pi / N) * nb * (nb + 1.0) * omega * S, 0.0)
    return dict(P=P, k_idx=k_idx, tables=tables)


def phonon_linewidth_at(system, mesh, q_idx, mu, kT, sigma, win_lo, win_hi, omega_min=1e-4,
                        tables=None, k_chunk=512):
    """P^{el-ph}_{q nu} at the given mesh points q only, same definition as
    ``phonon_linewidth`` (fixed Gaussian width).

    The double lattice sum is taken in the other order: at each q the sum over Rp
    first, g_q(Re) = sum_Rp e^{i 2 pi q.Rp} g(Re, Rp), then the sum over Re at
    every kept k.  Each q costs one pass over g(Re, Rp) and one product with the
    kept-k phases, so a few q of a large mesh are cheap.  Returns P [len(q_idx), nModes].
    """
    if tables is None:
        tables = mesh_tables(system, mesh)
    eps, U, omega, z = tables["eps"], tables["U"], tables["omega"], tables["z"]
    pts = tables["points"]
    N = pts.shape[0]
    nm, nW = system.n_modes, system.n_wannier
    mask_all = window_mask(eps, win_lo, win_hi)
    k_idx = kept_points(mask_all)
    f_all = fermi_dirac(eps, mu, kT)
    mdf = f_all * (1.0 - f_all) / kT
    re = np.asarray(system.re, dtype=np.float64)
    rp = np.asarray(system.rp, dtype=np.float64)
    g_flat = system.g_rr.reshape(re.shape[0], rp.shape[0], -1)       # [Re, Rp, sa a b]
    pp = polar_params(system)
    q_idx = np.asarray(q_idx, dtype=np.int64)
    P = np.zeros((q_idx.size, nm))
    for iq, q in enumerate(q_idx):
        w = omega[q]
        active = w >= omega_min
        l = phonon_length(omega[q:q + 1], system.mass, omega_min)[0]   # [nat, nu]
        zl = z[q] * np.repeat(l, 3, axis=0)                             # [sa, nu]
        L = polar_factor(pts[q:q + 1], z[q:q + 1], l[None], *pp)[0] if pp is not None else None
        ph_q = np.exp(2j * np.pi * (rp @ pts[q]))                       # [Rp]
        gq = np.einsum("p,epc->ec", ph_q, g_flat)                       # [Re, sa a b]
        tri = mesh_triples(mesh)
        nn = np.asarray(mesh, dtype=np.int64)
        s3 = (tri[k_idx] + tri[q][None, :]) % nn[None, :]
        kq_all = (s3[:, 0] * nn[1] + s3[:, 1]) * nn[2] + s3[:, 2]      # k + q of every kept k
        S = np.zeros(nm)
        for c0 in range(0, k_idx.size, k_chunk):
            ks = k_idx[c0:c0 + k_chunk]
            kq = kq_all[c0:c0 + k_chunk]
            ph_k = np.exp(2j * np.pi * (pts[ks] @ re.T))                # [k, Re]
            G = (ph_k @ gq).reshape(ks.size, nm, nW, nW)                # [k, sa, a, b]
            Y = np.conj(np.swapaxes(U[ks], -1, -2))[:, None] @ G @ U[kq][:, None]   # [k, sa, n, m]
            g = np.einsum("ksnm,sv->knvm", Y, zl)                       # [k, n, nu, m]
            if L is not None:
                O = np.conj(np.swapaxes(U[ks], -1, -2)) @ U[kq]         # [k, n, m]
                g = g + 1j * L[None, None, :, None] * O[:, :, None, :]
            g2 = (g * np.conj(g)).real
            x = eps[ks][:, :, None, None] - eps[kq][:, None, None, :] - w[None, None, :, None]
            wgt = mdf[ks] * mask_all[ks]                                # kept states only
            S += np.einsum("kn,knvm->v", wgt, g2 * gaussian_delta(x, sigma))
        nb = np.where(active, bose_einstein(np.where(active, w, 1.0), kT), 0.0)
        P[iq] = np.where(active, (2.0 * np.pi / N) * nb * (nb + 1.0) * w * S, 0.0)
    return P
