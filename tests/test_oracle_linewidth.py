"""Pins of the phonon el-ph scattering rate P^{el-ph}_{q nu} (phonon BTE).

* closed form: flat bands, Einstein phonons and a single lattice term make P
  the same at every q and equal to a short explicit sum;
* brute force: every sum written as explicit Python loops on a 2x2x2 mesh;
* P >= 0, and P = 0 for the acoustic modes at q = 0 (below omega_min).
"""

import itertools
import math

import numpy as np
import scipy.constants as sc

import synth
from oracle import linewidth, rates
from test_oracle_rates import _einstein_system

KB = sc.k / sc.electron_volt
C_OMEGA = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt
C_PH = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt


def test_einstein_flat_closed_form_same_at_every_q():
    s, e, kk, M, G0 = _einstein_system()
    T, mu, sigma = 300.0, 0.01, 0.04
    kT = KB * T
    w = C_OMEGA * np.sqrt(kk / M)       # z = identity: the spring constants are ascending
    l2 = C_PH / (2 * M * w)
    lo, hi = -0.07, 0.05                # bands 0 and 1 in the window, band 2 out
    ref = np.zeros(3)
    for v in range(3):
        nb = 1.0 / math.expm1(w[v] / kT)
        acc = 0.0
        for n in range(3):
            if not (lo < e[n] < hi):
                continue
            fn = 1.0 / (math.exp((e[n] - mu) / kT) + 1.0)
            for m in range(3):
                d = math.exp(-((e[n] - e[m] - w[v]) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                acc += abs(G0[v, n, m]) ** 2 * l2[v] * fn * (1 - fn) / kT * d
        ref[v] = 2 * math.pi * nb * (nb + 1) * w[v] * acc
    assert np.all(ref > 0)
    for mesh in [(2, 3, 2), (3, 3, 3)]:
        out = linewidth.phonon_linewidth(s, mesh, mu, kT, sigma, lo, hi)
        assert np.max(np.abs(out["P"] - ref[None, :])) < 1e-8 * np.max(ref)


def _brute_P(s, mesh, mu, kT, sigma, lo, hi, wmin):
    """Every sum as explicit loops; LAPACK only for the small eigenproblems."""
    pts = list(itertools.product(*[range(x) for x in mesh]))
    N = len(pts)

    def frac(t):
        return np.array([t[d] / mesh[d] for d in range(3)])

    def ham(kf):
        H = np.zeros((s.n_wannier, s.n_wannier), dtype=np.complex128)
        for i, R in enumerate(s.rh):
            H += s.h_r[i] * np.exp(2j * math.pi * sum(kf[d] * R[d] for d in range(3)))
        return np.linalg.eigh(H)

    def dyn(qf):
        nm = 3 * s.n_atoms
        D = np.zeros((nm, nm), dtype=np.complex128)
        for i, R in enumerate(s.rd):
            ph = np.exp(2j * math.pi * sum(qf[d] * R[d] for d in range(3)))
            for a in range(nm):
                for b in range(nm):
                    D[a, b] += s.phi_r[i, a, b] * ph / math.sqrt(s.mass[a // 3] * s.mass[b // 3])
        return np.linalg.eigh(D)

    out = np.zeros((N, 3 * s.n_atoms))
    for iq, tq in enumerate(pts):
        qf = frac(tq)
        lam, z = dyn(qf)
        for v in range(3 * s.n_atoms):
            w = C_OMEGA * math.sqrt(max(lam[v], 0.0))
            if w < wmin:
                continue
            nb = 1.0 / math.expm1(w / kT)
            acc = 0.0
            for ik, tk in enumerate(pts):
                kf = frac(tk)
                ek, Uk = ham(kf)
                tkq = tuple((tk[d] + tq[d]) % mesh[d] for d in range(3))
                ekq, Ukq = ham(frac(tkq))
                G = np.zeros(s.g_rr.shape[2:], dtype=np.complex128)
                for a, Re in enumerate(s.re):
                    for b, Rp in enumerate(s.rp):
                        ph = sum(kf[d] * Re[d] + qf[d] * Rp[d] for d in range(3))
                        G += np.exp(2j * math.pi * ph) * s.g_rr[a, b]
                for n in range(s.n_wannier):
                    if not (lo < ek[n] < hi):
                        continue
                    fn = 1.0 / (math.exp((ek[n] - mu) / kT) + 1.0)
                    for m in range(s.n_wannier):
                        gv = 0.0j
                        for sa in range(3 * s.n_atoms):
                            l = math.sqrt(C_PH / (2 * s.mass[sa // 3] * w))
                            for a in range(s.n_wannier):
                                for b in range(s.n_wannier):
                                    gv += np.conj(Uk[a, n]) * G[sa, a, b] * Ukq[b, m] * z[sa, v] * l
                        d = math.exp(-((ek[n] - ekq[m] - w) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                        acc += abs(gv) ** 2 * fn * (1 - fn) / kT * d
            out[iq, v] = 2 * math.pi / N * nb * (nb + 1) * w * acc
    return out


def test_brute_force_tiny_mesh():
    s = synth.small_system(seed=31, n_wannier=2, n_atoms=1, r=1)
    s.h_r = s.h_r * 0.05        # narrow bands: phonon-assisted transitions are resonant
    mesh = (2, 2, 2)
    kT, sigma, wmin = KB * 300.0, 0.05, 1e-4
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    lo, hi = mu - 0.15, mu + 0.15
    out = linewidth.phonon_linewidth(s, mesh, mu, kT, sigma, lo, hi, wmin, tables=t)
    ref = _brute_P(s, mesh, mu, kT, sigma, lo, hi, wmin)
    assert np.max(ref) > 0
    assert np.max(np.abs(out["P"] - ref)) < 1e-8 * np.max(ref)


def test_nonnegative_and_acoustic_modes_at_gamma():
    s = synth.config_c1()
    mesh = (4, 4, 4)
    t = rates.mesh_tables(s, mesh)
    mu = 0.5 * (t["eps"].min() + t["eps"].max())
    kT = KB * 300.0
    out = linewidth.phonon_linewidth(s, mesh, mu, kT, 0.05, mu - 0.5, mu + 0.5, tables=t)
    P = out["P"]
    assert np.all(P >= 0)
    assert np.max(P) > 0
    # q = 0: three acoustic modes below omega_min, left out
    assert np.all(P[0, :3] == 0.0) and np.all(P[0, 3:] > 0)


def test_polar_system_against_explicit_coupling_sum():
    """P of a polar system as an explicit sum over mesh pairs of oracle.coupling's g."""
    from oracle import coupling, mesh as omesh
    s = synth.add_polar(synth.small_system(seed=35, n_wannier=2, n_atoms=2, r=1), seed=35,
                        alpha=3.0, g_max=1, eps_scale=2.0)
    s.h_r = s.h_r * 0.05
    mesh = (3, 2, 2)
    kT, sigma, wmin = KB * 300.0, 0.05, 1e-4
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    lo, hi = mu - 0.2, mu + 0.2
    out = linewidth.phonon_linewidth(s, mesh, mu, kT, sigma, lo, hi, wmin, tables=t)
    pts = omesh.mesh_points(mesh)
    N = pts.shape[0]
    ref = np.zeros((N, s.n_modes))
    for ik in range(N):
        c = coupling.coupling(pts[ik:ik + 1], pts, s, omega_min=wmin)
        ek = c["eps_k"][0]
        for iq in range(N):
            for v in range(s.n_modes):
                w = c["omega_q"][iq, v]
                if w < wmin:
                    continue
                for n in range(s.n_wannier):
                    if not (lo < ek[n] < hi):
                        continue
                    fn = 1.0 / (math.exp((ek[n] - mu) / kT) + 1.0)
                    for m in range(s.n_wannier):
                        d = math.exp(-((ek[n] - c["eps_kq"][0, iq, m] - w) / sigma) ** 2) / (
                            math.sqrt(math.pi) * sigma)
                        ref[iq, v] += abs(c["g"][0, iq, v, n, m]) ** 2 * fn * (1 - fn) / kT * d
    om = t["omega"]
    nb = np.where(om >= wmin, 1.0 / np.expm1(np.maximum(om, wmin) / kT), 0.0)
    ref *= 2 * math.pi / N * nb * (nb + 1) * om
    assert np.max(ref) > 0
    assert np.max(np.abs(out["P"] - ref)) < 1e-9 * np.max(ref)


def test_linewidth_at_q_subset_other_sum_order():
    """P at a subset of q with the lattice sums in the other order (Rp first at each q,
    then Re at every kept k) equals the full-mesh evaluation (Re first per k), for a
    plain system and for a polar one; and reproduces the Einstein closed form."""
    for polar in (False, True):
        s = synth.small_system(33, n_wannier=4, n_atoms=2, r=1)
        s.h_r *= 0.3
        if polar:
            synth.add_polar(s, 5)
        mesh = (3, 2, 4)
        t = rates.mesh_tables(s, mesh)
        mu = float(np.median(t["eps"]))
        par = dict(mu=mu, kT=KB * 300.0, sigma=0.05, win_lo=mu - 0.7, win_hi=mu + 0.7)
        full = linewidth.phonon_linewidth(s, mesh, tables=t, **par)["P"]
        q = np.array([0, 5, 11, 23])
        sub = linewidth.phonon_linewidth_at(s, mesh, q, tables=t, k_chunk=3, **par)
        assert np.max(full) > 0
        assert np.max(np.abs(sub - full[q])) < 1e-12 * np.max(full)
    s, e, kk, M, G0 = _einstein_system()
    kT = KB * 300.0
    a = linewidth.phonon_linewidth(s, (2, 3, 2), 0.01, kT, 0.04, -0.07, 0.05)["P"]
    b = linewidth.phonon_linewidth_at(s, (2, 3, 2), [0, 7], 0.01, kT, 0.04, -0.07, 0.05)
    assert np.max(np.abs(b - a[[0, 7]])) < 1e-12 * np.max(a)
