"""Pins of the scattering-rate sum (electron BTE lifetime; Dirac delta and smearing).

* the Gaussian delta integrates to one with second moment sigma^2/2;
* detailed balance of the occupation factors: f_n (1 - f_m)(n + 1) =
  (1 - f_n) f_m n whenever eps_n - eps_m = hbar omega;
* closed form: flat bands and Einstein phonons with a single lattice term make
  the rate independent of the mesh and equal to a short explicit sum;
* brute force: every sum written as explicit Python loops on a 2x2x2 mesh;
* Gamma >= 0; explicit q lists with uniform weights reproduce the full mesh;
* the energy window and kept-point list against a brute-force scan.
"""

import itertools
import math

import numpy as np
import scipy.constants as sc

import synth
from oracle import bands, constants, rates

KB = sc.k / sc.electron_volt
C_OMEGA = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt
C_PH = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt


def test_gaussian_normalisation_and_width():
    sigma = 0.013
    x = np.linspace(-20 * sigma, 20 * sigma, 200001)
    d = rates.gaussian_delta(x, sigma)
    dx = x[1] - x[0]
    assert abs(np.sum(d) * dx - 1.0) < 1e-10
    assert abs(np.sum(x * x * d) * dx - sigma ** 2 / 2) < 1e-10 * sigma ** 2


def test_detailed_balance_of_occupations():
    kT, mu = 0.031, 0.2
    rng = np.random.default_rng(0)
    for _ in range(20):
        em = rng.uniform(-0.3, 0.5)
        w = rng.uniform(0.005, 0.2)
        en = em + w
        fn = bands.fermi_dirac(np.array([en]), mu, kT)[0]
        fm = bands.fermi_dirac(np.array([em]), mu, kT)[0]
        n = bands.bose_einstein(np.array([w]), kT)[0]
        lhs = fn * (1 - fm) * (n + 1)
        rhs = (1 - fn) * fm * n
        # 1 - f loses digits when f -> 1, hence the 1e-9 relative bound
        assert abs(lhs - rhs) < 1e-9 * max(lhs, rhs)


def _einstein_system(nW=3, M=1.7):
    rng = np.random.default_rng(5)
    R = synth.box_vectors(1)
    i0 = 13
    kk = np.array([0.6, 1.1, 1.45])
    phi = np.zeros((27, 3, 3))
    phi[i0] = np.diag(kk)
    e = np.array([-0.05, 0.02, 0.09])[:nW]
    h = np.zeros((27, nW, nW), dtype=np.complex128)
    h[i0] = np.diag(e)
    g = np.zeros((27, 27, 3, nW, nW), dtype=np.complex128)
    G0 = rng.standard_normal((3, nW, nW)) + 1j * rng.standard_normal((3, nW, nW))
    g[i0, i0] = G0
    s = synth.System(n_wannier=nW, n_atoms=1, positions=np.zeros((1, 3)), mass=np.array([M]),
                     rh=R, h_r=h, rd=R, phi_r=phi, re=R, rp=R, g_rr=g)
    return s, e, kk, M, G0


def test_einstein_flat_closed_form_independent_of_mesh():
    s, e, kk, M, G0 = _einstein_system()
    T, mu, sigma = 300.0, 0.01, 0.04
    kT = KB * T
    w = C_OMEGA * np.sqrt(kk / M)
    l2 = C_PH / (2 * M * w)
    ref = np.zeros(3)
    for n in range(3):
        for m in range(3):
            fm = 1.0 / (math.exp((e[m] - mu) / kT) + 1.0)
            for v in range(3):
                nb = 1.0 / math.expm1(w[v] / kT)
                g2 = abs(G0[v, n, m]) ** 2 * l2[v]
                d1 = math.exp(-((e[n] - e[m] - w[v]) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                d2 = math.exp(-((e[n] - e[m] + w[v]) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                ref[n] += 2 * math.pi * g2 * ((nb + 1 - fm) * d1 + (nb + fm) * d2)
    for mesh in [(2, 3, 2), (3, 3, 3)]:
        out = rates.scattering_rates(s, mesh, mu, kT, sigma, -1e9, 1e9)
        assert np.max(np.abs(out["gamma"] - ref[None, :])) < 1e-8 * np.max(ref)


def _brute_gamma(s, mesh, mu, kT, sigma, lo, hi, wmin):
    """Every sum as explicit loops; LAPACK only for the 2x2/3x3 eigenproblems."""
    pts = list(itertools.product(*[range(x) for x in mesh]))
    Nq = len(pts)

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

    out = np.zeros((Nq, s.n_wannier))
    for ik, tk in enumerate(pts):
        kf = frac(tk)
        ek, Uk = ham(kf)
        for iq, tq in enumerate(pts):
            qf = frac(tq)
            tkq = tuple((tk[d] + tq[d]) % mesh[d] for d in range(3))
            ekq, Ukq = ham(frac(tkq))
            lam, z = dyn(qf)
            G = np.zeros(s.g_rr.shape[2:], dtype=np.complex128)
            for a, Re in enumerate(s.re):
                for b, Rp in enumerate(s.rp):
                    ph = sum(kf[d] * Re[d] + qf[d] * Rp[d] for d in range(3))
                    G += np.exp(2j * math.pi * ph) * s.g_rr[a, b]
            for n in range(s.n_wannier):
                if not (lo < ek[n] < hi):
                    continue
                for v in range(3 * s.n_atoms):
                    w = C_OMEGA * math.sqrt(max(lam[v], 0.0))
                    if w < wmin:
                        continue
                    nb = 1.0 / math.expm1(w / kT)
                    for m in range(s.n_wannier):
                        gv = 0.0j
                        for sa in range(3 * s.n_atoms):
                            l = math.sqrt(C_PH / (2 * s.mass[sa // 3] * w))
                            for a in range(s.n_wannier):
                                for b in range(s.n_wannier):
                                    gv += np.conj(Uk[a, n]) * G[sa, a, b] * Ukq[b, m] * z[sa, v] * l
                        fm = 1.0 / (math.exp((ekq[m] - mu) / kT) + 1.0)
                        d1 = math.exp(-((ek[n] - ekq[m] - w) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                        d2 = math.exp(-((ek[n] - ekq[m] + w) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                        out[ik, n] += 2 * math.pi / Nq * abs(gv) ** 2 * ((nb + 1 - fm) * d1 + (nb + fm) * d2)
    return out


def test_brute_force_tiny_mesh():
    s = synth.small_system(seed=31, n_wannier=2, n_atoms=1, r=1)
    # shrink the band width so that phonon-assisted transitions are resonant
    s.h_r = s.h_r * 0.05
    mesh = (2, 2, 2)
    kT, sigma, wmin = KB * 300.0, 0.05, 1e-4
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    lo, hi = mu - 0.15, mu + 0.15
    out = rates.scattering_rates(s, mesh, mu, kT, sigma, lo, hi, wmin,
                                 k_idx=np.arange(8), tables=t)
    ref = _brute_gamma(s, mesh, mu, kT, sigma, lo, hi, wmin)
    assert np.max(ref) > 0
    assert np.max(np.abs(out["gamma"] - ref)) < 1e-8 * np.max(ref)
    assert np.array_equal(out["band_mask"], ((t["eps"] > lo) & (t["eps"] < hi)).astype(np.uint8))


def test_nonnegative_and_q_lists_reproduce_full_mesh():
    s = synth.config_c1()
    mesh = (6, 6, 6)
    kT = constants.kT_of(300.0)
    t = rates.mesh_tables(s, mesh)
    mu = 0.5 * (t["eps"].min() + t["eps"].max())
    k_idx = np.array([0, 7, 100, 215])
    full = rates.scattering_rates(s, mesh, mu, kT, 0.02, -1e9, 1e9, k_idx=k_idx, tables=t)
    assert np.all(full["gamma"] >= 0)
    nq = 216
    rng = np.random.default_rng(0)
    q_idx = np.concatenate([rng.permutation(nq) for _ in k_idx])
    q_off = np.arange(len(k_idx) + 1) * nq
    q_w = np.full(q_idx.size, 1.0 / nq)
    lst = rates.scattering_rates(s, mesh, mu, kT, 0.02, -1e9, 1e9, k_idx=k_idx, tables=t,
                                 q_lists=(q_off, q_idx, q_w), q_chunk=50)
    assert np.max(np.abs(lst["gamma"] - full["gamma"])) < 1e-12 * np.max(full["gamma"])


def test_window_and_kept_points_brute_force():
    rng = np.random.default_rng(4)
    eps = rng.uniform(-1, 1, size=(50, 4))
    lo, hi = -0.1, 0.05
    m = rates.window_mask(eps, lo, hi)
    kept = rates.kept_points(m)
    ref = [i for i in range(50) if any(lo < eps[i, b] < hi for b in range(4))]
    assert list(kept) == ref
    for i in range(50):
        for b in range(4):
            assert m[i, b] == (1 if lo < eps[i, b] < hi else 0)
