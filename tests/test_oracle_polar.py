"""Pins of the long-range (polar) coupling g^L (Electron Properties, polar decomposition).

* the Coulomb constant against scipy.constants;
* L(q, nu) against the same sum written as explicit Python loops over q, G,
  atoms and Cartesian indices;
* periodicity: L(q + G0) = L(q) for an integer G0 once the G box holds every
  non-negligible term;
* the q -> 0 limit: only the G = 0 term diverges, t L(t q^) tends to
  (4 pi e^2/(4 pi eps0)) / (2 pi) sum_s l_s (q^.Z*_s.z^s) / (q^.eps.q^);
* flat bands with U = 1 and no short-range coupling: g_{nu n m} = i L(q, nu) delta_nm;
* Wannier-gauge invariance of the degenerate-summed |g^S + g^L|^2;
* the rate sum with the polar term against explicit loops on a 3x2x2 mesh.
"""

import copy
import itertools
import math

import numpy as np
import scipy.constants as sc

import synth
from helpers import group_sum_g2, random_unitary
from oracle import bands, constants, coupling, polar, rates

KB = sc.k / sc.electron_volt
C_OMEGA = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt
C_PH = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt
E2 = sc.e / (4 * math.pi * sc.epsilon_0) / sc.angstrom       # e^2/(4 pi eps0) in eV A


def test_coulomb_constant():
    assert abs(constants.E2_4PIEPS0 - E2) < 1e-8 * E2


def _polar_case(seed=3, nat=2, alpha=2.0, g_max=2):
    rng = np.random.default_rng(seed)
    born = rng.standard_normal((nat, 3, 3))
    born -= born.mean(axis=0, keepdims=True)
    A = rng.standard_normal((3, 3))
    eps = 2.0 * np.eye(3) + A @ A.T / 4.0
    nm = 3 * nat
    q = rng.uniform(-1, 1, size=(3, 3))
    z = np.stack([np.linalg.qr(rng.standard_normal((nm, nm)) + 1j * rng.standard_normal((nm, nm)))[0]
                  for _ in range(3)])
    l = rng.uniform(0.05, 0.2, size=(3, nat, nm))
    return q, z, l, born, eps, alpha, g_max


def test_polar_factor_explicit_loops():
    q, z, l, born, eps, alpha, g_max = _polar_case()
    got = polar.polar_factor(q, z, l, born, eps, alpha, g_max)
    nat, nm = born.shape[0], z.shape[-1]
    for i in range(q.shape[0]):
        for v in range(nm):
            acc = 0.0j
            for G in itertools.product(range(-g_max, g_max + 1), repeat=3):
                K = [2 * math.pi * (q[i][d] + G[d]) for d in range(3)]
                if math.sqrt(sum(x * x for x in K)) < 1e-12:
                    continue
                den = sum(K[a] * eps[a, b] * K[b] for a in range(3) for b in range(3))
                damp = math.exp(-den / (4 * alpha))
                for s in range(nat):
                    num = 0.0j
                    for a in range(3):
                        for b in range(3):
                            num += K[a] * born[s, a, b] * z[i, 3 * s + b, v]
                    acc += l[i, s, v] * num * damp / den
            ref = 4 * math.pi * constants.E2_4PIEPS0 * acc
            assert abs(got[i, v] - ref) < 1e-12 * (abs(ref) + 1e-300) + 1e-14


def test_polar_factor_periodic_in_q():
    q, z, l, born, eps, _, _ = _polar_case(seed=4)
    alpha = 1.0          # with eps >= 2: the shell |G| = 3 is below e^-170
    a = polar.polar_factor(q, z, l, born, eps, alpha, 5)
    b = polar.polar_factor(q + np.array([1.0, -1.0, 0.0]), z, l, born, eps, alpha, 5)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_polar_factor_small_q_limit():
    _, z, l, born, eps, alpha, g_max = _polar_case(seed=5)
    qhat = np.array([0.3, -0.5, 0.8])
    qhat /= np.linalg.norm(qhat)
    lim = np.zeros(z.shape[-1], dtype=np.complex128)
    for s in range(born.shape[0]):
        lim += l[0, s] * (qhat @ born[s] @ z[0, 3 * s:3 * s + 3])
    lim *= 4 * math.pi * E2 / (2 * math.pi) / (qhat @ eps @ qhat)
    for t in (1e-5, 1e-7):
        got = t * polar.polar_factor(t * qhat[None], z[:1], l[:1], born, eps, alpha, g_max)[0]
        assert np.max(np.abs(got - lim)) < 20 * t * np.max(np.abs(lim)) + 1e-12 * np.max(np.abs(lim))


def _flat_polar_system():
    nW = 3
    R = synth.box_vectors(1)
    i0 = 13
    h = np.zeros((27, nW, nW), dtype=np.complex128)
    h[i0] = np.diag([-0.05, 0.02, 0.09])
    s = synth.small_system(seed=41, n_wannier=nW, n_atoms=2, r=1)
    s.rh, s.h_r = R, h
    s.g_rr = np.zeros_like(s.g_rr)
    return synth.add_polar(s, seed=41, alpha=3.0, g_max=2, eps_scale=2.0)


def test_flat_bands_no_short_range_gives_i_L_delta():
    s = _flat_polar_system()
    rng = np.random.default_rng(2)
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(5, 3))
    out = coupling.coupling(k, q, s)
    omega, z, _ = bands.phonon_modes(q, s.rd, s.phi_r, s.mass)
    l = coupling.phonon_length(omega, s.mass, 1e-4)
    L = polar.polar_factor(q, z, l, s.born, s.eps_inf, s.ewald_alpha, s.g_max)
    assert np.max(np.abs(L)) > 0
    ref = 1j * L[None, :, :, None, None] * np.eye(3)[None, None, None]
    assert np.max(np.abs(np.abs(out["g"]) - np.abs(ref))) < 1e-12 * np.max(np.abs(L))
    # the same magnitude at every k: U_k^dagger U_{k+q} is diagonal with unit entries
    assert np.max(np.abs(np.abs(out["g"][0]) - np.abs(out["g"][1]))) < 1e-12 * np.max(np.abs(L))


def test_wannier_gauge_invariance_with_polar():
    s = synth.add_polar(synth.small_system(seed=21, n_wannier=3, n_atoms=2, r=1), seed=21,
                        alpha=3.0, g_max=2, eps_scale=2.0)
    rng = np.random.default_rng(0)
    W = random_unitary(rng, 3)
    s2 = copy.deepcopy(s)
    Wh = np.conj(W.T)
    s2.h_r = Wh[None] @ s.h_r @ W[None]
    s2.g_rr = Wh @ s.g_rr @ W
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(4, 3))
    o1, o2 = coupling.coupling(k, q, s), coupling.coupling(k, q, s2)
    o0 = coupling.coupling(k, q, synth.small_system(seed=21, n_wannier=3, n_atoms=2, r=1))
    worst, change = 0.0, 0.0
    for i in range(2):
        for j in range(4):
            a = group_sum_g2(o1["g"][i, j], o1["eps_k"][i], o1["eps_kq"][i, j], o1["omega_q"][j])
            b = group_sum_g2(o2["g"][i, j], o2["eps_k"][i], o2["eps_kq"][i, j], o2["omega_q"][j])
            c = group_sum_g2(o0["g"][i, j], o0["eps_k"][i], o0["eps_kq"][i, j], o0["omega_q"][j])
            worst = max(worst, np.max(np.abs(a - b)) / np.max(a))
            change = max(change, np.max(np.abs(a - c)) / np.max(a))
    assert worst < 1e-11
    assert change > 1e-3          # the polar term is not negligible in this case


def _brute_gamma_polar(s, mesh, mu, kT, sigma, lo, hi, wmin):
    pts = list(itertools.product(*[range(x) for x in mesh]))
    Nq = len(pts)
    frac = lambda t: np.array([t[d] / mesh[d] for d in range(3)])

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

    def Lq(qf, w, z, v):
        acc = 0.0j
        for G in itertools.product(range(-s.g_max, s.g_max + 1), repeat=3):
            K = [2 * math.pi * (qf[d] + G[d]) for d in range(3)]
            if math.sqrt(sum(x * x for x in K)) < 1e-12:
                continue
            den = sum(K[a] * s.eps_inf[a, b] * K[b] for a in range(3) for b in range(3))
            damp = math.exp(-den / (4 * s.ewald_alpha))
            for at in range(s.n_atoms):
                l = math.sqrt(C_PH / (2 * s.mass[at] * w))
                num = sum(K[a] * s.born[at, a, b] * z[3 * at + b, v] for a in range(3) for b in range(3))
                acc += l * num * damp / den
        return 4 * math.pi * E2 * acc

    out = np.zeros((Nq, s.n_wannier))
    for ik, tk in enumerate(pts):
        kf = frac(tk)
        ek, Uk = ham(kf)
        for iq, tq in enumerate(pts):
            qf = frac(tq)
            tkq = tuple((tk[d] + tq[d]) % mesh[d] for d in range(3))
            ekq, Ukq = ham(frac(tkq))
            lam, z = dyn(qf)
            Lv = [Lq(qf, C_OMEGA * math.sqrt(max(lam[v], 0.0)), z, v)
                  if C_OMEGA * math.sqrt(max(lam[v], 0.0)) >= wmin else 0.0
                  for v in range(3 * s.n_atoms)]
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
                    L = Lv[v]
                    for m in range(s.n_wannier):
                        gv = 0.0j
                        for sa in range(3 * s.n_atoms):
                            l = math.sqrt(C_PH / (2 * s.mass[sa // 3] * w))
                            for a in range(s.n_wannier):
                                for b in range(s.n_wannier):
                                    gv += np.conj(Uk[a, n]) * G[sa, a, b] * Ukq[b, m] * z[sa, v] * l
                        ov = sum(np.conj(Uk[a, n]) * Ukq[a, m] for a in range(s.n_wannier))
                        gv += 1j * L * ov
                        fm = 1.0 / (math.exp((ekq[m] - mu) / kT) + 1.0)
                        d1 = math.exp(-((ek[n] - ekq[m] - w) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                        d2 = math.exp(-((ek[n] - ekq[m] + w) / sigma) ** 2) / (math.sqrt(math.pi) * sigma)
                        out[ik, n] += 2 * math.pi / Nq * abs(gv) ** 2 * ((nb + 1 - fm) * d1 + (nb + fm) * d2)
    return out


def test_rates_with_polar_brute_force_tiny_mesh():
    s = synth.add_polar(synth.small_system(seed=33, n_wannier=2, n_atoms=2, r=1), seed=33,
                        alpha=3.0, g_max=1, eps_scale=2.0)
    s.h_r = s.h_r * 0.05
    # a 2x2x2 mesh holds only points q = -q (mod G), where the odd sum over G
    # cancels: one axis of 3 points
    mesh = (3, 2, 2)
    kT, sigma, wmin = KB * 300.0, 0.05, 1e-4
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    lo, hi = mu - 0.2, mu + 0.2
    out = rates.scattering_rates(s, mesh, mu, kT, sigma, lo, hi, wmin, k_idx=np.arange(12), tables=t)
    ref = _brute_gamma_polar(s, mesh, mu, kT, sigma, lo, hi, wmin)
    assert np.max(ref) > 0
    assert np.max(np.abs(out["gamma"] - ref)) < 1e-8 * np.max(ref)
    s0 = copy.deepcopy(s)
    s0.born = None
    plain = rates.scattering_rates(s0, mesh, mu, kT, sigma, lo, hi, wmin, k_idx=np.arange(12), tables=t)
    assert np.max(np.abs(plain["gamma"] - out["gamma"])) > 1e-3 * np.max(ref)
