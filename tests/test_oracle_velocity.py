"""Pins of the velocity operator and adaptive smearing (Velocity; Dirac delta and Smearing).

* group velocities against the paper's central difference of the band
  energies (Cartesian step 2 pi delta / a);
* a degenerate pair of orbitals dispersing along x and along y: the
  diagonalised degenerate block gives the two orbital velocities, also after a
  random unitary change of the Wannier basis;
* the adaptive sigma is the standard deviation of the linearised energy change
  over a uniform displacement inside one mesh cell (Monte Carlo);
* flat bands have zero velocity: adaptive smearing equals fixed smearing at
  sigma_min, for the rates and for the phonon linewidth;
* rates with adaptive smearing against explicit loops on a 2x2x2 mesh.
"""

import itertools
import math

import numpy as np
import scipy.constants as sc

import synth
from helpers import random_unitary
from oracle import linewidth, rates, velocity
from test_oracle_rates import _einstein_system

KB = sc.k / sc.electron_volt
C_OMEGA = sc.hbar * math.sqrt(sc.electron_volt / sc.angstrom ** 2 / sc.atomic_mass) / sc.electron_volt
C_PH = sc.hbar ** 2 / (sc.atomic_mass * sc.angstrom ** 2) / sc.electron_volt


def test_velocity_matches_central_difference():
    s = synth.small_system(seed=61, n_wannier=4, n_atoms=2, r=2)
    rng = np.random.default_rng(3)
    k = rng.uniform(-1, 1, size=(6, 3))
    eps, v = velocity.group_velocities(k, s.rh, s.h_r)
    gaps = np.min(np.diff(eps, axis=1))
    assert gaps > 1e-3                       # non-degenerate: the diagonal is the velocity
    d = 1e-5
    for a in range(3):
        e1, _ = velocity.electron_bands(k + d * np.eye(3)[a], s.rh, s.h_r)
        e0, _ = velocity.electron_bands(k - d * np.eye(3)[a], s.rh, s.h_r)
        fd = (e1 - e0) / (2 * 2 * math.pi * d)
        assert np.max(np.abs(fd - v[:, :, a])) < 1e-6 * np.max(np.abs(v))


def _two_orbitals(t=0.7):
    R = synth.box_vectors(1)
    h = np.zeros((27, 2, 2), dtype=np.complex128)
    idx = {tuple(r): i for i, r in enumerate(R)}
    h[idx[(1, 0, 0)], 0, 0] = h[idx[(-1, 0, 0)], 0, 0] = t     # 2 t cos(2 pi k_x)
    h[idx[(0, 1, 0)], 1, 1] = h[idx[(0, -1, 0)], 1, 1] = t     # 2 t cos(2 pi k_y)
    return R, h


def test_degenerate_pair_closed_form_and_gauge():
    R, h = _two_orbitals()
    t = 0.7
    kap = 0.13
    k = np.array([[kap, kap, 0.3]])
    vx = -2 * t * math.sin(2 * math.pi * kap)       # d(2 t cos(2 pi k_x)) / d(2 pi k_x)
    ref = np.array([sorted([vx, 0.0]), sorted([vx, 0.0]), [0.0, 0.0]])     # [alpha, band]
    W = random_unitary(np.random.default_rng(0), 2)
    for hh in (h, np.conj(W.T)[None] @ h @ W[None]):
        eps, v = velocity.group_velocities(k, R, hh)
        assert abs(eps[0, 0] - eps[0, 1]) < 1e-12
        assert np.max(np.abs(v[0].T - ref)) < 1e-12


def test_adaptive_sigma_is_std_over_a_mesh_cell():
    rng = np.random.default_rng(7)
    mesh = (8, 5, 12)
    vn, vm = rng.standard_normal(3), rng.standard_normal(3)
    s = velocity.adaptive_sigma(vn, vm, mesh, 0.0)
    u = rng.uniform(-0.5, 0.5, size=(400000, 3))
    dk = 2 * math.pi * u / np.array(mesh)              # Cartesian displacements in one cell
    de = dk @ (vn - vm)
    assert abs(np.std(de) - s) < 5e-3 * s
    assert velocity.adaptive_sigma(vn, vn, mesh, 0.004) == 0.004


def test_flat_bands_adaptive_equals_fixed_at_sigma_min():
    s, e, kk, M, G0 = _einstein_system()
    kT, mu, smin = KB * 300.0, 0.01, 0.04
    mesh = (2, 3, 2)
    fixed = rates.scattering_rates(s, mesh, mu, kT, smin, -1e9, 1e9)
    adapt = rates.scattering_rates(s, mesh, mu, kT, 123.0, -1e9, 1e9,
                                   adaptive=dict(sigma_min=smin))
    assert np.max(np.abs(fixed["gamma"] - adapt["gamma"])) < 1e-12 * np.max(fixed["gamma"])
    pf = linewidth.phonon_linewidth(s, mesh, mu, kT, smin, -0.07, 0.05)
    pa = linewidth.phonon_linewidth(s, mesh, mu, kT, 123.0, -0.07, 0.05,
                                    adaptive=dict(sigma_min=smin))
    assert np.max(np.abs(pf["P"] - pa["P"])) < 1e-12 * np.max(pf["P"])


def _brute_gamma_adaptive(s, mesh, mu, kT, smin, lo, hi, wmin):
    pts = list(itertools.product(*[range(x) for x in mesh]))
    Nq = len(pts)
    frac = lambda t: np.array([t[d] / mesh[d] for d in range(3)])

    def bands_v(kf):
        H = np.zeros((s.n_wannier, s.n_wannier), dtype=np.complex128)
        dH = np.zeros((3, s.n_wannier, s.n_wannier), dtype=np.complex128)
        for i, R in enumerate(s.rh):
            ph = np.exp(2j * math.pi * sum(kf[d] * R[d] for d in range(3)))
            H += s.h_r[i] * ph
            for a in range(3):
                dH[a] += 1j * R[a] * s.h_r[i] * ph
        e, U = np.linalg.eigh(H)
        assert np.min(np.diff(e)) > 1e-6
        v = np.zeros((s.n_wannier, 3))
        for n in range(s.n_wannier):
            for a in range(3):
                v[n, a] = sum(np.conj(U[i, n]) * dH[a, i, j] * U[j, n]
                              for i in range(s.n_wannier) for j in range(s.n_wannier)).real
        return e, U, v

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
        ek, Uk, vk = bands_v(kf)
        for iq, tq in enumerate(pts):
            qf = frac(tq)
            tkq = tuple((tk[d] + tq[d]) % mesh[d] for d in range(3))
            ekq, Ukq, vkq = bands_v(frac(tkq))
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
                        var = sum((2 * math.pi * (vk[n, d] - vkq[m, d]) / mesh[d]) ** 2
                                  for d in range(3)) / 12.0
                        sig = max(math.sqrt(var), smin)
                        fm = 1.0 / (math.exp((ekq[m] - mu) / kT) + 1.0)
                        d1 = math.exp(-((ek[n] - ekq[m] - w) / sig) ** 2) / (math.sqrt(math.pi) * sig)
                        d2 = math.exp(-((ek[n] - ekq[m] + w) / sig) ** 2) / (math.sqrt(math.pi) * sig)
                        out[ik, n] += 2 * math.pi / Nq * abs(gv) ** 2 * ((nb + 1 - fm) * d1 + (nb + fm) * d2)
    return out


def test_rates_adaptive_brute_force_tiny_mesh():
    s = synth.small_system(seed=31, n_wannier=2, n_atoms=1, r=1)
    s.h_r = s.h_r * 0.05
    mesh = (2, 2, 2)
    kT, smin, wmin = KB * 300.0, 0.01, 1e-4
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    lo, hi = mu - 0.15, mu + 0.15
    out = rates.scattering_rates(s, mesh, mu, kT, 1.0, lo, hi, wmin, k_idx=np.arange(8), tables=t,
                                 adaptive=dict(sigma_min=smin))
    ref = _brute_gamma_adaptive(s, mesh, mu, kT, smin, lo, hi, wmin)
    assert np.max(ref) > 0
    assert np.max(np.abs(out["gamma"] - ref)) < 1e-8 * np.max(ref)
    # the widths vary: adaptive smearing is not fixed smearing at sigma_min
    fixed = rates.scattering_rates(s, mesh, mu, kT, smin, lo, hi, wmin, k_idx=np.arange(8), tables=t)
    assert np.max(np.abs(fixed["gamma"] - ref)) > 1e-3 * np.max(ref)
