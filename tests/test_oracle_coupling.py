"""Pins of the rotated coupling g_{n m nu}(k, q) (Electron Properties).

* gauge invariance: a k-independent unitary change of the Wannier basis,
  applied to H(R) and to both Wannier indices of g(Re, Rp), leaves the
  degenerate-summed |g|^2 unchanged (the Wannier gauge is arbitrary);
* Cartesian invariance: rotating the displacement basis of Phi(R) and of the
  s-alpha index of g(Re, Rp) leaves |g|^2 unchanged;
* closed form: flat bands in the eigenbasis (U = 1), Einstein phonons with
  distinct diagonal springs (z = 1) and a single lattice term give
  |g_{n m nu}|^2 = |g0_{nu n m}|^2 hbar / (2 M omega_nu);
* reciprocal-lattice periodicity of |g|^2.
"""

import copy
import math

import numpy as np
import scipy.constants as sc

import synth
from helpers import group_sum_g2, random_rotation, random_unitary
from oracle import coupling


def _compare_invariant(o1, o2, tol):
    g1, g2 = o1["g"], o2["g"]
    nk, nq = g1.shape[:2]
    worst = 0.0
    for i in range(nk):
        for j in range(nq):
            a = group_sum_g2(g1[i, j], o1["eps_k"][i], o1["eps_kq"][i, j], o1["omega_q"][j])
            b = group_sum_g2(g2[i, j], o2["eps_k"][i], o2["eps_kq"][i, j], o2["omega_q"][j])
            worst = max(worst, np.max(np.abs(a - b)) / np.max(np.abs(a)))
    assert worst < tol, worst


def test_wannier_gauge_invariance():
    s = synth.small_system(seed=21, n_wannier=3, n_atoms=2, r=1)
    rng = np.random.default_rng(0)
    W = random_unitary(rng, 3)
    s2 = copy.deepcopy(s)
    Wh = np.conj(W.T)
    s2.h_r = Wh[None] @ s.h_r @ W[None]
    s2.g_rr = Wh @ s.g_rr @ W
    k = rng.uniform(-1, 1, size=(3, 3))
    q = rng.uniform(-1, 1, size=(4, 3))
    _compare_invariant(coupling.coupling(k, q, s), coupling.coupling(k, q, s2), 1e-11)


def test_cartesian_rotation_invariance():
    s = synth.small_system(seed=22, n_wannier=2, n_atoms=2, r=1)
    rng = np.random.default_rng(1)
    O = random_rotation(rng)
    Ob = np.kron(np.eye(s.n_atoms), O)
    s2 = copy.deepcopy(s)
    s2.phi_r = Ob[None] @ s.phi_r @ Ob.T[None]
    s2.g_rr = np.einsum("ab,xybnm->xyanm", Ob, s.g_rr)
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(4, 3))
    o1, o2 = coupling.coupling(k, q, s), coupling.coupling(k, q, s2)
    assert np.max(np.abs(o1["omega_q"] - o2["omega_q"])) < 1e-13
    _compare_invariant(o1, o2, 1e-11)


def test_einstein_flat_closed_form():
    rng = np.random.default_rng(2)
    R = synth.box_vectors(1)
    i0 = 13
    nW, M = 3, 1.7
    kk = np.array([0.6, 1.1, 1.45])                   # distinct springs -> z = 1
    phi = np.zeros((27, 3, 3))
    phi[i0] = np.diag(kk)
    e = np.array([-0.4, 0.1, 0.7])
    h = np.zeros((27, nW, nW), dtype=np.complex128)
    h[i0] = np.diag(e)
    g = np.zeros((27, 27, 3, nW, nW), dtype=np.complex128)
    G0 = rng.standard_normal((3, nW, nW)) + 1j * rng.standard_normal((3, nW, nW))
    g[i0, i0] = G0
    s = synth.System(n_wannier=nW, n_atoms=1, positions=np.zeros((1, 3)), mass=np.array([M]),
                     rh=R, h_r=h, rd=R, phi_r=phi, re=R, rp=R, g_rr=g)
    k = rng.uniform(-1, 1, size=(3, 3))
    q = rng.uniform(-1, 1, size=(3, 3))
    out = coupling.coupling(k, q, s)
    hw = sc.hbar * np.sqrt(kk * sc.electron_volt / sc.angstrom ** 2 / (M * sc.atomic_mass))
    l2 = sc.hbar ** 2 / (2 * M * sc.atomic_mass * hw) / sc.angstrom ** 2     # (hbar/2 M omega) in A^2
    ref = np.abs(G0) ** 2 * l2[:, None, None]
    got = np.abs(out["g"]) ** 2
    assert np.max(np.abs(got - ref[None, None]) / np.max(ref)) < 1e-8


def test_reciprocal_lattice_periodicity():
    s = synth.small_system(seed=23, n_wannier=3, n_atoms=2, r=1)
    rng = np.random.default_rng(3)
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(3, 3))
    o1 = coupling.coupling(k, q, s)
    o2 = coupling.coupling(k + np.array([2, -1, 1]), q + np.array([-1, 0, 3]), s)
    _compare_invariant(o1, o2, 1e-10)
