"""Pins of the two phase sums of the coupling interpolation.

The double Fourier sum G(k,q) = sum_{Re,Rp} e^{i2pi(k.Re+q.Rp)} g(Re,Rp)
(Electron Properties, interpolation of g^0) is checked against
* NumPy's inverse FFT on full meshes (a library special case of the same sum),
* explicit loops over (Re, Rp) on tiny inputs,
* closed forms with a single non-zero lattice term,
* the inverse transform of the coarse-grid relation (Bloch to Wannier), which
  must give back g(Re, Rp) on a full mesh.
"""

import numpy as np

import synth
from oracle import coupling, mesh
from oracle.bands import fourier_sum


def _embed(rvecs, n):
    return [tuple(int(r[d]) % n[d] for d in range(3)) for r in rvecs]


def test_fourier_sum_is_ifftn_on_full_mesh():
    rng = np.random.default_rng(0)
    n = (4, 3, 5)
    R = synth.box_vectors(1)
    M = rng.standard_normal((R.shape[0], 2)) + 1j * rng.standard_normal((R.shape[0], 2))
    A = np.zeros(n + (2,), dtype=np.complex128)
    for (i, j, l), r in zip(_embed(R, n), range(R.shape[0])):
        A[i, j, l] += M[r]
    ref = np.fft.ifftn(A, axes=(0, 1, 2)) * np.prod(n)
    got = fourier_sum(mesh.mesh_points(n), R, M).reshape(n + (2,))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_double_sum_is_6d_ifftn_and_inverts():
    s = synth.small_system(seed=5, n_wannier=2, n_atoms=1, r=1)
    nk, nq = (3, 3, 4), (4, 3, 3)
    k = mesh.mesh_points(nk)
    q = mesh.mesh_points(nq)
    G = coupling.coupling_wannier_gauge(k, q, s.re, s.rp, s.g_rr)
    tail = s.g_rr.shape[2:]
    A = np.zeros(nk + nq + tail, dtype=np.complex128)
    for a, ea in enumerate(_embed(s.re, nk)):
        for b, pb in enumerate(_embed(s.rp, nq)):
            A[ea + pb] += s.g_rr[a, b]
    ref = np.fft.ifftn(A, axes=tuple(range(6))) * (np.prod(nk) * np.prod(nq))
    got = G.reshape(nk + nq + tail)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # Bloch -> Wannier on the full mesh recovers g(Re, Rp) (the coarse-grid relation)
    back = np.fft.fftn(got, axes=tuple(range(6))) / (np.prod(nk) * np.prod(nq))
    for a, ea in enumerate(_embed(s.re, nk)):
        for b, pb in enumerate(_embed(s.rp, nq)):
            assert np.max(np.abs(back[ea + pb] - s.g_rr[a, b])) < 1e-13


def test_two_stage_equals_brute_double_loop():
    s = synth.small_system(seed=7, n_wannier=2, n_atoms=1, r=1)
    rng = np.random.default_rng(1)
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(3, 3))
    a = coupling.coupling_wannier_gauge(k, q, s.re, s.rp, s.g_rr)
    b = coupling.coupling_wannier_gauge_brute(k, q, s.re, s.rp, s.g_rr)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_closed_forms_single_lattice_term():
    s = synth.small_system(seed=9, n_wannier=3, n_atoms=1, r=1)
    rng = np.random.default_rng(2)
    k = rng.uniform(-1, 1, size=(4, 3))
    q = rng.uniform(-1, 1, size=(5, 3))
    g = np.zeros_like(s.g_rr)
    i0 = 13                                         # (0,0,0) in box_vectors(1)
    assert not s.re[i0].any() and not s.rp[i0].any()
    g[i0, i0] = s.g_rr[i0, i0]
    G = coupling.coupling_wannier_gauge(k, q, s.re, s.rp, g)
    assert np.max(np.abs(G - g[i0, i0][None, None])) < 1e-14
    ia, ib = 5, 22
    g = np.zeros_like(s.g_rr)
    g[ia, ib] = s.g_rr[ia, ib]
    G = coupling.coupling_wannier_gauge(k, q, s.re, s.rp, g)
    ph = np.exp(2j * np.pi * ((k @ s.re[ia])[:, None] + (q @ s.rp[ib])[None, :]))
    ref = ph[:, :, None, None, None] * g[ia, ib][None, None]
    assert np.max(np.abs(G - ref)) < 1e-14


def test_g_periodicity_of_phase_sum():
    s = synth.small_system(seed=3, n_wannier=2, n_atoms=1, r=1)
    rng = np.random.default_rng(4)
    k = rng.uniform(-1, 1, size=(2, 3))
    q = rng.uniform(-1, 1, size=(2, 3))
    G1 = coupling.coupling_wannier_gauge(k, q, s.re, s.rp, s.g_rr)
    G2 = coupling.coupling_wannier_gauge(k + np.array([1, -2, 3]), q + np.array([0, 1, -1]),
                                         s.re, s.rp, s.g_rr)
    assert np.max(np.abs(G1 - G2)) < 1e-12
