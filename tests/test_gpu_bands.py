"""GPU band structure (phase tables + MFMA Fourier sum + batched Jacobi) vs the oracle.

Eigenvalues are compared with LAPACK's; eigenvectors through residuals
against the oracle's own H(k) and D(q) (any phase per vector is valid).
"""

import numpy as np
import pytest

import synth
from gpu_common import torch_cuda
from oracle import bands

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    torch_cuda()
    from paper_2111_14999_amd import Library
    L = Library(0)
    yield L
    L.close()


@pytest.mark.parametrize("make", [lambda: synth.config_c1(),
                                  lambda: synth.small_system(41, n_wannier=7, n_atoms=5, r=1),
                                  lambda: synth.small_system(42, n_wannier=1, n_atoms=1, r=2),
                                  lambda: synth.config_c2(with_coupling=False)],
                         ids=["toy", "nW7-5atoms", "nW1-1atom", "nW16-15modes"])
def test_electron_and_phonon_bands(lib, make):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = make()
    ds = DeviceSystem.from_host(s, with_coupling=False)
    rng = np.random.default_rng(0)
    k = rng.uniform(-1, 1, size=(333, 3))
    k[0] = 0.0
    kd = torch.from_numpy(k).cuda()
    nW, nm = s.n_wannier, s.n_modes
    eps = torch.empty((k.shape[0], nW), dtype=torch.float64, device="cuda")
    U = torch.empty((k.shape[0], nW, nW), dtype=torch.complex128, device="cuda")
    lib.electron_bands(ds, kd, eps, U)
    w = torch.empty((k.shape[0], nm), dtype=torch.float64, device="cuda")
    z = torch.empty((k.shape[0], nm, nm), dtype=torch.complex128, device="cuda")
    lib.phonon_modes(ds, kd, w, z)
    torch.cuda.synchronize()
    eps, U, w, z = eps.cpu().numpy(), U.cpu().numpy(), w.cpu().numpy(), z.cpu().numpy()

    e_ref, _ = bands.electron_bands(k, s.rh, s.h_r)
    H = bands.hamiltonian_k(k, s.rh, s.h_r)
    scale = np.max(np.abs(e_ref))
    assert np.max(np.abs(eps - e_ref)) < 1e-12 * scale
    assert np.max(np.abs(H @ U - U * eps[:, None, :])) < 1e-12 * scale
    assert np.max(np.abs(np.conj(np.swapaxes(U, 1, 2)) @ U - np.eye(nW))) < 1e-12

    w_ref, _, lam = bands.phonon_modes(k, s.rd, s.phi_r, s.mass)
    D = bands.dynamical_matrix(k, s.rd, s.phi_r, s.mass)
    # hbar omega = C sqrt(lambda) amplifies rounding of lambda ~ 0 (acoustic at q = 0)
    big = w_ref > 1e-4
    assert np.max(np.abs(w[big] - w_ref[big]) / w_ref[big]) < 1e-10
    assert np.max(np.abs(w[~big] - w_ref[~big]), initial=0.0) < 1e-6
    res = D @ z - z * np.maximum(lam, 0)[:, None, :]
    assert np.max(np.abs(res)) < 1e-11 * np.max(np.abs(lam))
    assert np.max(np.abs(np.conj(np.swapaxes(z, 1, 2)) @ z - np.eye(nm))) < 1e-12


def test_degenerate_spectrum(lib):
    """H(R) = 0 except H(0) = diag with repeated values: exact degeneracies."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = synth.small_system(43, n_wannier=6, n_atoms=1, r=1)
    s.h_r[:] = 0
    s.h_r[13] = np.diag([0.5, -1.0, 0.5, 2.0, -1.0, 0.5])
    ds = DeviceSystem.from_host(s, with_coupling=False)
    k = np.random.default_rng(1).uniform(-1, 1, size=(17, 3))
    kd = torch.from_numpy(k).cuda()
    eps = torch.empty((17, 6), dtype=torch.float64, device="cuda")
    lib.electron_bands(ds, kd, eps, None)
    torch.cuda.synchronize()
    ref = np.sort([0.5, -1.0, 0.5, 2.0, -1.0, 0.5])
    assert np.max(np.abs(eps.cpu().numpy() - ref[None])) < 1e-15
