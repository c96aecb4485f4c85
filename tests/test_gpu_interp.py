"""GPU el-ph coupling g(k, q) (phoebe_gpu_interp_g) vs the FP64 oracle.

g itself carries the eigensolvers' arbitrary phases, so the comparison is on
|g|^2 summed over degenerate groups of n, m and nu (gauge-free), plus the band
energies returned beside it.
"""

import numpy as np
import pytest

import synth
from gpu_common import rel_err, torch_cuda
from helpers import group_sum_g2
from oracle import coupling

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    torch_cuda()
    from paper_2111_14999_amd import Library
    L = Library(0)
    yield L
    L.close()


def _run(lib, s, k, q, omega_min=1e-4):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    ds = DeviceSystem.from_host(s)
    nk, nq, nW, nm = k.shape[0], q.shape[0], s.n_wannier, s.n_modes
    g = torch.empty((nk, nq, nm, nW, nW), dtype=torch.complex128, device="cuda")
    ek = torch.empty((nk, nW), dtype=torch.float64, device="cuda")
    ekq = torch.empty((nk, nq, nW), dtype=torch.float64, device="cuda")
    om = torch.empty((nq, nm), dtype=torch.float64, device="cuda")
    lib.interp_g(ds, torch.from_numpy(k).cuda(), torch.from_numpy(q).cuda(), g,
                 omega_min=omega_min, eps_k=ek, eps_kq=ekq, omega_q=om)
    torch.cuda.synchronize()
    return dict(g=g.cpu().numpy(), eps_k=ek.cpu().numpy(), eps_kq=ekq.cpu().numpy(),
                omega_q=om.cpu().numpy())


def _compare(got, ref, tol):
    nk, nq = ref["g"].shape[:2]
    a = np.empty(ref["g"].shape)
    b = np.empty(ref["g"].shape)
    for i in range(nk):
        for j in range(nq):
            a[i, j] = group_sum_g2(got["g"][i, j], ref["eps_k"][i], ref["eps_kq"][i, j],
                                   ref["omega_q"][j])
            b[i, j] = group_sum_g2(ref["g"][i, j], ref["eps_k"][i], ref["eps_kq"][i, j],
                                   ref["omega_q"][j])
    # error of each entry relative to the largest |g|^2 of its (k, q) pair: small
    # entries carry the rounding of the large ones they are computed beside
    blk = np.max(b.reshape(nk, nq, -1), axis=2)[:, :, None, None, None]
    err = np.abs(a - b) / np.maximum(blk, 1e-300)
    mx, med, _ = rel_err(a, b)
    print(f"|g|^2 err/pair-max {np.max(err):.3e}; entrywise rel err max {mx:.3e} "
          f"median {med:.3e}", flush=True)
    assert np.max(err) < tol
    sc = np.max(np.abs(ref["eps_k"]))
    assert np.max(np.abs(got["eps_k"] - ref["eps_k"])) < 1e-12 * sc
    assert np.max(np.abs(got["eps_kq"] - ref["eps_kq"])) < 1e-12 * sc


def test_toy_all_pairs_subset(lib):
    s = synth.config_c1()
    rng = np.random.default_rng(0)
    k = rng.uniform(-1, 1, size=(5, 3))
    q = rng.uniform(-1, 1, size=(37, 3))
    q[3] = 0.0                       # acoustic modes drop out (omega < omega_min)
    ref = coupling.coupling(k, q, s)
    got = _run(lib, s, k, q)
    _compare(got, ref, 1e-11)


@pytest.mark.parametrize("nW,nat,r", [(1, 1, 1), (5, 2, 2), (16, 5, 1), (9, 3, 1)])
def test_shapes(lib, nW, nat, r):
    s = synth.small_system(50 + nW, n_wannier=nW, n_atoms=nat, r=r)
    rng = np.random.default_rng(nW)
    k = rng.uniform(-1, 1, size=(3, 3))
    q = rng.uniform(-1, 1, size=(70, 3))     # 70 q: several 64-row tiles and a ragged tail
    ref = coupling.coupling(k, q, s)
    got = _run(lib, s, k, q)
    _compare(got, ref, 1e-11)


def test_realistic_size_bench_launch(lib):
    """Realistic system (nW 16, 15 modes, 343 Re and Rp) in the launch bench times.

    Two mesh k points against the whole 40^3 q mesh in one call, as bench.py
    times it; 64 seeded q of the result are checked against the oracle, which
    evaluates those pairs one by one.
    """
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = synth.config_c2()
    mesh = (40, 40, 40)
    N = int(np.prod(mesh))
    rng = np.random.default_rng(31)
    ik = np.sort(rng.choice(N, size=2, replace=False))
    iq = np.sort(rng.choice(N, size=64, replace=False))

    def frac(idx):
        i0, r = np.divmod(idx, mesh[1] * mesh[2])
        i1, i2 = np.divmod(r, mesh[2])
        return np.stack([i0 / mesh[0], i1 / mesh[1], i2 / mesh[2]], axis=1)

    k = frac(ik)
    q_all = frac(np.arange(N))
    ds = DeviceSystem.from_host(s)
    nW, nm = s.n_wannier, s.n_modes
    g = torch.empty((2, N, nm, nW, nW), dtype=torch.complex128, device="cuda")
    ek = torch.empty((2, nW), dtype=torch.float64, device="cuda")
    ekq = torch.empty((2, N, nW), dtype=torch.float64, device="cuda")
    lib.interp_g(ds, torch.from_numpy(k).cuda(), torch.from_numpy(q_all).cuda(), g,
                 omega_min=1e-4, eps_k=ek, eps_kq=ekq)
    torch.cuda.synchronize()
    sel = torch.from_numpy(iq).cuda()
    got = dict(g=g[:, sel].cpu().numpy(), eps_k=ek.cpu().numpy(), eps_kq=ekq[:, sel].cpu().numpy())
    del g, ekq, ds
    print("GPU done", flush=True)
    ref = coupling.coupling(k, q_all[iq], s)
    _compare(got, ref, 1e-11)
