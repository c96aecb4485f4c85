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


# ---------------------------------------------------------------------------
# phoebe_gpu_interp_g_mesh: q the full mesh, the sum over Rp axis by axis
# ---------------------------------------------------------------------------
def _mesh_frac(mesh, idx=None):
    N = int(np.prod(mesh))
    idx = np.arange(N) if idx is None else np.asarray(idx)
    i0, r = np.divmod(idx, mesh[1] * mesh[2])
    i1, i2 = np.divmod(r, mesh[2])
    return np.stack([i0 / mesh[0], i1 / mesh[1], i2 / mesh[2]], axis=1)


def _run_mesh(lib, s, k, mesh, precision="fp64", omega_min=1e-4):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    ds = DeviceSystem.from_host(s)
    nk, nq, nW, nm = k.shape[0], int(np.prod(mesh)), s.n_wannier, s.n_modes
    g = torch.empty((nk, nq, nm, nW, nW), dtype=torch.complex128, device="cuda")
    ek = torch.empty((nk, nW), dtype=torch.float64, device="cuda")
    ekq = torch.empty((nk, nq, nW), dtype=torch.float64, device="cuda")
    om = torch.empty((nq, nm), dtype=torch.float64, device="cuda")
    lib.interp_g_mesh(ds, torch.from_numpy(k).cuda(), mesh, g, omega_min=omega_min,
                      precision=precision, eps_k=ek, eps_kq=ekq, omega_q=om)
    torch.cuda.synchronize()
    return dict(g=g.cpu().numpy(), eps_k=ek.cpu().numpy(), eps_kq=ekq.cpu().numpy(),
                omega_q=om.cpu().numpy())


@pytest.mark.parametrize("nW,nat,r,mesh", [(5, 2, 2, (5, 4, 3)), (16, 5, 1, (3, 4, 5)),
                                           (9, 1, 2, (7, 1, 2)), (20, 2, 1, (4, 3, 3)),
                                           (8, 6, 1, (3, 4, 3)), (1, 1, 1, (2, 3, 2)),
                                           (6, 2, 1, (1, 4, 3))])
def test_mesh_form_matches_oracle_and_list_form(lib, nW, nat, r, mesh):
    """The factorised sum over Rp on a full (ragged) q mesh against the oracle, and
    against the dense contraction of phoebe_gpu_interp_g on the same q points (the
    same bands and modes, so g itself agrees, not only |g|^2).  Up to 16 bands and 16
    modes the last axis and the rotation run in one kernel; 20 bands, or 18 modes,
    take the two-kernel form; one band, and a mesh of a single q0 plane, are the edge
    cases of the fused kernel."""
    s = synth.small_system(60 + nW, n_wannier=nW, n_atoms=nat, r=r)
    rng = np.random.default_rng(nW)
    k = rng.uniform(-1, 1, size=(3, 3))
    q = _mesh_frac(mesh)
    got = _run_mesh(lib, s, k, mesh)
    ref = coupling.coupling(k, q, s)
    _compare(got, ref, 1e-11)
    lst = _run(lib, s, k, q)
    scale = np.max(np.abs(lst["g"]))
    d = np.max(np.abs(got["g"] - lst["g"]))
    print(f"mesh form vs list form: max |dg| / max |g| = {d / scale:.2e}", flush=True)
    assert d < 1e-12 * scale
    assert np.array_equal(got["eps_kq"], lst["eps_kq"])


@pytest.mark.parametrize("nW,nat,r,mesh", [(5, 2, 2, (5, 4, 3)), (16, 5, 1, (4, 3, 4))])
def test_mesh_form_k_on_mesh(lib, nW, nat, r, mesh):
    """k points on the q mesh (k + q on the mesh: the mesh's bands gathered per pair)
    against the oracle; a k written as -1/N0 + 1 exercises the wrap to the mesh index."""
    s = synth.small_system(70 + nW, n_wannier=nW, n_atoms=nat, r=r)
    N = int(np.prod(mesh))
    ik = np.array([0, 7 % N, N - 1])
    k = _mesh_frac(mesh, ik)
    k[2, 0] -= 1.0  # the same mesh point, one period away
    got = _run_mesh(lib, s, k, mesh)
    ref = coupling.coupling(k, _mesh_frac(mesh), s)
    _compare(got, ref, 1e-11)


def test_mesh_form_fp32(lib):
    """FP32 form of the mesh interpolation against the FP64 oracle."""
    s = synth.small_system(77, n_wannier=8, n_atoms=3, r=2)
    mesh = (4, 5, 3)
    k = np.random.default_rng(5).uniform(-1, 1, size=(2, 3))
    got = _run_mesh(lib, s, k, mesh, precision="fp32")
    ref = coupling.coupling(k, _mesh_frac(mesh), s)
    _compare(got, ref, 1e-6)


def test_mesh_form_argument_errors(lib):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem, PhoebeError
    s = synth.small_system(78, n_wannier=3, n_atoms=1, r=1)
    ds = DeviceSystem.from_host(s)
    k = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    g = torch.empty((1, 8, 3, 3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(PhoebeError) as e:
        lib.interp_g_mesh(ds, k, (2, 0, 4), g)
    assert e.value.status == -1


def test_realistic_size_mesh_launch(lib):
    """Realistic system (nW 16, 15 modes, 343 Re and Rp): two mesh k against the whole
    40^3 q mesh in one phoebe_gpu_interp_g_mesh call, as bench.py times it; 64 seeded
    q of the result against the oracle, which evaluates those pairs one by one."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = synth.config_c2()
    mesh = (40, 40, 40)
    N = int(np.prod(mesh))
    rng = np.random.default_rng(31)
    ik = np.sort(rng.choice(N, size=2, replace=False))
    iq = np.sort(rng.choice(N, size=64, replace=False))
    k = _mesh_frac(mesh, ik)
    ds = DeviceSystem.from_host(s)
    nW, nm = s.n_wannier, s.n_modes
    g = torch.empty((2, N, nm, nW, nW), dtype=torch.complex128, device="cuda")
    ek = torch.empty((2, nW), dtype=torch.float64, device="cuda")
    ekq = torch.empty((2, N, nW), dtype=torch.float64, device="cuda")
    lib.interp_g_mesh(ds, torch.from_numpy(k).cuda(), mesh, g, omega_min=1e-4, eps_k=ek,
                      eps_kq=ekq)
    torch.cuda.synchronize()
    sel = torch.from_numpy(iq).cuda()
    got = dict(g=g[:, sel].cpu().numpy(), eps_k=ek.cpu().numpy(), eps_kq=ekq[:, sel].cpu().numpy())
    del g, ekq, ds
    print("GPU done", flush=True)
    ref = coupling.coupling(k, _mesh_frac(mesh, iq), s)
    _compare(got, ref, 1e-11)


def test_realistic_size_mesh_launch_fp32(lib):
    """The FP32 form of phoebe_gpu_interp_g_mesh at the realistic size (nW 16, 15 modes,
    343 Re and Rp, the whole 40^3 q mesh): 32 seeded q of the result against the FP64
    oracle at the FP32 bound."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = synth.config_c2()
    mesh = (40, 40, 40)
    N = int(np.prod(mesh))
    rng = np.random.default_rng(37)
    ik = np.sort(rng.choice(N, size=1, replace=False))
    iq = np.sort(rng.choice(N, size=32, replace=False))
    k = _mesh_frac(mesh, ik)
    ds = DeviceSystem.from_host(s)
    nW, nm = s.n_wannier, s.n_modes
    g = torch.empty((1, N, nm, nW, nW), dtype=torch.complex128, device="cuda")
    ek = torch.empty((1, nW), dtype=torch.float64, device="cuda")
    ekq = torch.empty((1, N, nW), dtype=torch.float64, device="cuda")
    lib.interp_g_mesh(ds, torch.from_numpy(k).cuda(), mesh, g, omega_min=1e-4, precision="fp32",
                      eps_k=ek, eps_kq=ekq)
    torch.cuda.synchronize()
    sel = torch.from_numpy(iq).cuda()
    got = dict(g=g[:, sel].cpu().numpy(), eps_k=ek.cpu().numpy(), eps_kq=ekq[:, sel].cpu().numpy())
    del g, ekq, ds
    print("GPU done", flush=True)
    ref = coupling.coupling(k, _mesh_frac(mesh, iq), s)
    _compare(got, ref, 1e-6)
