"""Reduced-precision forms (FP32 MFMA, split-BF16 x3 / x6) vs the FP64 oracle.

Phases are formed in FP64 and the band structure, occupations, Gaussians and
the rate sum stay FP64; only the phase and rotation contractions change.  The
bounds below are the measured errors with headroom; the errors themselves are
printed (and reported by bench.py --precision).

FP32 and BF16X6 are held to the stated 1e-6 on Gamma.  BF16X3 (hi + lo BF16
pieces per real operand, the lo x lo product dropped) keeps about 16 bits of
each product, so its products carry relative errors near 2^-17; summed over the
q mesh they leave Gamma errors of a few 1e-6, and its bound is 2e-5.
"""

import numpy as np
import pytest

import synth
from gpu_common import rel_err, torch_cuda, workload_params
from helpers import group_sum_g2
from oracle import constants, coupling, rates

pytestmark = pytest.mark.gpu

# max relative error of Gamma allowed per form (states above 1e-10 of the maximum)
GAMMA_BOUND = {"fp32": 1e-6, "bf16x3": 2e-5, "bf16x6": 1e-6}
# max error of |g|^2 relative to the largest |g|^2 of its (k, q) pair
G2_BOUND = {"fp32": 1e-6, "bf16x3": 2e-5, "bf16x6": 1e-6}


@pytest.fixture(scope="module")
def lib():
    torch_cuda()
    from paper_2111_14999_amd import Library
    L = Library(0)
    yield L
    L.close()


@pytest.fixture(scope="module")
def toy():
    s = synth.config_c1()
    p = workload_params()["toy"]
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    mesh = tuple(p["mesh"])
    ref = rates.scattering_rates(s, mesh, **par)
    return s, mesh, par, ref


def _rates(lib, s, mesh, par, prec):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    ds = DeviceSystem.from_host(s)
    N = int(np.prod(mesh))
    gamma = torch.zeros((N, s.n_wannier), dtype=torch.float64, device="cuda")
    n = lib.scatter_rates(ds, mesh, par, gamma, precision=prec)
    torch.cuda.synchronize()
    return n, gamma.cpu().numpy()[:n]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_toy_rates(lib, toy, prec):
    s, mesh, par, ref = toy
    n, g = _rates(lib, s, mesh, par, prec)
    assert n == len(ref["k_idx"])
    mx, med, ab = rel_err(g, ref["gamma"])
    print(f"[{prec}] Gamma rel err max {mx:.3e} median {med:.3e}", flush=True)
    assert mx < GAMMA_BOUND[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_toy_coupling(lib, toy, prec):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = toy[0]
    rng = np.random.default_rng(5)
    k = rng.uniform(-1, 1, size=(3, 3))
    q = rng.uniform(-1, 1, size=(40, 3))
    ref = coupling.coupling(k, q, s)
    ds = DeviceSystem.from_host(s)
    nk, nq, nW, nm = 3, 40, s.n_wannier, s.n_modes
    g = torch.empty((nk, nq, nm, nW, nW), dtype=torch.complex128, device="cuda")
    lib.interp_g(ds, torch.from_numpy(k).cuda(), torch.from_numpy(q).cuda(), g, precision=prec)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    a = np.empty(g.shape)
    b = np.empty(g.shape)
    for i in range(nk):
        for j in range(nq):
            a[i, j] = group_sum_g2(g[i, j], ref["eps_k"][i], ref["eps_kq"][i, j], ref["omega_q"][j])
            b[i, j] = group_sum_g2(ref["g"][i, j], ref["eps_k"][i], ref["eps_kq"][i, j],
                                   ref["omega_q"][j])
    blk = np.max(b.reshape(nk, nq, -1), axis=2)[:, :, None, None, None]
    err = np.abs(a - b) / blk
    mx, med, _ = rel_err(a, b, floor_frac=1e-6)
    print(f"[{prec}] |g|^2 err/pair-max {np.max(err):.3e}; entrywise (>1e-6 max) max {mx:.3e} "
          f"median {med:.3e}", flush=True)
    assert np.max(err) < G2_BOUND[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
@pytest.mark.parametrize("seed,nW,nat,mesh", [(71, 5, 2, (3, 5, 4)), (72, 16, 5, (2, 3, 4))])
def test_ragged_windows(lib, prec, seed, nW, nat, mesh):
    s = synth.small_system(seed, n_wannier=nW, n_atoms=nat, r=1)
    s.h_r *= 0.3
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.7, win_hi=mu + 0.7,
               omega_min=1e-4)
    ref = rates.scattering_rates(s, mesh, tables=t, **par)
    n, g = _rates(lib, s, mesh, par, prec)
    assert n == len(ref["k_idx"])
    mx, med, ab = rel_err(g, ref["gamma"])
    print(f"[{prec}] ragged Gamma rel err max {mx:.3e} median {med:.3e}", flush=True)
    assert mx < GAMMA_BOUND[prec]


@pytest.mark.parametrize("case", ["toy", "sparse-r", "ragged-5x6x7"])
def test_fp32_mesh_sum_forms(lib, toy, case):
    """FP32 form: the direct and the factorised full-mesh sums both meet the FP32 bound."""
    if case == "toy":
        s, mesh, par, ref = toy
    else:
        rng = np.random.default_rng(8)
        s = synth.small_system(77, n_wannier=5, n_atoms=2, r=2)
        if case == "sparse-r":
            keep_e = np.sort(rng.choice(len(s.re), size=40, replace=False))
            keep_p = np.sort(rng.choice(len(s.rp), size=50, replace=False))
            s.re, s.rp = s.re[keep_e].copy(), s.rp[keep_p].copy()
            s.g_rr = np.ascontiguousarray(s.g_rr[keep_e][:, keep_p])
            mesh = (6, 4, 5)
        else:
            mesh = (5, 6, 7)
        s.h_r *= 0.3
        t = rates.mesh_tables(s, mesh)
        mu = float(np.median(t["eps"]))
        par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.8,
                   win_hi=mu + 0.8, omega_min=1e-4)
        ref = rates.scattering_rates(s, mesh, tables=t, **par)
    try:
        for mode in ("direct", "factored"):
            lib.set_mesh_sum(mode)
            n, g = _rates(lib, s, mesh, par, "fp32")
            assert n == len(ref["k_idx"])
            mx, med, ab = rel_err(g, ref["gamma"])
            print(f"[fp32 {mode}] {case} Gamma rel err max {mx:.3e} median {med:.3e}", flush=True)
            assert mx < GAMMA_BOUND["fp32"]
    finally:
        lib.set_mesh_sum("auto")


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
def test_realistic_size_sampled(lib, prec):
    """Realistic workload (40^3 meshes, nW 16, 343 Re and Rp) in each reduced-precision
    form, in the launch configuration bench.py --precision times; Gamma of 3 seeded
    kept k against the oracle over the full q mesh."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    p = workload_params()["realistic"]
    mesh = tuple(p["mesh"])
    N = int(np.prod(mesh))
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    s = synth.config_c2()
    ds = DeviceSystem.from_host(s)
    gamma = torch.zeros((N, 16), dtype=torch.float64, device="cuda")
    kept = torch.zeros((N,), dtype=torch.int32, device="cuda")
    n = lib.scatter_rates(ds, mesh, par, gamma, kept_k_out=kept, precision=prec)
    torch.cuda.synchronize()
    assert n == p["n_kept"]
    g = gamma.cpu().numpy()[:n]
    kidx = kept.cpu().numpy()[:n]
    del ds
    sample = np.sort(np.random.default_rng(2025).choice(n, size=3, replace=False))
    ref = rates.scattering_rates(s, mesh, k_idx=kidx[sample], **par)
    mx, med, ab = rel_err(g[sample], ref["gamma"])
    print(f"[{prec}] realistic Gamma rel err max {mx:.3e} median {med:.3e}", flush=True)
    assert mx < GAMMA_BOUND[prec]
