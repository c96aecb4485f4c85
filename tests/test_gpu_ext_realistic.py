"""The observables beyond the plain rates at the realistic size, in the launch
configurations bench.py times (perovskite, 15 modes, nW = 16, 343 Re and Rp,
40^3 k and q meshes, window +-0.3 eV):

* phonon linewidth P^{el-ph} (Transport Methods, phonon BTE) on every q of the
  mesh; the oracle evaluates 4 seeded q (its lattice sums in the other order,
  over every kept k); the electron rates of the same pass equal the plain path's;
* adaptive smearing (Dirac delta and Smearing) and the polar long-range coupling
  (Electron Properties): Gamma on every kept k, the oracle on 2 seeded kept k
  over the full q mesh;
* 3-phonon coupling V3 (Phonon Properties) for 16 q x 4096 q' on the perovskite
  with third-order constants on [-2, 2]^3: |V3| of 2 x 24 seeded pairs against
  the oracle.
"""

import numpy as np
import pytest

import synth
from gpu_common import rel_err, torch_cuda, workload_params
from oracle import linewidth, phonon3, rates

pytestmark = pytest.mark.gpu

BOUND = 1e-9


def _realistic():
    p = workload_params()["realistic"]
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    return p, tuple(p["mesh"]), par


@pytest.fixture(scope="module")
def lib():
    torch_cuda()
    from paper_2111_14999_amd import Library
    L = Library(0)
    yield L
    L.close()


@pytest.fixture(scope="module")
def c2():
    s = synth.config_c2()
    p, mesh, par = _realistic()
    return s, mesh, par, rates.mesh_tables(s, mesh)


def test_linewidth_realistic_sampled_q(lib, c2):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s, mesh, par, t = c2
    N = int(np.prod(mesh))
    ds = DeviceSystem.from_host(s)
    P = torch.full((N, s.n_modes), -1.0, dtype=torch.float64, device="cuda")
    gam = torch.zeros((N, s.n_wannier), dtype=torch.float64, device="cuda")
    n = lib.phonon_linewidth(ds, mesh, par, P, gamma_out=gam)
    gp = torch.zeros_like(gam)
    n2 = lib.scatter_rates(ds, mesh, par, gp)
    torch.cuda.synchronize()
    del ds
    assert n == n2 == workload_params()["realistic"]["n_kept"]
    Ph = P.cpu().numpy()
    assert np.all(Ph >= 0.0) and np.max(Ph) > 0.0
    d = np.max(np.abs(gam.cpu().numpy()[:n] - gp.cpu().numpy()[:n]))
    assert d <= 1e-12 * np.max(gp.cpu().numpy())
    q = np.sort(np.random.default_rng(41).choice(N, size=4, replace=False))
    ref = linewidth.phonon_linewidth_at(s, mesh, q, tables=t, **par)
    mx, med, ab = rel_err(Ph[q], ref)
    print(f"[linewidth realistic] q {q.tolist()}: P rel err max {mx:.2e} median {med:.2e}",
          flush=True)
    assert mx < BOUND


@pytest.mark.parametrize("kind", ["adaptive", "polar"])
def test_rates_realistic_sampled_k(lib, c2, kind):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s, mesh, par, t = c2
    N = int(np.prod(mesh))
    kw, par_g = {}, dict(par)
    if kind == "adaptive":
        kw["adaptive"] = dict(sigma_min=par["sigma"], prefactor=1.0)
        par_g.update(smearing="adaptive", adaptive_scale=1.0)
    else:
        s = synth.add_polar(synth.config_c2(), 7)
    ds = DeviceSystem.from_host(s)
    gam = torch.zeros((N, s.n_wannier), dtype=torch.float64, device="cuda")
    kept = torch.zeros(N, dtype=torch.int32, device="cuda")
    n = lib.scatter_rates(ds, mesh, par_g, gam, kept_k_out=kept)
    torch.cuda.synchronize()
    del ds
    g = gam.cpu().numpy()[:n]
    kidx = kept.cpu().numpy()[:n]
    sample = np.sort(np.random.default_rng(43).choice(n, size=2, replace=False))
    ref = rates.scattering_rates(s, mesh, k_idx=kidx[sample], tables=t, **kw, **par)
    mx, med, ab = rel_err(g[sample], ref["gamma"])
    print(f"[{kind} realistic] {n} kept k; Gamma rel err max {mx:.2e} median {med:.2e}",
          flush=True)
    assert mx < BOUND


def test_v3_realistic_sampled_pairs(lib):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem3
    s = synth.config_c2(with_coupling=False)
    r, phi3 = synth.third_order_constants(11, s.n_atoms)
    s.r1, s.r2, s.phi3 = r, r, phi3
    g = np.random.default_rng(12)
    q = g.uniform(-1, 1, size=(16, 3))
    qp = g.uniform(-1, 1, size=(4096, 3))
    d3 = DeviceSystem3.from_host(s, r, phi3)
    nm = s.n_modes
    V = torch.zeros((16, 4096, nm, nm, nm), dtype=torch.complex128, device="cuda")
    lib.interp_v3(d3, torch.from_numpy(q).cuda(), torch.from_numpy(qp).cuda(), V)
    torch.cuda.synchronize()
    iq = np.array([3, 12])
    jq = np.sort(g.choice(4096, size=24, replace=False))
    got = V[torch.from_numpy(iq).cuda()][:, torch.from_numpy(jq).cuda()].cpu().numpy()
    del V, d3
    ref = phonon3.interp_v3(q[iq], qp[jq], s)["v3"]
    err = np.max(np.abs(np.abs(got) - np.abs(ref))) / np.max(np.abs(ref))
    print(f"[V3 realistic] max ||V3| - ref| / max = {err:.2e}", flush=True)
    assert err < 1e-11
