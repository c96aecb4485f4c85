"""GPU scattering rates (phoebe_gpu_scatter_rates) vs the FP64 oracle.

* window masks, kept-k list and row order: bit-exact;
* Gamma_nk: relative error <= 1e-9 on states with Gamma above 1e-10 of the
  maximum (the FP64 form; the method's stated bound is 1e-6), absolute
  below that;
* ragged cases: meshes that are not multiples of the 64-point q tile, empty
  windows, a single k, explicit weighted q lists;
* determinism: two runs are bitwise equal.
"""

import numpy as np
import pytest

import synth
from gpu_common import rel_err, torch_cuda, workload_params
from oracle import constants, rates

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    torch_cuda()
    from paper_2111_14999_amd import Library
    L = Library(0)
    yield L
    L.close()


def _gpu_rates(lib, s, mesh, par, k_idx=None, q_lists=None, ds=None):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    ds = ds or DeviceSystem.from_host(s)
    N = int(np.prod(mesh))
    rows = N if k_idx is None else len(k_idx)
    gamma = torch.full((max(rows, 1), s.n_wannier), -1.0, dtype=torch.float64, device="cuda")
    mask = torch.empty((max(rows, 1), s.n_wannier), dtype=torch.uint8, device="cuda")
    kept = torch.empty((max(rows, 1),), dtype=torch.int32, device="cuda")
    kd = None if k_idx is None else torch.from_numpy(np.asarray(k_idx, dtype=np.int32)).cuda()
    ql = None
    if q_lists is not None:
        ql = (torch.from_numpy(np.asarray(q_lists[0], dtype=np.int64)).cuda(),
              torch.from_numpy(np.asarray(q_lists[1], dtype=np.int32)).cuda(),
              torch.from_numpy(np.asarray(q_lists[2], dtype=np.float64)).cuda())
    n = lib.scatter_rates(ds, mesh, par, gamma, k_idx=kd, q_lists=ql, band_mask=mask,
                          kept_k_out=kept)
    torch.cuda.synchronize()
    return n, gamma.cpu().numpy()[:n], mask.cpu().numpy()[:n], kept.cpu().numpy()[:n]


def _check(n, g, m, kept, ref, tol=1e-9):
    assert n == len(ref["k_idx"])
    assert np.array_equal(kept, ref["k_idx"].astype(np.int32))
    assert np.array_equal(m, ref["band_mask"])
    assert np.all(g[m == 0] == 0.0)
    mx, med, ab = rel_err(g, ref["gamma"])
    print(f"Gamma rel err max {mx:.3e} median {med:.3e}  abs(small) {ab:.3e}", flush=True)
    assert mx < tol
    assert ab < 1e-10 * max(np.max(ref["gamma"]), 1e-300)




@pytest.fixture(scope="module")
def toy():
    s = synth.config_c1()
    p = workload_params()["toy"]
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    mesh = tuple(p["mesh"])
    ref = rates.scattering_rates(s, mesh, **par)
    return s, mesh, par, ref


def test_toy_workload_all_states(lib, toy):
    s, mesh, par, ref = toy
    n, g, m, kept = _gpu_rates(lib, s, mesh, par)
    assert n == 216
    _check(n, g, m, kept, ref)


def test_toy_deterministic(lib, toy):
    s, mesh, par, ref = toy
    a = _gpu_rates(lib, s, mesh, par)
    b = _gpu_rates(lib, s, mesh, par)
    assert np.array_equal(a[1], b[1])


@pytest.mark.parametrize("seed,nW,nat,r,mesh,half", [
    (61, 3, 2, 1, (4, 3, 5), 0.8),       # 60 q: a single ragged tile
    (62, 5, 1, 2, (5, 5, 3), 0.5),
    (63, 16, 5, 1, (3, 4, 6), 1.5),      # C2-like column tiling, 72 q
    (64, 2, 2, 1, (1, 1, 1), 5.0),       # single point
    (65, 7, 3, 1, (2, 7, 5), 0.7),
])
def test_windows_and_ragged_meshes(lib, seed, nW, nat, r, mesh, half):
    s = synth.small_system(seed, n_wannier=nW, n_atoms=nat, r=r)
    s.h_r *= 0.3
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - half,
               win_hi=mu + half, omega_min=1e-4)
    ref = rates.scattering_rates(s, mesh, tables=t, **par)
    n, g, m, kept = _gpu_rates(lib, s, mesh, par)
    _check(n, g, m, kept, ref)


def test_empty_window(lib, toy):
    s, mesh, par, ref = toy
    p = dict(par, win_lo=100.0, win_hi=101.0)
    n, g, m, kept = _gpu_rates(lib, s, mesh, p)
    assert n == 0


def test_explicit_k_and_weighted_q_lists(lib, toy):
    s, mesh, par, _ = toy
    rng = np.random.default_rng(3)
    k_idx = np.array([5, 0, 215, 77], dtype=np.int64)
    lens = [1, 100, 216, 17]
    q_idx = np.concatenate([rng.integers(0, 216, size=L) for L in lens])
    q_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    q_w = rng.uniform(0.0, 0.01, size=q_idx.size)
    ref = rates.scattering_rates(s, mesh, k_idx=k_idx, q_lists=(q_off, q_idx, q_w), **par)
    n, g, m, kept = _gpu_rates(lib, s, mesh, par, k_idx=k_idx, q_lists=(q_off, q_idx, q_w))
    _check(n, g, m, kept, ref)


def test_argument_errors(lib, toy):
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem, PhoebeError
    s, mesh, par, _ = toy
    ds = DeviceSystem.from_host(s)
    gamma = torch.empty((216, 4), dtype=torch.float64, device="cuda")
    for bad, status in [(dict(par, sigma=0.0), -1), (dict(par, kT=-1.0), -1)]:
        with pytest.raises(PhoebeError) as e:
            lib.scatter_rates(ds, mesh, bad, gamma)
        assert e.value.status == status
    with pytest.raises(PhoebeError) as e:
        lib.scatter_rates(ds, (0, 2, 2), par, gamma)
    assert e.value.status == -1
    # precision enum out of range, through the raw C ABI
    import ctypes
    from paper_2111_14999_amd import binding
    c = ds.c_struct()
    m = (ctypes.c_int32 * 3)(*mesh)
    p = binding.rate_params(par)
    st = lib.lib.phoebe_gpu_scatter_rates(lib.handle, ctypes.byref(c), m, m, None, 0, None, None,
                                          None, ctypes.byref(p), 7, gamma.data_ptr(), None, None,
                                          None, None)
    assert st == -1
    # smearing enum out of range; adaptive scale <= 0; a q mesh other than the k mesh
    with pytest.raises(PhoebeError) as e:
        lib.scatter_rates(ds, mesh, dict(par, smearing="adaptive", adaptive_scale=0.0), gamma)
    assert e.value.status == -1
    p.smearing = 5
    st = lib.lib.phoebe_gpu_scatter_rates(lib.handle, ctypes.byref(c), m, m, None, 0, None, None,
                                          None, ctypes.byref(p), 0, gamma.data_ptr(), None, None,
                                          None, None)
    assert st == -1
    with pytest.raises(PhoebeError) as e:
        lib.scatter_rates(ds, mesh, par, gamma, q_mesh=(mesh[0] * 2, mesh[1], mesh[2]))
    assert e.value.status == -4
    # the extensions are FP64 only
    with pytest.raises(PhoebeError) as e:
        lib.scatter_rates(ds, mesh, dict(par, smearing="adaptive"), gamma, precision="fp32")
    assert e.value.status == -4


# ---------------------------------------------------------------------------
# full-mesh sum over Rp: direct contraction vs the per-axis factorised form
# ---------------------------------------------------------------------------

def _sparse_rp(s, seed, keep_frac):
    """The same system with a random subset of its Rp vectors (not a full box)."""
    rng = np.random.default_rng(seed)
    keep = np.sort(rng.choice(len(s.rp), size=max(1, int(keep_frac * len(s.rp))), replace=False))
    s.rp = np.ascontiguousarray(s.rp[keep])
    s.g_rr = np.ascontiguousarray(s.g_rr[:, keep])
    return s


def _sparse_re(s, seed, keep_frac):
    """The same system with a random subset of its Re vectors."""
    rng = np.random.default_rng(seed)
    keep = np.sort(rng.choice(len(s.re), size=max(1, int(keep_frac * len(s.re))), replace=False))
    s.re = np.ascontiguousarray(s.re[keep])
    s.g_rr = np.ascontiguousarray(s.g_rr[keep])
    return s


@pytest.mark.parametrize("case", ["toy", "ragged-5x6x7", "sparse-rp", "sparse-re", "c2-tiling",
                                  "single-line", "nW16-sparse-re", "axis0-70", "rp-box-9",
                                  "18-modes", "30-modes", "nW20-15-modes", "nW32-3-modes",
                                  "nW18-30-modes", "nW17-sparse-rp"])
def test_mesh_sum_forms_match_oracle(lib, toy, case):
    """Both full-mesh forms against the oracle.  "axis0-70", "rp-box-9" and "18-modes"
    take the line kernel's general path: more than 64 points on axis 0 (point lists in
    LDS, two ballot chunks), an Rp box 9 wide (T2 read per K step, three K steps), 18
    modes (twelve column tiles per wave in two-wave work-groups, term items beyond one per
    thread) and 30 modes (sixteen tiles per wave).  The nW > 16
    cases take its two-tiles-per-mode form (columns sa*32 + b): 15 modes (eight tiles
    per wave), 3 modes (two tiles, most of the waves' modes beyond nModes), 30 modes
    (sixteen tiles per wave) and 17 bands with a sparse Rp list (a half-empty second
    tile of every mode)."""
    if case == "toy":
        s, mesh, par, ref = toy
    else:
        if case == "ragged-5x6x7":
            s, mesh = synth.small_system(71, n_wannier=5, n_atoms=2, r=2), (5, 6, 7)
        elif case == "sparse-rp":
            s, mesh = _sparse_rp(synth.small_system(72, n_wannier=4, n_atoms=2, r=2), 5, 0.4), (6, 4, 5)
        elif case == "sparse-re":
            s, mesh = _sparse_re(synth.small_system(75, n_wannier=4, n_atoms=2, r=2), 6, 0.3), (5, 4, 6)
        elif case == "c2-tiling":
            s, mesh = synth.small_system(73, n_wannier=16, n_atoms=5, r=1), (17, 3, 2)
        elif case == "nW16-sparse-re":  # the folded stage 1 over a sparse 5^3 Re box
            s, mesh = _sparse_re(synth.small_system(76, n_wannier=16, n_atoms=1, r=2), 7, 0.4), (6, 3, 4)
        elif case == "axis0-70":
            s, mesh = synth.small_system(78, n_wannier=3, n_atoms=1, r=2), (70, 2, 1)
        elif case == "rp-box-9":
            s = synth.make_system(79, 4, np.zeros((1, 3)), [1.0], r_h=1, r_e=1, r_p=4)
            s, mesh = _sparse_rp(s, 8, 0.2), (4, 3, 2)
            assert int(np.abs(s.rp).max()) == 4  # box width 9
        elif case == "18-modes":
            s, mesh = synth.small_system(80, n_wannier=4, n_atoms=6, r=1), (4, 3, 2)
            assert 3 * s.mass.shape[0] == 18
        elif case == "30-modes":
            s, mesh = synth.small_system(90, n_wannier=4, n_atoms=10, r=1), (3, 2, 3)
        elif case == "nW20-15-modes":
            s, mesh = synth.small_system(86, n_wannier=20, n_atoms=5, r=1), (5, 4, 3)
        elif case == "nW32-3-modes":
            s, mesh = synth.small_system(87, n_wannier=32, n_atoms=1, r=1), (3, 5, 4)
        elif case == "nW18-30-modes":
            s, mesh = synth.small_system(88, n_wannier=18, n_atoms=10, r=1), (3, 2, 3)
        elif case == "nW17-sparse-rp":
            s, mesh = _sparse_rp(synth.small_system(89, n_wannier=17, n_atoms=2, r=2), 9, 0.5), (4, 5, 3)
        else:
            s, mesh = synth.small_system(74, n_wannier=3, n_atoms=1, r=2), (33, 1, 1)
        s.h_r *= 0.3
        t = rates.mesh_tables(s, mesh)
        mu = float(np.median(t["eps"]))
        par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.8,
                   win_hi=mu + 0.8, omega_min=1e-4)
        ref = rates.scattering_rates(s, mesh, tables=t, **par)
    out = {}
    try:
        for mode in ("direct", "factored"):
            lib.set_mesh_sum(mode)
            out[mode] = _gpu_rates(lib, s, mesh, par)
            _check(*out[mode], ref)
    finally:
        lib.set_mesh_sum("auto")
    gd, gf = out["direct"][1], out["factored"][1]
    scale = max(np.max(np.abs(gd)), 1e-300)
    assert np.max(np.abs(gd - gf)) < 1e-12 * scale


@pytest.mark.parametrize("system", ["toy", "nW16"])
def test_mesh_sum_forms_unsorted_k_list(lib, toy, system):
    """Explicit k rows in no particular order over the full q mesh, both forms."""
    if system == "toy":
        s, mesh, par, _ = toy
        k_idx = np.array([77, 5, 215, 0, 100, 3, 36, 37, 180, 1], dtype=np.int64)
    else:
        s, mesh = synth.small_system(77, n_wannier=16, n_atoms=1, r=1), (5, 4, 3)
        s.h_r *= 0.3
        mu = float(np.median(rates.mesh_tables(s, mesh)["eps"]))
        par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.8,
                   win_hi=mu + 0.8, omega_min=1e-4)
        k_idx = np.array([41, 7, 59, 0, 23, 12, 36, 35, 50, 2, 19], dtype=np.int64)
    ref = rates.scattering_rates(s, mesh, k_idx=k_idx, **par)
    out = {}
    try:
        for mode in ("direct", "factored"):
            lib.set_mesh_sum(mode)
            out[mode] = _gpu_rates(lib, s, mesh, par, k_idx=k_idx)
            _check(*out[mode], ref)
    finally:
        lib.set_mesh_sum("auto")


def test_mesh_sum_mode_errors(lib, toy):
    from paper_2111_14999_amd import PhoebeError
    s, mesh, par, _ = toy
    assert lib.lib.phoebe_gpu_set_mesh_sum(lib.handle, 3) == -1
    assert lib.lib.phoebe_gpu_set_mesh_sum(lib.handle, -1) == -1
    # the factorised form needs the full q mesh
    lib.set_mesh_sum("factored")
    try:
        with pytest.raises(PhoebeError) as e:
            _gpu_rates(lib, s, mesh, par, k_idx=[1, 2],
                       q_lists=(np.array([0, 3, 5]), np.array([0, 1, 2, 3, 4]), np.ones(5)))
        assert e.value.status == -4
    finally:
        lib.set_mesh_sum("auto")


def test_table_cache_bitwise_and_keyed():
    """Rates with the table cache on: the second call reuses the tables and gives the
    same bits as a call without the cache; a different kT, mesh or system rebuilds."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem, Library
    lib = Library(0)
    s = synth.small_system(17, n_wannier=5, n_atoms=2, r=1)
    s.h_r *= 0.3
    mesh = (4, 3, 5)
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.8, win_hi=mu + 0.8,
               omega_min=1e-4)
    ds = DeviceSystem.from_host(s)
    N = int(np.prod(mesh))

    def run(p, m=mesh):
        g = torch.zeros((int(np.prod(m)), s.n_wannier), dtype=torch.float64, device="cuda")
        n = lib.scatter_rates(ds, m, p, g)
        torch.cuda.synchronize()
        return g.cpu().numpy()[:n]

    ref = run(par)
    par2 = dict(par, kT=constants.kT_of(400.0))
    ref2 = run(par2)
    ref3 = run(par, (3, 3, 3))
    lib.set_table_cache(True)
    for _ in range(2):  # build, then reuse
        assert np.array_equal(run(par), ref)
    assert np.array_equal(run(par2), ref2)        # kT changed: rebuilt
    assert np.array_equal(run(par, (3, 3, 3)), ref3)
    assert np.array_equal(run(par), ref)
    lib.set_table_cache(False)
    assert np.array_equal(run(par), ref)
    o = rates.scattering_rates(s, mesh, tables=t, **par)
    assert np.max(np.abs(ref - o["gamma"])) < 1e-9 * np.max(o["gamma"])
    lib.close()


def test_injected_device_error_and_recovery():
    """A HIP failure inside the rate call (forced from the host: the n-th checked HIP
    call is reported as failed) returns PHOEBE_E_DEVICE with its message; the handle
    then runs the same call to the oracle's result."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem, Library, PhoebeError
    lib = Library(0)
    s = synth.config_c1()
    p = workload_params()["toy"]
    mesh = tuple(p["mesh"])
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    ds = DeviceSystem.from_host(s)
    N = int(np.prod(mesh))
    ref = rates.scattering_rates(s, mesh, **par)
    for at in (1, 3, 10, 40):
        g = torch.zeros((N, s.n_wannier), dtype=torch.float64, device="cuda")
        lib.set_fault_injection(at)
        with pytest.raises(PhoebeError) as e:
            lib.scatter_rates(ds, mesh, par, g)
        assert e.value.status == -3
        assert "(injected)" in str(e.value)
        torch.cuda.synchronize()
        n = lib.scatter_rates(ds, mesh, par, g)   # disarmed after firing once
        torch.cuda.synchronize()
        got = g.cpu().numpy()[:n]
        assert np.max(np.abs(got - ref["gamma"])) < 1e-9 * np.max(ref["gamma"])
    lib.set_fault_injection(10 ** 9)   # armed beyond the call's checks: no effect
    g = torch.zeros((N, s.n_wannier), dtype=torch.float64, device="cuda")
    lib.scatter_rates(ds, mesh, par, g)
    lib.set_fault_injection(0)
    lib.close()


@pytest.mark.parametrize("nW,nat,mesh", [(20, 5, (5, 4, 3)), (32, 1, (3, 5, 4))])
def test_two_tile_modes_fp32_factored(lib, nW, nat, mesh):
    """FP32 form of the factorised sums with two column tiles per mode (16 < nW <= 32)
    against the FP64 oracle at the FP32 bound."""
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem
    s = synth.small_system(90 + nW, n_wannier=nW, n_atoms=nat, r=1)
    s.h_r *= 0.3
    t = rates.mesh_tables(s, mesh)
    mu = float(np.median(t["eps"]))
    par = dict(mu=mu, kT=constants.kT_of(300.0), sigma=0.05, win_lo=mu - 0.8,
               win_hi=mu + 0.8, omega_min=1e-4)
    ref = rates.scattering_rates(s, mesh, tables=t, **par)
    N = int(np.prod(mesh))
    gamma = torch.full((N, nW), -1.0, dtype=torch.float64, device="cuda")
    lib.set_mesh_sum("factored")
    try:
        n = lib.scatter_rates(DeviceSystem.from_host(s), mesh, par, gamma, precision="fp32")
    finally:
        lib.set_mesh_sum("auto")
    torch.cuda.synchronize()
    assert n == len(ref["k_idx"])
    mx, med, _ = rel_err(gamma.cpu().numpy()[:n], ref["gamma"])
    print(f"nW {nW}: FP32 factorised Gamma rel err max {mx:.2e} median {med:.2e}")
    assert mx < 1e-6
