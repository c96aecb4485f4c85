"""Realistic workload at full size, in the launch configuration bench.py times.

perovskite (15 modes), nW = 16, |Re| = |Rp| = 343, 40^3 k and q mesh, window
+-0.3 eV around the stored chemical potential.  The GPU computes every kept k;
the oracle checks the kept-k list and window masks bit for bit (its band
tables cover the whole mesh) and Gamma on a seeded sample of 16 kept k, each over
the full 64,000-q mesh.  The two forms of the full-mesh sum over Rp (per-axis
factorised, the default here, and the direct contraction) agree at every kept
state, and so do the two forms of the factorised stage 1 (the first Re-axis
intermediate held for every k0 plane of the call, the default with a large
workspace budget, or for the k0 planes of one batch under a smaller budget),
bit for bit, since every state's arithmetic is the same in both.
"""

import numpy as np
import pytest

import synth
from gpu_common import rel_err, torch_cuda, workload_params
from oracle import rates

pytestmark = pytest.mark.gpu


def test_realistic_workload_sampled_parity():
    torch = torch_cuda()
    from paper_2111_14999_amd import DeviceSystem, Library
    p = workload_params()["realistic"]
    mesh = tuple(p["mesh"])
    N = int(np.prod(mesh))
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    s = synth.config_c2()
    print("inputs ready", flush=True)
    lib = Library(0)
    lib.set_timing(True)
    ds = DeviceSystem.from_host(s)
    gamma = torch.zeros((N, 16), dtype=torch.float64, device="cuda")
    mask = torch.zeros((N, 16), dtype=torch.uint8, device="cuda")
    kept = torch.zeros((N,), dtype=torch.int32, device="cuda")
    n = lib.scatter_rates(ds, mesh, par, gamma, band_mask=mask, kept_k_out=kept)
    torch.cuda.synchronize()
    print(f"GPU done: {n} kept k", flush=True)
    assert lib.kernel_time("stage1_planes")[0] == 1  # every k0 plane in one pass
    g = gamma.cpu().numpy()[:n]
    m = mask.cpu().numpy()[:n]
    kidx = kept.cpu().numpy()[:n]
    # the direct contraction over the Rp list gives the same rates at every kept k
    lib.set_mesh_sum("direct")
    gamma.zero_()
    n2 = lib.scatter_rates(ds, mesh, par, gamma)
    torch.cuda.synchronize()
    gd = gamma.cpu().numpy()[:n2]
    assert n2 == n
    sel = g > 0
    dmax = np.max(np.abs(gd[sel] - g[sel]) / g[sel])
    print(f"direct vs factorised sum: max rel diff {dmax:.3e} over {int(sel.sum())} states",
          flush=True)
    assert dmax < 1e-11
    assert np.all(gd[~sel] == 0.0)
    lib.close()
    # a 40 GB workspace budget holds the k0 planes of one batch only
    small = Library(0, workspace_budget=40 * 10**9)
    small.set_timing(True)
    gamma.zero_()
    n3 = small.scatter_rates(ds, mesh, par, gamma)
    torch.cuda.synchronize()
    assert small.kernel_time("stage1_planes")[0] == 0
    assert small.kernel_time("stage1_axes")[0] > 0
    assert n3 == n
    assert np.array_equal(gamma.cpu().numpy()[:n], g)
    print("per-batch and all-plane stage 1 agree bit for bit", flush=True)
    small.close()
    del ds

    tables = rates.mesh_tables(s, mesh)
    mask_all = rates.window_mask(tables["eps"], par["win_lo"], par["win_hi"])
    kref = rates.kept_points(mask_all)
    assert n == p["n_kept"] == len(kref)
    assert np.array_equal(kidx, kref.astype(np.int32))
    assert np.array_equal(m, mask_all[kref])
    assert np.all(g[m == 0] == 0.0)
    assert np.all(g[m == 1] > 0.0)
    sample = np.sort(np.random.default_rng(2024).choice(n, size=16, replace=False))
    ref = rates.scattering_rates(s, mesh, k_idx=kref[sample], tables=tables, **par)
    mx, med, ab = rel_err(g[sample], ref["gamma"])
    print(f"sampled Gamma rel err max {mx:.3e} median {med:.3e}", flush=True)
    assert mx < 1e-9
