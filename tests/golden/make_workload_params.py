"""Write workload_params.json: chemical potentials and windows of the workloads.

Calls only the oracle (and the seeded input generator); run from the repo root:
    python tests/golden/make_workload_params.py

* toy workload (CsCl, nW=4, 6x6x6): mu at mid-band, 0.5 (min eps + max eps)
  over the mesh; no energy window (every state kept);
* realistic workload (perovskite, nW=16, 40x40x40): window |eps - mu| < 0.3 eV;
  mu found by bisection upward from the band bottom so that 2,850..3,150 k
  points keep a state, then checked to keep every eigenvalue at least 1e-9 eV
  away from both window edges (so window decisions are not rounding-dependent);
* batched workload (32 systems of synth.config_c4_specs): the same rule per
  system with a kept fraction of 2.5..3.5 % of the mesh, sigma 0.01 eV, 300 K.

    python tests/golden/make_workload_params.py [--only toy|realistic|batched]
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import constants, rates  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_params.json")
MARGIN = 1e-9


def _margin(eps, lo, hi):
    return float(min(np.min(np.abs(eps - lo)), np.min(np.abs(eps - hi))))


def toy():
    s = synth.config_c1()
    mesh = (6, 6, 6)
    t = rates.mesh_tables(s, mesh)
    mu = 0.5 * (float(t["eps"].min()) + float(t["eps"].max()))
    return dict(seed=1, mesh=list(mesh), mu=mu, temperature=300.0, kT=constants.kT_of(300.0),
                sigma=0.02, win_lo=-1e30, win_hi=1e30, omega_min=1e-4,
                n_kept=int(np.prod(mesh)), n_states=int(np.prod(mesh)) * s.n_wannier)


def bisect_mu(eps, half, lo_count, hi_count):
    """mu rising from the band bottom until lo_count..hi_count k points keep a state."""

    def count(mu):
        return int(rates.kept_points(rates.window_mask(eps, mu - half, mu + half)).size)

    lo, hi = float(eps.min()) - half, float(eps.min()) + 3.0
    while count(hi) <= hi_count:
        hi += 1.0
    assert count(lo) < lo_count
    mid = lo
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        c = count(mid)
        if lo_count <= c <= hi_count:
            break
        if c < lo_count:
            lo = mid
        else:
            hi = mid
    return mid


def realistic():
    s = synth.config_c2(with_coupling=False)
    mesh = (40, 40, 40)
    t = rates.mesh_tables(s, mesh)
    eps = t["eps"]
    half = 0.3
    mu = bisect_mu(eps, half, 2850, 3150)
    for _ in range(100):
        if _margin(eps, mu - half, mu + half) >= MARGIN:
            break
        mu += 1e-7
    m = rates.window_mask(eps, mu - half, mu + half)
    kept = rates.kept_points(m)
    return dict(seed=2, mesh=list(mesh), mu=mu, temperature=300.0, kT=constants.kT_of(300.0),
                sigma=0.01, win_lo=mu - half, win_hi=mu + half, omega_min=1e-4,
                n_kept=int(kept.size), n_states=int(m.sum()),
                min_margin=_margin(eps, mu - half, mu + half))


def batched():
    out = []
    for spec in synth.config_c4_specs():
        pos, shells = synth.random_structure(spec["seed"], spec["n_atoms"])
        s = synth.make_system(spec["seed"], spec["n_wannier"], pos, shells, r_h=spec["r_h"],
                              r_e=spec["r_g"], r_p=spec["r_g"], with_coupling=False)
        mesh = (spec["mesh"],) * 3
        N = int(np.prod(mesh))
        t = rates.mesh_tables(s, mesh)
        eps = t["eps"]
        half = 0.3
        mu = bisect_mu(eps, half, int(0.025 * N), int(0.035 * N))
        for _ in range(100):
            if _margin(eps, mu - half, mu + half) >= MARGIN:
                break
            mu += 1e-7
        m = rates.window_mask(eps, mu - half, mu + half)
        out.append(dict(spec, mu=mu, temperature=300.0, kT=constants.kT_of(300.0), sigma=0.01,
                        win_lo=mu - half, win_hi=mu + half, omega_min=1e-4,
                        n_kept=int(rates.kept_points(m).size), n_states=int(m.sum()),
                        min_margin=_margin(eps, mu - half, mu + half)))
        print(spec["seed"], out[-1]["n_kept"], out[-1]["n_states"], flush=True)
    return out


if __name__ == "__main__":
    only = sys.argv[sys.argv.index("--only") + 1] if "--only" in sys.argv else None
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    for name, fn in (("toy", toy), ("realistic", realistic), ("batched", batched)):
        if only is None or only == name:
            out[name] = fn()
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
