"""Benchmark: Gamma_nk k-points/s of the full el-ph rate path on one MI355X.

One step = one phoebe_gpu_scatter_rates call on the realistic workload: band
structure and phonons on the 40^3 mesh, energy window, stage-1 and stage-2
phase sums, rotations and the smeared rate sum for every kept k over the full
40^3 q mesh (inputs resident in HBM).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload realistic|toy]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "el-ph g(k,q) elements/s + Γ_nk k-pts/s at stated err vs FP64 oracle, 1 GPU"
PEAK_FP64_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mesh_points_frac(mesh, idx):
    """Crystal coordinates of mesh points given by linear index (third axis fastest)."""
    idx = np.asarray(idx, dtype=np.int64)
    i2 = idx % mesh[2]
    i1 = (idx // mesh[2]) % mesh[1]
    i0 = idx // (mesh[1] * mesh[2])
    return np.stack([i0 / mesh[0], i1 / mesh[1], i2 / mesh[2]], axis=1)


def load_params(name):
    with open(os.path.join(ROOT, "tests", "golden", "workload_params.json")) as f:
        return json.load(f)[name]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="realistic", choices=["realistic", "toy", "batched"])
    ap.add_argument("--tune-cache", default=None, help="JSON tile cache of the batched form")
    ap.add_argument("--cpu-sample", type=int, default=6, help="kept k points timed on the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--interp-k", type=int, default=2, help="k points of the interp_g rate run")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the rate sum shards over kept k points without collectives).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2111_14999_amd import DeviceSystem, Library

    if args.workload == "batched":
        return bench_batched(args)
    p = load_params(args.workload)
    mesh = tuple(p["mesh"])
    N = int(np.prod(mesh))
    par = dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"], win_hi=p["win_hi"],
               omega_min=p["omega_min"])
    t0 = time.perf_counter()
    s = synth.config_c2() if args.workload == "realistic" else synth.config_c1()
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s (g(Re,Rp) {s.g_rr.nbytes / 1e9:.2f} GB)")
    ds = DeviceSystem.from_host(s)
    torch.cuda.synchronize()
    lib = Library(0)
    nW, nm, n_rp = s.n_wannier, s.n_modes, s.rp.shape[0]
    gamma = torch.zeros((N, nW), dtype=torch.float64, device="cuda")
    mask = torch.zeros((N, nW), dtype=torch.uint8, device="cuda")
    kept = torch.zeros((N,), dtype=torch.int32, device="cuda")

    def step():
        return lib.scatter_rates(ds, mesh, par, gamma, band_mask=mask, kept_k_out=kept,
                                 precision=args.precision)

    for i in range(args.warmup):
        n_kept = step()
        torch.cuda.synchronize()
        log(f"warmup {i} done, {n_kept} kept k")
    lib.set_timing(True)
    lib.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        n_kept = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    lib.set_timing(False)
    log(f"{args.steps} timed steps, {dt * 1e3:.1f} ms/step")
    n_st2, ms_st2 = lib.kernel_time("stage2_rates")
    n_st1, ms_st1 = lib.kernel_time("stage1_phase")
    g = gamma.cpu().numpy()[:n_kept]
    m = mask.cpu().numpy()[:n_kept]
    kidx = kept.cpu().numpy()[:n_kept]
    n_states = int(m.sum())

    # algorithmic FP64 flops of the dominant kernel (the Rp phase sum, 8 flops per
    # complex multiply-add; rotation and rate terms not counted) per step
    flops_st2 = 8.0 * n_states * N * n_rp * nm * nW
    avg_ms = ms_st2 / max(n_st2, 1)
    launches_per_step = n_st2 / args.steps
    achieved = flops_st2 / launches_per_step / (avg_ms * 1e-3) / 1e12 if n_st2 else 0.0
    # peak of the MFMA the form runs on; split-BF16 executes 3 or 6 BF16 products per
    # real product, so its complex-GEMM flops are measured against BF16 peak / products
    peak = {"fp64": PEAK_FP64_TFLOPS, "fp32": 157.3, "bf16x3": 2500.0 / 3,
            "bf16x6": 2500.0 / 6}[args.precision]
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=round(peak, 2),
                    unit="TFLOP/s", frac=round(achieved / peak, 4), traffic=None,
                    kernel="stage2_rates", launches_per_step=launches_per_step,
                    avg_launch_ms=round(avg_ms, 4),
                    flops_per_launch=flops_st2 / max(launches_per_step, 1))
    log(f"stage2: {n_st2} launches, avg {avg_ms:.3f} ms, {achieved:.2f} TFLOP/s; "
        f"stage1: {n_st1} launches, {ms_st1 / max(args.steps, 1):.1f} ms/step")

    # interp_g element rate (all (nu, n, m) of nk kept k x the full q mesh)
    gel = None
    if args.interp_k > 0 and n_kept > 0:
        kf = torch.from_numpy(mesh_points_frac(mesh, kidx[:args.interp_k])).cuda()
        qf = torch.from_numpy(mesh_points_frac(mesh, np.arange(N))).cuda()
        nk_i = kf.shape[0]
        gout = torch.empty((nk_i, N, nm, nW, nW), dtype=torch.complex128, device="cuda")
        lib.interp_g(ds, kf, qf, gout, omega_min=par["omega_min"], precision=args.precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.interp_g(ds, kf, qf, gout, omega_min=par["omega_min"], precision=args.precision)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t1
        gel = nk_i * N * nm * nW * nW / ti
        del gout
        log(f"interp_g: {nk_i} k x {N} q in {ti * 1e3:.1f} ms = {gel:.3e} elements/s")

    # oracle on a bounded sample: error of the GPU result and the CPU baseline rate
    err = None
    cpu = None
    if not args.no_cpu_baseline and n_kept > 0:
        from oracle import rates
        rng = np.random.default_rng(12345)
        sample = np.sort(rng.choice(n_kept, size=min(args.cpu_sample, n_kept), replace=False))
        t1 = time.perf_counter()
        tables = rates.mesh_tables(s, mesh)
        t_tab = time.perf_counter() - t1
        t1 = time.perf_counter()
        ref = rates.scattering_rates(s, mesh, k_idx=kidx[sample], tables=tables, **par)
        t_k = time.perf_counter() - t1
        per_k = t_k / len(sample) + t_tab / n_kept
        cpu = dict(value=round(1.0 / per_k, 4), unit="k-pts/s", cores=os.cpu_count(),
                   kind="oracle",
                   sample=f"{len(sample)} seeded kept k of {n_kept} over the full {N}-q mesh "
                          f"({t_k:.1f} s) + band/phonon tables on the mesh ({t_tab:.1f} s) "
                          f"pro-rated per kept k; NumPy/OpenBLAS threads = host cores")
        got = g[sample]
        rm = ref["gamma"]
        sel = rm > 1e-10 * rm.max()
        rel = np.abs(got[sel] - rm[sel]) / rm[sel]
        err = dict(max_rel=float(rel.max()), median_rel=float(np.median(rel)),
                   states=int(sel.sum()), sample=f"{len(sample)} kept k")
        log(f"oracle sample: max rel err {rel.max():.3e}, cpu {cpu['value']} k-pts/s")

    out = {
        "metric": METRIC,
        "value": round(n_kept / dt, 3),
        "unit": "k-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32acc",
                  "bf16x6": "bf16x6+f32acc"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {s.n_atoms} atoms ({nm} modes), nW={nW}, "
                         f"|Re|=|Rp|={n_rp}, k and q mesh {mesh[0]}x{mesh[1]}x{mesh[2]}, "
                         f"window ({par['win_lo']:.4f}, {par['win_hi']:.4f}) eV -> {n_kept} kept k, "
                         f"{n_states} states, sigma {par['sigma']} eV, kT {par['kT']:.6f} eV"),
            "kept_k": n_kept, "states": n_states, "q_points": N,
        },
        "g_elements_per_s": gel,
        "err_vs_oracle": err,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    lib.close()


def bench_batched(args):
    """32 independent systems in one captured graph (persistent multi-system kernel)."""
    import tempfile

    import torch

    import synth
    from paper_2111_14999_amd import DeviceSystem, Library

    plist = load_params("batched")
    t0 = time.perf_counter()
    systems, dsys, meshes, pars = [], [], [], []
    for p in plist:
        s = synth.config_c4(p)
        systems.append(s)
        dsys.append(DeviceSystem.from_host(s))
        s.g_rr = None  # host copy no longer needed
        meshes.append((p["mesh"],) * 3)
        pars.append(dict(mu=p["mu"], kT=p["kT"], sigma=p["sigma"], win_lo=p["win_lo"],
                         win_hi=p["win_hi"], omega_min=p["omega_min"]))
    torch.cuda.synchronize()
    log(f"{len(plist)} systems generated and uploaded in {time.perf_counter() - t0:.1f} s")
    lib = Library(0)
    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(), "tiles.json")
    t0 = time.perf_counter()
    plan = lib.batched_plan(dsys, meshes, pars, precision="fp32", tune_cache=cache)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    info = [plan.info(i) for i in range(len(plist))]
    log(f"plan (tables, windows, autotune {info[0]['tune_ms']:.0f} ms, capture) in {t_plan:.1f} s; "
        f"{info[0]['tasks']} queue tasks")
    outs = [torch.zeros((max(n, 1), s.n_wannier), dtype=torch.float64, device="cuda")
            for n, s in zip(plan.n_kept, systems)]
    for _ in range(args.warmup):
        plan.run(outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(outs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n_kept = sum(plan.n_kept)
    flops = 0.0
    for p, s, inf in zip(plist, systems, info):
        flops += 8.0 * inf["states"] * p["mesh"] ** 3 * s.rp.shape[0] * s.n_modes * s.n_wannier
    log(f"graph replay {dt * 1e3:.1f} ms: {n_kept / dt:.1f} kept k/s, "
        f"{flops / dt / 1e12:.1f} TFLOP/s (stage-2 algorithmic, whole graph)")
    err = None
    if not args.no_cpu_baseline:
        from oracle import rates
        rels = []
        for i in (0, len(plist) // 2):
            if plan.n_kept[i] == 0:
                continue
            s = synth.config_c4(plist[i])
            tabs = rates.mesh_tables(s, meshes[i])
            kept = rates.kept_points(rates.window_mask(tabs["eps"], pars[i]["win_lo"],
                                                       pars[i]["win_hi"]))
            ref = rates.scattering_rates(s, meshes[i], k_idx=kept[:1], tables=tabs, **pars[i])
            got = outs[i].cpu().numpy()[:1]
            sel = ref["gamma"] > 1e-10 * ref["gamma"].max()
            rels.extend((np.abs(got[sel] - ref["gamma"][sel]) / ref["gamma"][sel]).tolist())
        if rels:
            err = dict(max_rel=float(np.max(rels)), median_rel=float(np.median(rels)),
                       sample="first kept k of systems 0 and 16")
            log(f"oracle sample: max rel err {err['max_rel']:.3e}")
    tiles = {}
    for inf in info:
        key = f"tq{inf['tq']}_tn{inf['tn']}"
        tiles[key] = tiles.get(key, 0) + 1
    out = {
        "metric": METRIC,
        "value": round(n_kept / dt, 3),
        "unit": "k-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched: {len(plist)} systems, nW 4..24, nModes 6..30, |R| 125..729, "
                         f"meshes 16^3..32^3, +-0.3 eV windows, one captured graph with the "
                         f"persistent multi-system kernel (complex64 contractions)"),
            "kept_k": n_kept, "plan_s": round(t_plan, 2), "tiles": tiles,
        },
        "stage2_tflops_whole_graph": round(flops / dt / 1e12, 3),
        "err_vs_oracle": err,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    lib.close()


if __name__ == "__main__":
    main()
