"""Benchmark of the improved MRT pseudopotential D2Q9 step on one MI355X.

Workload: droplet splashing on a thin film, 8192 x 4096 lattice (the 2048 x 1024
splash geometry scaled by 4: R = 400, film 80, gap 20), x periodic, halfway
bounce-back walls in y, Carnahan-Starling a = 0.25, T = 0.45 T_c, sigma = 0.114,
s_e = s_zeta = 0.8, s_q = 1.1, U = 0.05, nu_l = 0.05, nu_g = 0.75.  Synthetic,
seedless (the initial field is a deterministic tanh profile).

One "step" is one full time step over the lattice (pull streaming, density, psi,
force, MRT collision with the improved forcing, store).  The metric is MLUPS
(million lattice-site updates per second) with the distributions resident in HBM.

    python bench.py [--steps K] [--warmup W] [--store f32|f16|bf16|f16local|bf16local|f16dest] [--no-cpu-baseline]
    python bench.py --workload batch [--instances 512] [--steps 10000] [--store f32|f16dest|f16local]
    python bench.py --workload learned [--train-runs 4096] [--eval-droplets 256] [--relax-steps 30000]
    python bench.py --workload splash1k  (2048x1024 splash, Re 40/200/1000, 20,000 steps: stability, mass)
    python bench.py --workload lamb      (droplet oscillation against Lamb, Sec. IV.A)
    python bench.py --workload sweeps    (coexistence curves, stability edges, Table I, Fig. 4)
    python bench.py --workload spread    (splash spread radius and Weber number, Sec. IV.C)
    python bench.py --workload precision (every storage encoding's speed against the same run's FP32)

The batch workload advances 512 independent droplet lattices (seed 1211: sides 64-512,
a in {0.25, 0.5, 1}, T/Tc in [0.5, 0.85], half of them elliptic): strip heights are
autotuned on the device, then 10,000 steps in captured stepwise launches give the
aggregate MLUPS, and 10,000 more in the persistent launch (one workgroup per lattice)
give the p50 / p99 per-lattice completion times.

The learned workload runs the droplet-initialiser protocol: 4096 tanh-started
droplets on 256 x 256 lattices (seed 1212) relax for 30,000 steps; the network
trains on their least-squares profiles on the device and the FP64 level model on
their interior levels; 256 held-out droplets (seed 1213) start from tanh, from the
anchored prediction and from the network alone, and run 30,000 steps together.
The value is the median per-droplet ratio of steps to convergence (tanh / learned),
convergence meaning max|u| within 5 % and the pressure jump within 1 % of the tanh
run's final values; the max|u|-only ratio, the network-only arm and the final-state
errors are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BYTES_PER_SITE = {"f32": 72, "f16": 36, "bf16": 36, "f16local": 44, "bf16local": 44, "f16dest": 40}
PEAK_HBM_GBPS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(store, nsites):
    """HBM bytes per step launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), if it was taken on the current
    kernel source and workload size (else None)."""
    from paper_1211_6932_amd.prof import kernel_hash

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = doc.get(store)
    if not ent or ent.get("kernel_sha") != kernel_hash() or ent.get("sites") != nsites:
        return None
    return ent.get("bytes_per_launch")


def copy_probe_gbps(torch, lbmp, stream, nbytes=1 << 30, reps=20):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        lbmp.lb_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbmp.lb_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle as it stands, on the same workload, timed on the host cores."""
    import numpy as np
    from oracle import lbref as O

    p = O.Params(**w.params)
    rho0 = np.asarray(w.rho0, dtype=np.float32).astype(np.float64)
    ux0 = np.asarray(w.ux0, dtype=np.float32).astype(np.float64)
    uy0 = np.asarray(w.uy0, dtype=np.float32).astype(np.float64)
    st = O.State(p, rho0, ux0, uy0)
    t0 = time.perf_counter()
    st.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(20, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    st.step(n)
    dt = time.perf_counter() - t0
    sites = w.params["nx"] * w.params["ny"]
    return {
        "value": sites * n / dt / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
        "sample": f"{n} FP64 steps of the full {w.params['nx']}x{w.params['ny']} workload "
                  f"(after 1 untimed step), {dt:.1f} s",
    }


def bench_batch(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp

    torch.cuda.set_device(0)
    lbmp.load()
    ws = W.batch_instances(args.instances, seed=1211)
    sites = sum(w.params["nx"] * w.params["ny"] for w in ws)
    log(f"batch of {len(ws)} lattices, {sites} sites: init")
    b = lbmp.Batch([w.params for w in ws], [torch.from_numpy(np.asarray(w.rho0, np.float32)) for w in ws],
                   store=args.store)
    b.set_launch(lbmp.LB_BATCH_STEPWISE)
    t0 = time.perf_counter()
    rows = b.tune(trial_steps=8) if not args.no_tune else None
    t_tune = time.perf_counter() - t0
    if rows is not None:
        log(f"tuned strip heights in {t_tune:.2f} s: " +
            ", ".join(f"{r} rows x {rows.count(r)}" for r in sorted(set(rows))))
    b.step(args.warmup)
    b.stream.synchronize()
    log(f"timed {args.steps} steps (stepwise)")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.step(args.steps)
    ev1.record(b.stream)
    b.stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = ev0.elapsed_time(ev1) / args.steps
    mlups = sites * args.steps / wall / 1e6
    bps = BYTES_PER_SITE[args.store]
    achieved = bps * sites / (step_ms * 1e-3) / 1e9
    log(f"{mlups:.0f} MLUPS aggregate, {wall:.2f} s, {step_ms:.4f} ms per step (events)")
    copy_gbps = None
    if not args.no_copy_probe:
        copy_gbps = copy_probe_gbps(torch, lbmp, b.stream)
        log(f"copy probe {copy_gbps:.0f} GB/s")
    per_lattice = None
    if not args.no_persistent:
        # per-lattice completion times: the persistent launch gives each lattice its own
        # workgroup for all steps (the stepwise launches finish every lattice together)
        b.set_launch(lbmp.LB_BATCH_PERSISTENT)
        log(f"timed {args.steps} steps (persistent, per-lattice completion times)")
        t0 = time.perf_counter()
        b.step(args.steps)
        b.stream.synchronize()
        pwall = time.perf_counter() - t0
        times = np.array(b.times())
        per_lattice = {"mode": "persistent", "steps": args.steps, "aggregate_MLUPS": round(sites * args.steps / pwall / 1e6, 1),
                       "p50_s": round(float(np.percentile(times, 50)), 4),
                       "p99_s": round(float(np.percentile(times, 99)), 4),
                       "min_s": round(float(times.min()), 4), "max_s": round(float(times.max()), 4)}
        log(f"persistent: {per_lattice['aggregate_MLUPS']:.0f} MLUPS, p50 {per_lattice['p50_s']:.2f} s, "
            f"p99 {per_lattice['p99_s']:.2f} s")
    unstable = [b.diagnostics(i, 0.0, 0.0, 1.0, 2.0, raise_unstable=False)["unstable"] for i in range(len(ws))]
    n_unstable = sum(1 for u in unstable if u)
    out = {
        "metric": "aggregate MLUPS of a batched multi-lattice sweep (D2Q9 MRT improved pseudopotential)",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.store == "f32" else f"{args.store} storage, f32 compute",
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} periodic droplet lattices (seed 1211), sides 64-512, "
                               f"{sites} sites", "batch_mode": "stepwise", "store": args.store,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None, "bytes_per_site": bps,
                     "step_ms_events": round(step_ms, 5),
                     "copy_probe_GBps": None if copy_gbps is None else round(copy_gbps, 1)},
        "per_lattice_stepwise": {"p50_s": round(wall, 4), "p99_s": round(wall, 4),
                                 "note": "every lattice completes with the last launch"},
        "per_lattice_persistent": per_lattice,
        "tuning": None if rows is None else {"seconds": round(t_tune, 3),
                                             "rows_histogram": {str(r): rows.count(r) for r in sorted(set(rows))}},
        "checks": {"unstable_lattices": int(n_unstable),
                   "unstable": [dict(i=i, side=ws[i].params["nx"], a=ws[i].params["a"],
                                     t_over_tc=round(ws[i].info["t_over_tc"], 3), R0=round(ws[i].info["R0"], 1))
                                for i in range(len(ws)) if unstable[i]]},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_splash1k(args):
    """The splash case at its own size and length: 2048 x 1024, walls in y, x periodic,
    a = 0.25, T = 0.45 T_c (liquid/vapour density ratio about 2400), R = 100, film 20,
    U = 0.05, nu_g = 15 nu_l, Re = U D / nu_l in {40, 200, 1000}, 20,000 steps (Ut/D = 5).
    Records, per Re, whether the run stays stable (the first step that flags an unstable
    site otherwise, to the checking interval), the FP64 mass drift, max|u| and the
    spread of the droplet over the film."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp

    torch.cuda.set_device(0)
    lbmp.load()
    steps = args.steps
    every = 10
    runs = {}
    t_all = time.perf_counter()
    for Re in (40, 200, 1000):
        w = W.splash(scale=1, Re=Re)
        nx, ny = w.params["nx"], w.params["ny"]
        sim = lbmp.Sim(w.params, torch.from_numpy(np.asarray(w.rho0, np.float32)),
                       torch.from_numpy(np.asarray(w.ux0, np.float32)),
                       torch.from_numpy(np.asarray(w.uy0, np.float32)))
        c = (nx / 2.0, w.info["film"] + w.info["R"] + 5.0)
        d0 = sim.diagnostics(c[0], c[1], 1.0, 2.0)
        first_bad, umax, drift_max = None, d0["max_u"], 0.0
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(every, steps - done)
            sim.step(n)
            done += n
            if lbmp.lb_check(sim.ctx) != lbmp.LB_OK:
                first_bad = done
                break
            if done % 1000 == 0:
                d = sim.diagnostics(c[0], c[1], 1.0, 2.0)
                umax = max(umax, d["max_u"])
                drift_max = max(drift_max, abs(d["mass"] / d0["mass"] - 1.0))
        wall = time.perf_counter() - t0
        res = {"nu_l": w.params["nu_l"], "nu_g": w.params["nu_g"], "stable": first_bad is None,
               "first_unstable_step": first_bad, "steps_run": done, "wall_s": round(wall, 2),
               "MLUPS_with_checks": round(nx * ny * done / wall / 1e6, 1)}
        if first_bad is None:
            d1 = sim.diagnostics(c[0], c[1], 1.0, 2.0)
            rho = sim.moments()[0].cpu().numpy()
            film = w.info["film"]
            # liquid half-width on the row just above the undisturbed film surface
            row = rho[int(film) + 1]
            liquid = np.nonzero(row > 0.5 * (w.info["rho_l"] + w.info["rho_g"]))[0]
            res.update(mass_rel_drift_final=(d1["mass"] - d0["mass"]) / d0["mass"],
                       mass_rel_drift_max=max(drift_max, abs(d1["mass"] / d0["mass"] - 1.0)),
                       max_u_final=d1["max_u"], max_u_seen=max(umax, d1["max_u"]),
                       liquid_width_above_film=int(liquid.size), rho_min=float(rho.min()), rho_max=float(rho.max()))
        runs[str(Re)] = res
        log(f"Re={Re}: " + json.dumps(res))
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out = {
        "metric": "stability and mass conservation of the 2048x1024 splash over 20,000 steps, Re = 40, 200, 1000",
        "value": sum(1 for r in runs.values() if r["stable"]), "unit": "stable runs of 3", "n_gpus": 1,
        "steps": steps, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "droplet splash on a thin film, 2048x1024, walls in y, x periodic, a=0.25, "
                               "T=0.45Tc, sigma=0.114, s_e=s_zeta=0.8, U=0.05, R=100, film 20, nu_g=15 nu_l",
                   "parallelism": "single GPU"},
        "runs": runs, "wall_seconds": round(time.perf_counter() - t_all, 2), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """Every storage encoding on the 8192x4096 splash in one process: MLUPS, step-kernel
    time (HIP events on the library stream) and the speed ratio to the same run's FP32
    step.  The error of each encoding against the FP64 oracle is a GPU test."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp

    torch.cuda.set_device(0)
    lbmp.load()
    w = W.splash(scale=args.scale, Re=200)
    nx, ny = w.params["nx"], w.params["ny"]
    sites = nx * ny
    f = lambda a: torch.from_numpy(np.asarray(a, np.float32))
    res = {}
    for store in ("f32", "f16dest", "f16local", "f16", "bf16local", "bf16"):
        rho_ref = w.info["rho_l"] if store in ("f16", "bf16") else 0.0
        sim = lbmp.Sim(w.params, f(w.rho0), f(w.ux0), f(w.uy0), store=store, rho_ref=rho_ref)
        sim.step(args.warmup)
        sim.stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(sim.stream)
        sim.step(args.steps)
        e1.record(sim.stream)
        sim.stream.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = e0.elapsed_time(e1) / args.steps
        stable = lbmp.lb_check(sim.ctx) == lbmp.LB_OK
        sim.close()
        del sim
        torch.cuda.empty_cache()
        bps = BYTES_PER_SITE[store]
        res[store] = {"MLUPS": round(sites * args.steps / wall / 1e6, 1), "kernel_ms": round(kern_ms, 5),
                      "bytes_per_site": bps,
                      "hbm_frac": round(bps * sites / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                      "stable": bool(stable)}
        log(f"{store}: {res[store]['MLUPS']:.0f} MLUPS, step {kern_ms:.4f} ms")
    for store, r in res.items():
        r["vs_f32"] = round(r["MLUPS"] / res["f32"]["MLUPS"], 3)
    out = {
        "metric": "MLUPS of destination-scaled FP16 storage over the same run's FP32 step",
        "value": res["f16dest"]["vs_f32"], "unit": "x", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "16-bit storage, f32 compute", "data": "synthetic",
        "config": {"workload": f"droplet splash on a thin film, {nx}x{ny}, walls in y, x periodic, a=0.25, "
                               "T=0.45Tc, Re=200, every storage encoding", "parallelism": "single GPU"},
        "stores": res,
        "roofline": {"bound": "hbm", "achieved": round(40 * sites / (res["f16dest"]["kernel_ms"] * 1e-3) / 1e9, 1),
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": res["f16dest"]["hbm_frac"], "traffic": None,
                     "kernel": "f16dest step (40 B/site)"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_learned(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import initialiser as I
    from paper_1211_6932_amd import lbmp

    torch.cuda.set_device(0)
    lbmp.load()
    train_ws = W.learned_train_instances(n=args.train_runs, side_lo=256, side_hi=256)
    sites = sum(w.params["nx"] * w.params["ny"] for w in train_ws)
    t0 = time.perf_counter()
    X, base, T, kept = I.generate(train_ws, args.relax_steps, every=1000, log=log)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    model, losses = I.train(X, base, T, steps=args.train_steps, log=log)
    t_train = time.perf_counter() - t0
    eval_ws = W.learned_eval_instances(n=args.eval_droplets, side=256)
    t0 = time.perf_counter()
    res, _ = I.evaluate(model, eval_ws, steps=args.relax_steps, every=50, log=log, ablation=True)
    t_eval = time.perf_counter() - t0
    model.close()
    u, strict = res["summary"]["u"], res["summary"]["strict"]
    gen_gbps = BYTES_PER_SITE["f32"] * sites * args.relax_steps / t_gen / 1e9
    out = {
        "metric": "steps to convergence (max|u| within 5 % and pressure jump within 1 % of the tanh run's "
                  "final values), tanh start / learned start, median per droplet",
        "value": round(strict.get("median_ratio", float("nan")), 3), "unit": "x", "n_gpus": 1,
        "steps": args.relax_steps, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 network (f32 accumulate), f32 lattice",
        "data": "synthetic",
        "config": {"workload": f"learned droplet initialiser: {args.train_runs} training runs and "
                               f"{args.eval_droplets} held-out droplets on 256x256, {args.relax_steps} steps",
                   "parallelism": "single GPU"},
        "strict": strict, "ratio_of_medians": round(strict.get("ratio_of_medians", float("nan")), 3),
        "spurious_current_only": u, "network_only": res["network_only"],
        "wall_seconds": {"training_runs": round(t_gen, 2), "training": round(t_train, 2),
                         "inference_and_placement": round(res["infer_seconds"], 3),
                         "evaluation_runs": round(t_eval, 2)},
        "training": {"profiles": int(X.shape[0]), "dropped_unstable": int((~kept).sum()),
                     "final_loss": losses[-1][1], "steps": args.train_steps},
        "roofline": {"bound": "hbm", "achieved": round(gen_gbps, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(gen_gbps / PEAK_HBM_GBPS, 4), "traffic": None,
                     "kernel": "batched lattice step during the training runs (72 B/site)"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_sweeps(args):
    import json as _json

    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp
    from paper_1211_6932_amd import sweeps as S

    torch.cuda.set_device(0)
    lbmp.load()
    golden = _json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    t0 = time.perf_counter()
    improved_T = [0.49, 0.5, 0.55, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95]
    edge_T = [round(0.76 + 0.0025 * i, 4) for i in range(29)]
    groups = {"improved_0.8": W.coexistence_droplets(improved_T, tau_nu=0.8),
              "original_0.6": W.coexistence_droplets(edge_T, sigma=0.0, tau_nu=0.6),
              "original_0.8": W.coexistence_droplets(edge_T, sigma=0.0, tau_nu=0.8),
              "table1": [w for a in (1.0, 0.5, 0.25) for w in W.coexistence_droplets([0.5, 0.55], tau_nu=0.8, a=a)]}
    ws = [w for g in groups.values() for w in g]
    res, k, out_groups = S.droplet_sweep(ws, log=log), 0, {}
    for name, g in groups.items():
        out_groups[name] = res[k:k + len(g)]
        k += len(g)
    t_sweep = time.perf_counter() - t0
    curve = [{"T_over_Tc": r["t_over_tc"], "rho_l": r["rho_l"], "rho_g": r["rho_g"],
              "maxwell": W.coexistence(r["t_over_tc"])} for r in out_groups["improved_0.8"]]
    edges = {}
    for tau in ("0.6", "0.8"):
        rows = out_groups[f"original_{tau}"]
        t_low = S.lowest_stable(rows)
        edges[tau] = {"lowest_T_over_Tc": t_low,
                      "ratio": [r["ratio"] for r in rows if r["t_over_tc"] == t_low][0]}
    table1 = [{"a": r["a"], "T_over_Tc": r["t_over_tc"], "max_u": r["max_u"]} for r in out_groups["table1"]]
    nus = [float(v) for v in np.geomspace(0.001, 0.2, 24)]
    ratios = (1, 20, 50)
    t1 = time.perf_counter()
    failed, failed_u = S.survival([W.paper_splash(nu, r) for r in ratios for nu in nus], 4000)
    t_visc = time.perf_counter() - t1
    visc = {str(r): S.lowest_stable_viscosity(nus, failed[i * len(nus):(i + 1) * len(nus)])
            for i, r in enumerate(ratios)}
    visc_u = {str(r): S.lowest_stable_viscosity(nus, failed_u[i * len(nus):(i + 1) * len(nus)])
              for i, r in enumerate(ratios)}
    t2 = {row[0]: row for row in golden["table2"]["rows"]}
    by_t = {c["T_over_Tc"]: c for c in curve}
    worst_l = max(abs(by_t[t]["rho_l"] / t2[t][1] - 1) for t in t2)
    out = {
        "metric": "coexistence densities vs Table II (max relative error, liquid, tau_nu = 0.8)",
        "value": round(worst_l, 5), "unit": "fraction", "n_gpus": 1, "steps": 40000, "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} droplets 200x200 R=50 (Sec. IV.A/B) + 36 splash runs 600x250 "
                               "(Sec. IV.C), one batched launch each", "parallelism": "single GPU"},
        "improved_curve_tau0.8": curve, "original_edge": edges,
        "paper_original_edge": {"T_over_Tc": 0.8, "ratio_tau0.6": 30.0, "ratio_tau0.8": 56.5},
        "table1": table1, "lowest_nu_l": visc, "lowest_nu_l_max_u_below_cs": visc_u,
        "viscosity_grid": nus, "paper_lowest_nu_l": {"1": 0.075, "20": 0.009, "50": 0.0039},
        "wall_seconds": {"droplet_sweep": round(t_sweep, 2), "viscosity_search": round(t_visc, 2)},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_spread(args):
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp
    from paper_1211_6932_amd import validation as V

    torch.cuda.set_device(0)
    lbmp.load()
    t0 = time.perf_counter()
    runs = {}
    for Re, ratio in ((40, 1.0), (100, 1.0), (1000, 15.0)):
        w = W.paper_splash(0.125 * 100 / Re, ratio)
        sp = V.splash_spread(w, t_end_star=2.0, log=log)
        t, r = sp["t_star"], sp["r_over_D"]
        runs[str(Re)] = {"nu_g_over_nu_l": ratio,
                         "C_short": round(V.power_law_coefficient(t, r, 0.02, 0.2), 4),
                         "C_0.5_1.5": round(V.power_law_coefficient(t, r, 0.5, 1.5), 4),
                         "r_over_D": {f"{x:.2f}": round(float(r[abs(t - x).argmin()]), 4)
                                      for x in (0.05, 0.1, 0.2, 0.4, 0.7, 1.0, 1.5, 1.9)}}
    st = V.surface_tension(W.laplace_droplets(radii=(30.0, 40.0, 50.0), n=256, t_over_tc=0.5, a=0.25), log=log)
    p50 = [p for p in st["points"] if p["R0"] == 50.0][0]
    we = p50["rho_in"] * 0.125 ** 2 * 100.0 / p50["theta"]
    wall = time.perf_counter() - t0
    out = {
        "metric": "splash spread coefficient C of r/D = C sqrt(Ut/D) at short times (Re = 100)",
        "value": runs["100"]["C_short"], "unit": "dimensionless", "n_gpus": 1, "steps": None, "warmup": 0,
        "ms_per_step": None, "higher_is_better": None, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "600x250 splash, D = 100, U = 0.125, a = 0.25, T = 0.5Tc, walls in y (Sec. IV.C)",
                   "parallelism": "single GPU"},
        "runs": runs, "weber": {"theta": p50["theta"], "rho_l": p50["rho_in"], "We": round(we, 2)},
        "paper": {"C": 1.3, "We": 103}, "wall_seconds": round(wall, 2), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_lamb(args):
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp
    from paper_1211_6932_amd import validation as V

    torch.cuda.set_device(0)
    lbmp.load()
    R0 = W.oscillating_droplet().info["R0"]
    t0 = time.perf_counter()
    st = V.surface_tension(W.laplace_droplets(radii=(20.0, 25.0, R0, 30.0, 35.0)), log=log)
    theta = [p["theta"] for p in st["points"] if p["R0"] == R0][0]
    runs = {}
    for nu in (0.05, 0.1):
        w = W.oscillating_droplet(nu_l=nu)
        o = V.oscillation(w, log=log)
        ta = V.lamb_period(theta, o["rho_l"], R0)
        runs[str(nu)] = {"period_damped": round(o["period"], 1), "period_undamped": round(o["period0"], 1),
                         "lamb": round(ta, 1), "rel_error": round(o["period0"] / ta - 1.0, 5),
                         "decay_steps": round(o["decay"], 0), "viscous_decay_steps": round(R0 ** 2 / (4 * nu), 0),
                         "rho_l": round(o["rho_l"], 5)}
    wall = time.perf_counter() - t0
    err = max(abs(r["rel_error"]) for r in runs.values())
    out = {
        "metric": "droplet oscillation period vs Lamb's Eq. (32), max relative error over nu_l = 0.05, 0.1",
        "value": round(err, 5), "unit": "fraction", "n_gpus": 1, "steps": 10400, "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "200x200 ellipse 30x27, T=0.5Tc, a=0.5, nu_g=0.3 (Sec. IV.A, Fig. 2)",
                   "parallelism": "single GPU"},
        "surface_tension": {"theta_at_R0": theta, "laplace_slope": st["theta"], "laplace_intercept": st["c"],
                            "r2": st["r2"]},
        "runs": runs, "paper": {"numerical": 2600.0, "analytical": 2593.8}, "wall_seconds": round(wall, 2),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="splash",
                    choices=["splash", "splash1k", "precision", "batch", "learned", "lamb", "sweeps", "spread"])
    ap.add_argument("--train-runs", type=int, default=4096)
    ap.add_argument("--eval-droplets", type=int, default=256)
    ap.add_argument("--relax-steps", type=int, default=30000)
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--no-tune", action="store_true", help="batch: keep the measured strip-height table")
    ap.add_argument("--no-persistent", action="store_true", help="batch: skip the per-lattice timing run")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default 2000 (splash), 10000 (batch)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--store", default="f32", choices=sorted(BYTES_PER_SITE))
    ap.add_argument("--scale", type=int, default=4, help="splash geometry scale (4 -> 8192x4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-copy-probe", action="store_true")
    args = ap.parse_args()

    if args.steps is None:
        args.steps = {"batch": 10000, "splash1k": 20000}.get(args.workload, 2000)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "splash1k":
        return bench_splash1k(args)
    if args.workload == "lamb":
        return bench_lamb(args)
    if args.workload == "sweeps":
        return bench_sweeps(args)
    if args.workload == "spread":
        return bench_spread(args)
    if args.workload == "precision":
        return bench_precision(args)

    import numpy as np
    import torch

    import workloads as W
    from paper_1211_6932_amd import lbmp

    torch.cuda.set_device(0)
    lbmp.load()
    w = W.splash(scale=args.scale, Re=200)
    nx, ny = w.params["nx"], w.params["ny"]
    rho_ref = w.info["rho_l"] if args.store in ("f16", "bf16") else 0.0
    log(f"workload {w.name} store={args.store}: init")
    sim = lbmp.Sim(w.params, torch.from_numpy(np.asarray(w.rho0, np.float32)),
                   torch.from_numpy(np.asarray(w.ux0, np.float32)),
                   torch.from_numpy(np.asarray(w.uy0, np.float32)), store=args.store, rho_ref=rho_ref)
    c = (nx / 2.0, w.info["film"] + w.info["R"] + 5.0 * args.scale)
    d0 = sim.diagnostics(c[0], c[1], 1.0, 2.0)

    log(f"warmup {args.warmup} steps")
    sim.step(args.warmup)
    sim.stream.synchronize()
    torch.cuda.synchronize()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log(f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(sim.stream)
    sim.step(args.steps)
    e1.record(sim.stream)
    sim.stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e0.elapsed_time(e1) / args.steps

    stable = lbmp.lb_check(sim.ctx) == lbmp.LB_OK
    d1 = sim.diagnostics(c[0], c[1], 1.0, 2.0, raise_unstable=False)
    sites = nx * ny
    mlups = sites * args.steps / wall / 1e6
    bps = BYTES_PER_SITE[args.store]
    achieved = bps * sites / (kern_ms * 1e-3) / 1e9
    tbytes = measured_traffic(args.store, sites)
    traffic = None if tbytes is None else tbytes / (kern_ms * 1e-3) / 1e9
    log(f"{mlups:.0f} MLUPS, step {kern_ms:.4f} ms, {achieved:.0f} GB/s algorithmic, stable={stable}")

    copy_gbps = None
    if not args.no_copy_probe:
        copy_gbps = copy_probe_gbps(torch, lbmp, sim.stream)
        log(f"copy probe {copy_gbps:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        del sim
        torch.cuda.empty_cache()
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"cpu baseline {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

    out = {
        "metric": "MLUPS (D2Q9 MRT improved pseudopotential step) and % of HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.store == "f32" else f"{args.store} storage, f32 compute",
        "data": "synthetic",
        "config": {
            "workload": f"droplet splash on a thin film, {nx}x{ny}, walls in y, x periodic, "
                        f"a=0.25, T=0.45Tc, sigma=0.114, U=0.05, nu_l=0.05, nu_g=0.75",
            "nx": nx, "ny": ny, "store": args.store, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": None if traffic is None else round(traffic, 1),
            "traffic_bytes_per_launch": tbytes, "algorithmic_bytes_per_launch": bps * sites,
            "bytes_per_site": bps, "kernel_ms": round(kern_ms, 5),
            "copy_probe_GBps": None if copy_gbps is None else round(copy_gbps, 1),
        },
        "cpu_baseline": cpu,
        "checks": {
            "stable": bool(stable),
            "mass_rel_drift": (d1["mass"] - d0["mass"]) / d0["mass"],
            "max_u": d1["max_u"],
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
