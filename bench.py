#!/usr/bin/env python3
"""Throughput of the short-range MD hot path on one MI355X.

One step = one velocity-Verlet step of the whole path (kick + drift + skin
check, cell binning/sort and neighbour search when due, pair forces with the
second half kick, energy/virial reductions) over the whole system.

Workload (default): 1,048,576-particle binary Lennard-Jones mixture (80:20,
eps/sigma tensors of the paper's mixture, rc = 2.5 sigma_ab shifted force),
number density 1.2, FCC + 0.05 sigma jitter, Maxwell velocities at T = 2.0,
NVE, dt = 0.005, skin 0.3 sigma.  Inputs are seeded synthetic arrays resident
in HBM before the timed region.  `value` is the plain FP64 path; the FP32-force
mixed form and the batched-replica form are reported beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "particle-steps/sec on 1 MI355X + % HBM roofline; mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_particle(nbar: float, mixed: bool) -> float:
    """Algorithmic HBM bytes per particle of one in-step force launch.

    count (4) + list entries (4 nbar) + x_i (24) + species (4) + F write
    (24 FP64 / 12 FP32) + v read and write of the fused second half kick (48).
    Neighbour positions x_j are gathered from cache and not counted.
    """
    return 4 + 4 * nbar + 24 + 4 + (12 if mixed else 24) + 48


def counters_traffic(kernel_src: str, key: str):
    """HBM bytes per force launch from committed rocprofv3 counter runs, or None
    when the force kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "force_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    ent = d.get(key)
    if not ent or d.get("force_src_sha256") != sha:
        return None
    return ent["fetch_kib"] * 1024 * d["copy_factor_fetch"] + \
        ent["write_kib"] * 1024 * d["copy_factor_write"]


def run_form(torch, precision: int, inputs, steps: int, warmup: int, prof_every: int):
    from paper_1105_5613_amd import System, make_params
    import initconf
    eps, sig, rc, mass = initconf.mixture_tables()
    p = make_params(eps, sig, rc, mass, skin=0.3, dt=0.005, precision=precision)
    n = inputs["n"]
    sysm = System(p, [n], [inputs["L"]])
    sysm.set_state(inputs["x"], inputs["v"], inputs["type"])
    sysm.step(warmup)
    sysm.profile(prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sysm.profile_read()
    sysm.profile(0)
    nbar, nmax = sysm.list_stats()
    obs = sysm.observables()[0]
    sysm.close()
    return {"wall_s": wall, "rate": n * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "force_ms_avg": prof["force_ms"] / max(prof["force_launches"], 1),
            "force_launches_timed": prof["force_launches"], "nbar": nbar, "nmax": nmax,
            "rebuilds": obs["n_rebuild"], "steps_total": obs["step"]}


def cpu_baseline(inputs, nsteps: int):
    import initconf
    import oracle
    eps, sig, rc, mass = initconf.mixture_tables()
    p = oracle.make_params(eps, sig, rc, mass, skin=0.3)
    sim = oracle.Sim(p, inputs["n"], inputs["L"], 0.005)
    sim.set_state(inputs["x"], inputs["v"], inputs["type"])
    sim.forces()  # first list build and F(0), untimed
    t0 = time.perf_counter()
    sim.step(nsteps)
    wall = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": inputs["n"] * nsteps / wall, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{nsteps} velocity-Verlet steps (with their list rebuilds) of the same "
                      f"{inputs['n']}-particle system after its first list build; FP64 C "
                      f"oracle, OpenMP over particles, {wall:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--profile-every", type=int, default=4,
                    help="bracket the force launch of every k-th timed step with hipEvents")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=1048576)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, ROOT)
    import torch
    import initconf
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    log(f"generating inputs n={args.n}")
    inputs = initconf.fcc_system(args.n, seed=2, temperature=2.0)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    res = {}
    for f in forms:
        if f not in ("fp64", "mixed"):
            continue
        log(f"timing form {f}: {args.steps} steps after {args.warmup} warmup")
        res[f] = run_form(torch, 1 if f == "mixed" else 0, inputs, args.steps, args.warmup,
                          args.profile_every)
        log(f"  {f}: {res[f]['rate']:.4e} particle-steps/s, {res[f]['ms_per_step']:.4f} ms/step, "
            f"force {res[f]['force_ms_avg']:.4f} ms, nbar {res[f]['nbar']:.2f}, "
            f"rebuilds {res[f]['rebuilds']}")
    head = res.get("fp64") or next(iter(res.values()))
    head_mixed = "fp64" not in res
    n = args.n
    bpp = force_bytes_per_particle(head["nbar"], head_mixed)
    achieved = n * bpp / (head["force_ms_avg"] * 1e-3) / 1e9
    src = os.path.join(ROOT, "paper_1105_5613_amd", "csrc", "force.hip")
    traffic = counters_traffic(src, "mixed" if head_mixed else "fp64")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "kernel": "k_force (pair forces + fused second half kick)",
            "algorithmic_bytes_per_launch": round(n * bpp),
            "force_ms_avg": round(head["force_ms_avg"], 5)}
    forms_out = {}
    for f, r in res.items():
        b = force_bytes_per_particle(r["nbar"], f == "mixed")
        forms_out[f] = {"value": round(r["rate"], 1), "ms_per_step": round(r["ms_per_step"], 5),
                        "force_ms_avg": round(r["force_ms_avg"], 5),
                        "force_frac_hbm": round(n * b / (r["force_ms_avg"] * 1e-3) / 1e9
                                                / HBM_PEAK_GBS, 4),
                        "mean_list_length": round(r["nbar"], 3), "rebuilds": r["rebuilds"]}
    if "fp64" in res and "mixed" in res:
        forms_out["speedup_mixed_vs_fp64"] = round(res["mixed"]["rate"] / res["fp64"]["rate"], 4)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle: {args.cpu_steps} steps")
        cpu = cpu_baseline(inputs, args.cpu_steps)
        log(f"  oracle: {cpu['value']:.4e} particle-steps/s on {cpu['cores']} threads")
    out = {
        "metric": METRIC, "value": round(head["rate"], 1), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-force/f64" if head_mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"lj{n}: {n}-particle binary Lennard-Jones mixture 80:20, rho 1.2, "
                               "FCC+0.05 jitter, T=2.0 NVE, dt 0.005, rc 2.5 sigma_ab shifted "
                               "force, skin 0.3, full neighbour list",
                   "particles": n, "form": "mixed" if head_mixed else "fp64"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
