#!/usr/bin/env python3
"""Throughput of the short-range MD hot path on one MI355X.

One step = one velocity-Verlet step of the whole path (kick + drift + skin
check, cell binning/sort and neighbour search when due, pair forces with the
second half kick, energy/virial reductions) over the whole system.

Headline workload: 1,048,576-particle binary Lennard-Jones mixture (80:20,
eps/sigma tensors of the paper's mixture, rc = 2.5 sigma_ab shifted force),
number density 1.2, FCC + 0.05 sigma jitter, Maxwell velocities at T = 2.0,
NVE, dt = 0.005, skin 0.3 sigma.  Inputs are seeded synthetic arrays resident
in HBM before the timed region.  `value` is the plain FP64 path; the
FP32-force mixed form and the batched-replica form (256 boxes of 1,000 to
65,536 particles at T in [0.4, 2.0] with the velocity-rescale thermostat) are
reported beside it.

Prints one JSON line on stdout; progress goes to stderr.

Other modes (used to make the committed profiles/ summaries):
  --calibrate-copy          a plain 1 GiB device copy (counter calibration)
  --counters-summary DIRS   turn rocprofv3 --pmc outputs into
                            profiles/force_counters.json
  --long-drift N            only the energy drift of the 1M FP64 / mixed
                            forms over an N-step NVE run (one JSON line)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "particle-steps/sec on 1 MI355X + % HBM roofline; mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0
FORCE_SRC = os.path.join(ROOT, "paper_1105_5613_amd", "csrc", "force.hip")
# the list build fixes the order in which the force kernel gathers, and so
# its traffic: the counters hold for this pair of sources only
LIST_SRC = os.path.join(ROOT, "paper_1105_5613_amd", "csrc", "nlist.hip")
COUNTERS_JSON = os.path.join(ROOT, "profiles", "force_counters.json")
FP64_OPS_JSON = os.path.join(ROOT, "profiles", "fp64_ops.json")
FP64_PEAK_TFLOPS = 78.6
LARGE_N = 67108864  # the large mixed form; its counters hold for this size only
CSRC = os.path.join(ROOT, "paper_1105_5613_amd", "csrc")
# kernels whose FP64 operation counts the bench turns into FLOP/s: name
# fragment in the counter output -> source file
FLOP_KERNELS = {"cells_fp64": ("k_force_cells<false", "force_cells.hip"),
                "nlist_fp64": ("k_nlist_cells<4, false", "nlist.hip"),
                "force_fp64": ("k_force<false, 2", "force.hip")}
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_particle(nbar: float, mixed: bool) -> float:
    """Algorithmic HBM bytes per particle of one in-step force launch of an
    NVE step, which also applies the next step's half kick and drift.

    count (4) + list entries (4 nbar) + the home particle's position and
    species (24 + 4) + v read and write (48) + x_ref (24) + the drifted
    position written (24); mixed also reads and writes the 16-byte gather
    record (32).  The forces stay in registers; neighbour positions x_j are
    gathered from cache and not counted.  These are the bytes the method
    moves: the stored position record is 32 bytes (species kept as a
    double), and its 4 padding bytes per read and 8 per write are not
    counted.
    """
    return 4 + 4 * nbar + 28 + 48 + 24 + 24 + (32 if mixed else 0)


def step_bytes_per_particle(nbar: float, mixed: bool, rebuilds_per_step: float) -> float:
    """Algorithmic HBM bytes per particle-step of the whole step: the force
    launch (kick and drift included) and one rebuild (bin 28, sort keys 24,
    reorder 160, list write 4 nbar + 4) times the measured rebuilds per step."""
    rebuild = 28 + 24 + 160 + 4 * nbar + 4
    return force_bytes_per_particle(nbar, mixed) + rebuild * rebuilds_per_step


def copy_gbs(torch) -> float:
    """HBM bandwidth of a plain 1 GiB device copy (read + write), timed with
    events over 5 copies after one warm-up copy."""
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def src_sha(path: str = FORCE_SRC) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def fp64_flops_per_particle(key: str):
    """FP64 FLOP per particle of one launch of a kernel, from the committed
    rocprofv3 operation counts (64 lanes x (ADD + MUL + 2 FMA + TRANS) wave
    instructions per dispatch, over the particles of the measured box), or
    None when the kernel's source changed since the counters were taken."""
    if not os.path.exists(FP64_OPS_JSON):
        return None
    with open(FP64_OPS_JSON) as f:
        d = json.load(f)
    ent = d.get("kernels", {}).get(key)
    if not ent or ent.get("src_sha256") != src_sha(os.path.join(CSRC, FLOP_KERNELS[key][1])):
        return None
    return ent["flop_per_dispatch"] / ent["particles"]


def counters_traffic(key: str):
    """HBM bytes per force launch from the committed rocprofv3 counter runs, or
    None when the force kernel or the list build (the gather order) changed
    since the counters were taken."""
    if not os.path.exists(COUNTERS_JSON):
        return None
    with open(COUNTERS_JSON) as f:
        d = json.load(f)
    ent = d.get("forms", {}).get(key)
    if not ent or d.get("force_src_sha256") != src_sha() or \
            d.get("list_src_sha256") != src_sha(LIST_SRC):
        return None
    return ent["fetch_kib"] * 1024 * d["copy_factor_fetch"] + \
        ent["write_kib"] * 1024 * d["copy_factor_write"]


def mixture():
    import initconf
    return initconf.mixture_tables()


LOG_EVERY = 10  # observables logged every 10 timed steps
DRIFT_STEPS = 1100  # the NVE window of the drift figure, whatever --steps is
DRIFT_BURN = 100
FORCE_SAMPLE = 4096  # particles whose forces are checked against the oracle


def energy_drift(E, n: int, burn: int = DRIFT_BURN):
    """Energy drift D of an NVE run whose total energy E was logged after
    every step 1, 2, ...: |least-squares slope of E/N| per 1,000 steps over
    the steps after a burn-in (the start-up transient of a lattice start).
    Also the largest |E - E(burn)|/N.  None when fewer than 900 steps follow
    the burn-in."""
    import numpy as np
    e = np.asarray(E, dtype=np.float64) / n
    step = 1.0 + np.arange(len(e), dtype=np.float64)
    keep = step >= burn
    if len(e) - burn < 900:
        return None
    d = float(abs(np.polyfit(step[keep], e[keep], 1)[0]) * 1000.0)
    return {"D": d, "max_abs_dE_per_particle": float(np.max(np.abs(e[keep] - e[keep][0])))}


def floored_force_error(F_sel, Fo_sel, frms: float) -> float:
    """e = max_i |F_i - F_i^ref| / max(|F_i^ref|, F_rms) over the sample."""
    import numpy as np
    d = np.linalg.norm(np.asarray(F_sel, dtype=np.float64) - Fo_sel, axis=1)
    return float(np.max(d / np.maximum(np.linalg.norm(Fo_sel, axis=1), frms)))


def run_drift(precision: int, inputs, path: int = 1, potential: int = 0, global_rc=None,
              dt: float = 0.005, steps: int = DRIFT_STEPS):
    """D over `steps` (default DRIFT_STEPS) NVE steps of a fresh context from
    the form's initial state (energies every step), so the figure does not
    depend on --steps."""
    from paper_1105_5613_amd import System, make_params
    import initconf
    eps, sig, rc, mass = initconf.mixture_tables(global_rc=global_rc)
    p = make_params(eps, sig, rc, mass, skin=0.3, dt=dt, precision=precision, path=path,
                    potential=potential)
    n = inputs["n"]
    sysm = System(p, [n], [inputs["L"]])
    sysm.set_state(inputs["x"], inputs["v"], inputs["type"])
    lg = sysm.step(steps, log_every=1)
    sysm.close()
    out = energy_drift(lg["E"][:, 0], n)
    out["window"] = f"steps {DRIFT_BURN}..{steps} of an NVE run from the initial state, " \
                    f"dt {dt}, E logged every step"
    return out


def run_single(torch, precision: int, inputs, steps: int, warmup: int, prof_every: int,
               path: int = 1, potential: int = 0, global_rc=None, dt: float = 0.005, T0=None,
               graph_steps: int = 0, sample_forces: bool = False):
    from paper_1105_5613_amd import System, make_params
    import initconf
    eps, sig, rc, mass = initconf.mixture_tables(global_rc=global_rc)
    p = make_params(eps, sig, rc, mass, skin=0.3, dt=dt, precision=precision, path=path,
                    potential=potential, graph_steps=graph_steps)
    n = inputs["n"]
    sysm = System(p, [n], [inputs["L"]])
    sysm.set_state(inputs["x"], inputs["v"], inputs["type"])
    sysm.step(warmup, T0=T0)
    tuned = sysm.autotune(reps=3)
    sysm.profile(prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lg = sysm.step(steps, T0=T0, log_every=LOG_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sysm.profile_read()
    sysm.profile(0)
    nbar, nmax = (0.0, 0) if path == 3 else sysm.list_stats()
    obs = sysm.observables()[0]
    sample = None
    if sample_forces:
        # the forces on the state the timed run reached, for the CPU leg's
        # comparison with the oracle (a sample of FORCE_SAMPLE particles)
        import numpy as np
        x = sysm.get_state()[0].cpu().numpy()
        sysm.forces()
        F = sysm.get_forces().cpu().numpy().astype(np.float64)
        sel = np.random.default_rng(11).choice(n, FORCE_SAMPLE, replace=False)
        sample = {"x": x, "type": inputs["type"], "L": inputs["L"], "sel": sel,
                  "F_sel": F[sel], "frms": float(np.sqrt(np.mean(np.sum(F * F, axis=1))))}
    sysm.close()
    return {"wall_s": wall, "rate": n * steps / wall, "ms_per_step": 1e3 * wall / steps,
            # None when no launch was timed (--profile-every 0)
            "force_ms_avg": (prof["force_ms"] / prof["force_launches"]
                             if prof["force_launches"] else None),
            "force_launches_timed": prof["force_launches"], "nbar": nbar, "nmax": nmax,
            "rebuilds": obs["n_rebuild"], "steps_total": obs["step"], "sample": sample,
            "tuned": {"tpp": tuned["tpp"], "unroll": tuned["unroll"]}}


def replica_inputs(nrep: int):
    import initconf
    sizes = initconf.replica_sizes(nrep, 1000, 65536, seed=4)
    temps = initconf.replica_temperatures(nrep, 0.4, 2.0, seed=4)
    systems = initconf.batched_systems(sizes, temps, seed=4)
    return systems, temps


TUNE_SKINS = (0.2, 0.3, 0.4)


def run_batched(torch, precision: int, systems, temps, steps: int, warmup: int,
                graph_steps: int, tune: bool = True):
    """The batch in one context.  tune: first pick the kernel path, the skin
    (which sets the cell side, the smallest the 27-cell stencil allows for
    it), the staged tile length and the force variant by short trial runs of
    the same batch (paper_1105_5613_amd.tune, not timed)."""
    import initconf
    from paper_1105_5613_amd import System, make_params
    eps, sig, rc, mass = mixture()
    x, v, t, n, L = initconf.concat_replicas(systems)
    p = make_params(eps, sig, rc, mass, skin=0.3, dt=0.005, precision=precision,
                    graph_steps=graph_steps)
    choice = None
    if tune:
        from paper_1105_5613_amd import tune as tuner
        p, rep_ = tuner.autotune(p, n, L, x, v, t, T0=temps, steps=60, warmup=20,
                                 skins=TUNE_SKINS, tile_cells=(0,), use_cache=False,
                                 cache_path=None)
        choice = {"choice": rep_.get("choice"),
                  "trials": [{**tr["choice"], "rate": round(tr["rate"], 1)}
                             for tr in rep_.get("trials", [])]}
    sysm = System(p, n, L)
    sysm.set_state(x, v, t)
    sysm.step(warmup, T0=temps)
    tuned = sysm.autotune(reps=3)
    sysm.step(graph_steps, T0=temps)  # captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(steps, T0=temps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = sysm.observables()
    sysm.close()
    terr = max(abs(o["T"] - tt) / tt for o, tt in zip(obs, temps))
    return {"rate": sum(n) * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "particles": sum(n), "max_rel_T_error": terr,
            "tuned": {"path": int(p.path), "skin": float(p.skin), "tpp": tuned["tpp"],
                      "unroll": tuned["unroll"]},
            "tuner": choice}


def run_one_at_a_time(torch, systems, temps, steps: int):
    """The same replicas, each its own context, plain FP64, run one after another."""
    from paper_1105_5613_amd import System, make_params
    eps, sig, rc, mass = mixture()
    p = make_params(eps, sig, rc, mass, skin=0.3, dt=0.005, precision=0)
    ctxs = []
    for s, tt in zip(systems, temps):
        c = System(p, [s["n"]], [s["L"]])
        c.set_state(s["x"], s["v"], s["type"])
        c.step(5, T0=[tt])
        ctxs.append((c, tt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, tt in ctxs:
        c.step(steps, T0=[tt])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for c, _ in ctxs:
        c.close()
    return {"rate": sum(s["n"] for s in systems) * steps / wall, "steps": steps}


def oracle_force_errors(samples):
    """The CPU leg's accuracy check: for each GPU form, the oracle's forces on
    the sampled particles of the state the form reached, and the floored
    error e of the GPU forces against them."""
    import oracle
    eps, sig, rc, mass = mixture()
    p = oracle.make_params(eps, sig, rc, mass, skin=0.3)
    out = {}
    for form, sm in samples.items():
        Fo, _, _ = oracle.forces_cells(p, sm["x"], sm["type"], sm["L"], sel=sm["sel"])
        out[form] = {"e": floored_force_error(sm["F_sel"], Fo, sm["frms"]),
                     "sample": f"{len(sm['sel'])} random particles of the state after the "
                               "timed steps, FP64 oracle cell-list forces",
                     "norm": "max_i |dF_i| / max(|F_i|, F_rms)"}
    return out


def cpu_baseline(inputs, nsteps: int, nsteps_1t: int = 4):
    import oracle
    eps, sig, rc, mass = mixture()
    p = oracle.make_params(eps, sig, rc, mass, skin=0.3)
    sim = oracle.Sim(p, inputs["n"], inputs["L"], 0.005)
    sim.set_state(inputs["x"], inputs["v"], inputs["type"])
    sim.forces()  # first list build and F(0), untimed
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    sim.step(nsteps)
    wall = time.perf_counter() - t0
    # the same oracle on one thread, over a shorter stretch of the same run
    oracle.set_threads(1)
    t1 = time.perf_counter()
    sim.step(nsteps_1t)
    wall1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": inputs["n"] * nsteps / wall, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{nsteps} velocity-Verlet steps (with their list rebuilds) of the same "
                      f"{inputs['n']}-particle system after its first list build; FP64 C "
                      f"oracle, OpenMP over particles, {wall:.1f} s",
            "one_thread": {"value": inputs["n"] * nsteps_1t / wall1,
                           "sample": f"the next {nsteps_1t} steps on one thread, {wall1:.1f} s"}}


def cells_flops(n: int, force_ms: float):
    """The list-free force kernel is bound by FP64 vector issue, not HBM: its
    FP64 FLOP rate (committed operation counts per particle x n / the
    measured mean launch time) against the 78.6 TFLOP/s FP64 vector peak."""
    fpp = fp64_flops_per_particle("cells_fp64")
    if fpp is None or not force_ms:
        return None
    tf = fpp * n / (force_ms * 1e-3) / 1e12
    return {"bound": "fp64 vector alu", "flop_per_particle": round(fpp, 1),
            "achieved_tflops": round(tf, 2), "peak_tflops": FP64_PEAK_TFLOPS,
            "frac": round(tf / FP64_PEAK_TFLOPS, 4),
            "source": "profiles/fp64_ops.json (rocprofv3 SQ_INSTS_VALU_*_F64)"}


def calibrate_copy(torch):
    """A plain device-to-device copy of COPY_BYTES (counter calibration)."""
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {COPY_BYTES} bytes 3 times")


def _counter_rows(d, name_part):
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if name_part in r["Kernel_Name"]:
                out.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(
                    float(r["Counter_Value"]))
    return out


def fp64_ops_summary(args):
    """FP64 operation counts (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64, wave
    instructions per dispatch) of the kernels in FLOP_KERNELS, averaged over
    the dispatches that did work, into profiles/fp64_ops.json."""
    out = {"commands": args.commands, "particles": args.n, "kernels": {}}
    for key, (frag, src) in FLOP_KERNELS.items():
        rows = _counter_rows(args.flops_dir, frag)
        per = {}
        for (k, c), vs in rows.items():
            per.setdefault(c, []).extend(vs)
        need = ["SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                "SQ_INSTS_VALU_TRANS_F64"]
        if not all(c in per for c in need):
            continue
        # dispatches that did work (a gated launch counts next to nothing)
        tot = [sum(per[c][i] for c in need) for i in range(len(per[need[0]]))]
        keep = [i for i, t in enumerate(tot) if t > 0.05 * max(tot)]
        mean = {c: sum(per[c][i] for i in keep) / len(keep) for c in need}
        flop = 64.0 * (mean[need[0]] + mean[need[1]] + 2.0 * mean[need[2]] + mean[need[3]])
        out["kernels"][key] = {"kernel": frag, "dispatches": len(keep), "particles": args.n,
                               "wave_instructions": mean, "flop_per_dispatch": flop,
                               "src_sha256": src_sha(os.path.join(CSRC, src))}
    with open(FP64_OPS_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def counters_summary(args):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the in-step force kernels,
    scaled by what the same counters read for the plain copy."""
    def mean_for(d, kern, counter, keyword):
        rows = _counter_rows(d, kern)
        vals = [v for (k, c), vs in rows.items() if c == counter and keyword in k for v in vs]
        return sum(vals) / len(vals), len(vals)

    cf, _ = mean_for(args.copy_fetch_dir, "", "FETCH_SIZE", "copy")
    cw, _ = mean_for(args.copy_write_dir, "", "WRITE_SIZE", "copy")
    copy_kib = COPY_BYTES / 1024
    out = {"force_src_sha256": src_sha(), "list_src_sha256": src_sha(LIST_SRC),
           "copy_bytes": COPY_BYTES, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "copy_factor_fetch": copy_kib / cf, "copy_factor_write": copy_kib / cw,
           "forms": {}, "commands": args.commands}
    runs = [("fp64", "k_force<false, 2", args.fetch_dir, args.write_dir),
            ("mixed", "k_force<true, 2", args.fetch_dir, args.write_dir)]
    if args.large_fetch_dir and args.large_write_dir:
        runs.append(("large_mixed", "k_force<true, 2", args.large_fetch_dir,
                     args.large_write_dir))
    for form, key, fdir, wdir in runs:
        try:
            f, nf = mean_for(fdir, "k_force", "FETCH_SIZE", key)
            w, nw = mean_for(wdir, "k_force", "WRITE_SIZE", key)
        except ZeroDivisionError:
            continue
        out["forms"][form] = {"fetch_kib": f, "write_kib": w, "dispatches": nf}
    os.makedirs(os.path.dirname(COUNTERS_JSON), exist_ok=True)
    with open(COUNTERS_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--forms", default="fp64,mixed,small,large,batched,cells,soft")
    ap.add_argument("--profile-every", type=int, default=4,
                    help="bracket the force launch of every k-th timed step with hipEvents")
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-drift", action="store_true",
                    help="skip the untimed 1,100-step drift runs (profiler sessions)")
    ap.add_argument("--n", type=int, default=1048576)
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--large-n", type=int, default=LARGE_N)
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--serial-steps", type=int, default=50)
    ap.add_argument("--graph-steps", type=int, default=100,
                    help="steps per captured hipGraph in the batched form (0: direct launches)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--long-drift", type=int, default=0)
    ap.add_argument("--counters-summary", action="store_true")
    ap.add_argument("--fp64-ops-summary", action="store_true")
    ap.add_argument("--flops-dir")
    ap.add_argument("--fetch-dir")
    ap.add_argument("--write-dir")
    ap.add_argument("--copy-fetch-dir")
    ap.add_argument("--copy-write-dir")
    ap.add_argument("--large-fetch-dir")
    ap.add_argument("--large-write-dir")
    ap.add_argument("--commands", default="")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, ROOT)
    if args.counters_summary:
        counters_summary(args)
        return
    if args.fp64_ops_summary:
        fp64_ops_summary(args)
        return
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    import initconf
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    n = args.n
    log(f"generating inputs n={n}")
    inputs = initconf.fcc_system(n, seed=2, temperature=2.0)
    if args.long_drift:
        out = {"particles": n, "steps": args.long_drift, "forms": {}}
        for f in forms:
            if f in ("fp64", "mixed"):
                log(f"drift of form {f} over {args.long_drift} NVE steps")
                out["forms"][f] = run_drift(1 if f == "mixed" else 0, inputs,
                                            steps=args.long_drift)
                log(f"  {f}: D {out['forms'][f]['D']:.3e}")
        print(json.dumps(out))
        return
    res = {}
    for f in forms:
        if f not in ("fp64", "mixed"):
            continue
        log(f"timing form {f}: {args.steps} steps after {args.warmup} warmup")
        res[f] = run_single(torch, 1 if f == "mixed" else 0, inputs, args.steps, args.warmup,
                            args.profile_every, sample_forces=not args.no_cpu_baseline)
        res[f]["drift"] = None if args.no_drift else run_drift(1 if f == "mixed" else 0, inputs)
        log(f"  {f}: {res[f]['rate']:.4e} particle-steps/s, {res[f]['ms_per_step']:.4f} ms/step, "
            f"force {res[f]['force_ms_avg']} ms, nbar {res[f]['nbar']:.2f}, "
            f"rebuilds {res[f]['rebuilds']}, drift {(res[f]['drift'] or {}).get('D')}")
    def gbs(nb, ms):
        return None if not ms else nb / (ms * 1e-3) / 1e9

    def rnd(v, k):
        return None if v is None else round(v, k)

    forms_out = {}
    for f, r in res.items():
        b = force_bytes_per_particle(r["nbar"], f == "mixed")
        tr = counters_traffic(f)
        ach = gbs(n * b, r["force_ms_avg"])
        forms_out[f] = {"value": round(r["rate"], 1), "ms_per_step": round(r["ms_per_step"], 5),
                        "force_ms_avg": rnd(r["force_ms_avg"], 5),
                        "force_achieved_gbs": rnd(ach, 1),
                        "force_frac_hbm": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
                        "force_traffic_bytes": None if tr is None else round(tr),
                        "force_traffic_over_algorithmic": None if tr is None else round(tr / (n * b), 3),
                        "step_algorithmic_frac_hbm": round(
                            r["rate"] * step_bytes_per_particle(
                                r["nbar"], f == "mixed",
                                r["rebuilds"] / max(r["steps_total"], 1)) / 1e9 / HBM_PEAK_GBS, 4),
                        "mean_list_length": round(r["nbar"], 3), "rebuilds": r["rebuilds"],
                        "energy_drift_per_particle_per_1000_steps": (r["drift"] or {}).get("D"),
                        "energy_drift": r["drift"],
                        "tuned": r["tuned"]}
    if "fp64" in res and "mixed" in res:
        forms_out["speedup_mixed_vs_fp64"] = round(res["mixed"]["rate"] / res["fp64"]["rate"], 4)
    if "large" in forms:
        nl = args.large_n
        log(f"generating inputs n={nl}")
        big = initconf.fcc_system(nl, seed=3, temperature=2.0)
        log(f"timing the large mixed form: {args.large_steps} steps after 20 warmup")
        rl = run_single(torch, 1, big, args.large_steps, 20, args.profile_every)
        log(f"  large mixed drift window: {DRIFT_STEPS} NVE steps")
        rl["drift"] = None if args.no_drift else run_drift(1, big)
        del big
        bl = force_bytes_per_particle(rl["nbar"], True)
        ach = gbs(nl * bl, rl["force_ms_avg"])
        trl = counters_traffic("large_mixed") if nl == LARGE_N else None
        log(f"  large mixed: {rl['rate']:.4e} particle-steps/s, {rl['ms_per_step']:.3f} ms/step, "
            f"force {rl['force_ms_avg']} ms")
        forms_out["large_mixed"] = {
            "workload": f"lj{nl}: {nl}-particle binary LJ mixture, mixed precision, T=2.0 NVE, "
                        "dt 0.005, skin 0.3",
            "value": round(rl["rate"], 1), "ms_per_step": round(rl["ms_per_step"], 4),
            "force_ms_avg": rnd(rl["force_ms_avg"], 4), "force_achieved_gbs": rnd(ach, 1),
            "force_frac_hbm": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
            "force_traffic_bytes": None if trl is None else round(trl),
            "force_traffic_over_algorithmic": None if trl is None else round(trl / (nl * bl), 3),
            "mean_list_length": round(rl["nbar"], 3), "rebuilds": rl["rebuilds"],
            "energy_drift_per_particle_per_1000_steps": (rl["drift"] or {}).get("D"),
            "energy_drift": rl["drift"], "tuned": rl["tuned"]}
    if "small" in forms:
        log(f"timing the 4000-particle box (FP64): {args.steps} steps, direct and in graphs")
        small = initconf.fcc_system(4000, seed=1, temperature=2.0)
        rd = run_single(torch, 0, small, args.steps, args.warmup, 0)
        rg = run_single(torch, 0, small, args.steps, args.warmup, 0, graph_steps=100)
        dsmall = None if args.no_drift else run_drift(0, small)
        log(f"  small: direct {rd['rate']:.4e}, graphs {rg['rate']:.4e} particle-steps/s")
        forms_out["small_fp64"] = {
            "workload": "lj4000: 4,000-particle binary LJ mixture (FCC n=10, L=14.938, 5 cells "
                        "per side), FP64, T=2.0 NVE, dt 0.005, skin 0.3; launch-bound",
            "value_direct": round(rd["rate"], 1), "ms_per_step_direct": round(rd["ms_per_step"], 5),
            "value_graphs_100": round(rg["rate"], 1),
            "ms_per_step_graphs_100": round(rg["ms_per_step"], 5),
            "rebuilds": rd["rebuilds"],
            "energy_drift_per_particle_per_1000_steps": (dsmall or {}).get("D"),
            "energy_drift": dsmall}
    if "cells" in forms:
        log(f"timing the list-free cell path (FP64): {args.steps} steps")
        rcell = run_single(torch, 0, inputs, args.steps, args.warmup, args.profile_every, path=3)
        rcell["drift"] = None if args.no_drift else run_drift(0, inputs, path=3)
        log(f"  cell path: {rcell['rate']:.4e} particle-steps/s, {rcell['ms_per_step']:.4f} ms/step, "
            f"force {rcell['force_ms_avg']} ms")
        forms_out["cells_fp64"] = {
            "workload": f"lj{n} as the headline, list-free cell path (no neighbour list; the "
                        "27-cell stencil searched in every force launch)",
            "value": round(rcell["rate"], 1), "ms_per_step": round(rcell["ms_per_step"], 5),
            "force_ms_avg": rnd(rcell["force_ms_avg"], 5), "rebuilds": rcell["rebuilds"],
            "force_fp64": cells_flops(n, rcell["force_ms_avg"]),
            "energy_drift_per_particle_per_1000_steps": (rcell["drift"] or {}).get("D"),
            "energy_drift": rcell["drift"]}
        if "fp64" in res:
            forms_out["cells_fp64"]["rate_vs_list_fp64"] = round(rcell["rate"] / res["fp64"]["rate"], 4)
    if "soft" in forms:
        log(f"timing the soft-sphere workload: {args.steps} steps")
        soft_in = initconf.fcc_system(n, seed=6, temperature=0.5)
        rs = run_single(torch, 0, soft_in, args.steps, args.warmup, args.profile_every,
                        potential=1, global_rc=1.2, dt=0.001, T0=0.5)
        dsoft = None if args.no_drift else run_drift(0, soft_in, potential=1, global_rc=1.2,
                                                     dt=0.001)
        del soft_in
        log(f"  soft sphere: {rs['rate']:.4e} particle-steps/s, {rs['ms_per_step']:.4f} ms/step")
        forms_out["soft_fp64"] = {
            "workload": f"soft{n}: binary soft-sphere mixture Eq. (2), rho 1.2, canonical T=0.5 "
                        "(velocity rescale), rc=1.2 for every pair, dt 0.001, skin 0.3, FP64",
            "value": round(rs["rate"], 1), "ms_per_step": round(rs["ms_per_step"], 5),
            "force_ms_avg": rnd(rs["force_ms_avg"], 5),
            "mean_list_length": round(rs["nbar"], 3), "rebuilds": rs["rebuilds"],
            "nve_energy_drift_per_particle_per_1000_steps": (dsoft or {}).get("D"),
            "nve_energy_drift": None if dsoft is None else dict(
                dsoft, note="the same box and start run NVE (the timed run is canonical, "
                "where energy is not conserved)")}
    if "batched" in forms:
        log(f"timing batched replicas: {args.replicas} boxes, {args.batched_steps} steps")
        systems, temps = replica_inputs(args.replicas)
        bf = run_batched(torch, 0, systems, temps, args.batched_steps, 20, args.graph_steps)
        bm = run_batched(torch, 1, systems, temps, args.batched_steps, 20, args.graph_steps)
        log(f"  batched fp64 {bf['rate']:.4e}, mixed {bm['rate']:.4e} particle-steps/s "
            f"({bf['particles']} particles)")
        ser = None
        if args.serial_steps > 0:
            log(f"timing the same replicas one at a time: {args.serial_steps} steps each")
            ser = run_one_at_a_time(torch, systems, temps, args.serial_steps)
            log(f"  one at a time fp64 {ser['rate']:.4e} particle-steps/s")

        def vs_serial(rate):
            return None if ser is None else round(rate / ser["rate"], 3)
        forms_out["batched"] = {
            "workload": f"replicas{args.replicas}: sizes log-uniform 1000..65536 "
                        f"({bf['particles']} particles), T0 in [0.4, 2.0], velocity rescale "
                        f"every step, dt 0.005, {args.graph_steps}-step hipGraph chunks; "
                        f"path, skin in {list(TUNE_SKINS)} (with it the cell side), tile and "
                        "force variant autotuned on the batch",
            "tuned_fp64": bf["tuned"], "tuned_mixed": bm["tuned"],
            "tuner_fp64": bf["tuner"], "tuner_mixed": bm["tuner"],
            "value_fp64": round(bf["rate"], 1), "value_mixed": round(bm["rate"], 1),
            "ms_per_step_fp64": round(bf["ms_per_step"], 5),
            "one_at_a_time_fp64": None if ser is None else round(ser["rate"], 1),
            "speedup_batched_vs_one_at_a_time_fp64": vs_serial(bf["rate"]),
            "speedup_batched_mixed_vs_one_at_a_time_fp64": vs_serial(bm["rate"]),
            "max_rel_T_error": bf["max_rel_T_error"]}
    head = res.get("fp64") or res.get("mixed")
    head_mixed = "fp64" not in res
    roof = None
    if head is not None and head["force_ms_avg"]:
        bpp = force_bytes_per_particle(head["nbar"], head_mixed)
        achieved = gbs(n * bpp, head["force_ms_avg"])
        traffic = counters_traffic("mixed" if head_mixed else "fp64")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": "k_force (pair forces, second half kick, next step's half kick, "
                          "drift and skin check)",
                "algorithmic_bytes_per_launch": round(n * bpp),
                "force_ms_avg": round(head["force_ms_avg"], 5)}
        cgbs = copy_gbs(torch)
        roof["copy_gbs_measured"] = round(cgbs, 1)
        roof["frac_of_copy"] = round(achieved / cgbs, 4)
        if traffic is not None and head["force_ms_avg"] > 0:
            tgbs = traffic / (head["force_ms_avg"] * 1e-3) / 1e9
            roof["traffic_gbs"] = round(tgbs, 1)
            roof["traffic_frac_of_copy"] = round(tgbs / cgbs, 4)
    cpu = None
    if not args.no_cpu_baseline and head is not None:
        log(f"timing the CPU oracle: {args.cpu_steps} steps")
        cpu = cpu_baseline(inputs, args.cpu_steps)
        log(f"  oracle: {cpu['value']:.4e} particle-steps/s on {cpu['cores']} threads")
        samples = {f: r["sample"] for f, r in res.items() if r.get("sample") is not None}
        if samples:
            log(f"oracle forces on {FORCE_SAMPLE} sampled particles per form")
            for f, er in oracle_force_errors(samples).items():
                forms_out[f]["force_error_vs_oracle"] = er
                log(f"  {f}: e = {er['e']:.3e}")
    out = {
        "metric": METRIC, "value": None if head is None else round(head["rate"], 1),
        "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None if head is None else round(head["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-force/f64" if head_mixed else "f64", "data": "synthetic",
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
