"""Supercooling quench ensembles on the batched path (glass-transition
section): many replicas equilibrated at a high temperature, then cooled
linearly to a low one with the isokinetic velocity rescale, logging per
replica the potential energy per particle, the temperature and the
mean-squared displacement from the start of the quench (unwrapped
positions).  The caloric curve U(T) of the log gives the glass-transition
estimate as the temperature where its slope stops rising (caloric_slope).

    python -m paper_1105_5613_amd.quench --replicas 64 --n 131072 \\
        --equil 10000 --quench 100000 --log-every 1000 --out quench.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import md


def caloric_slope(T, U, window: int = 9):
    """Apparent heat capacity of a cooling curve and its glass-transition
    estimate.  The slope dU/dT is taken from least-squares lines over sliding
    windows of `window` consecutive temperatures; on cooling it rises while
    the liquid stays in equilibrium and falls once the structure freezes, so
    the temperature of the largest slope marks the change of slope.
    Returns (T_centres, slopes, T_at_max_slope, max_slope, slope_coldest)."""
    T = np.asarray(T, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    if len(T) < window + 2 or window < 3:
        raise ValueError("caloric_slope needs window >= 3 and more than window + 1 points")
    o = np.argsort(T)
    T, U = T[o], U[o]
    tc, sl = [], []
    for k in range(len(T) - window + 1):
        t, u = T[k:k + window], U[k:k + window]
        b = np.polyfit(t, u, 1)[0]
        tc.append(float(t.mean()))
        sl.append(float(b))
    tc, sl = np.array(tc), np.array(sl)
    m = int(np.argmax(sl))
    return tc, sl, float(tc[m]), float(sl[m]), float(sl[0])


def run_quench(nrep: int, n: int, *, seed: int = 5, precision: int = md.MD_MIXED,
               T_hot: float = 2.0, T_cold: float = 0.3, equil: int = 10000,
               quench: int = 100000, log_every: int = 1000, nve: int = 0, dt: float = 0.005,
               skin: float = 0.3, graph_steps: int = 100, potential: int = md.MD_POT_LJ,
               progress=None):
    """Run one quench ensemble; returns a dict of per-replica logs.

    The linear ramp T(k) = T_hot + (T_cold - T_hot) k / quench is applied in
    segments of log_every steps, each a linear ramp between its end points
    (the same schedule as one call ramping over all quench steps).  nve > 0
    appends an NVE segment at T_cold with per-step total energy, for the
    drift measure."""
    import torch
    import initconf
    say = progress or (lambda *a: None)
    if quench % log_every or equil % log_every:
        raise ValueError("equil and quench must be multiples of log_every")
    systems = initconf.batched_systems([n] * nrep, [T_hot] * nrep, seed=seed)
    x, v, t, ns, L = initconf.concat_replicas(systems)
    eps, sig, rc, mass = initconf.mixture_tables()
    p = md.make_params(eps, sig, rc, mass, skin=skin, dt=dt, precision=precision,
                       graph_steps=graph_steps, potential=potential)
    s = md.System(p, ns, L)
    s.set_state(x, v, t)
    del x, v
    out = {"replicas": nrep, "n": n, "precision": precision, "T_hot": T_hot, "T_cold": T_cold,
           "equil": equil, "quench": quench, "log_every": log_every, "dt": dt, "seed": seed}
    for k in range(0, equil, log_every):
        s.step(log_every, T0=T_hot)
        say(f"equilibration {k + log_every}/{equil}")
    s.autotune(reps=3)
    s.msd_reference()
    logs = {"step": [], "T_target": [], "pe_per_particle": [], "T": [], "msd": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(0, quench, log_every):
        ta = T_hot + (T_cold - T_hot) * k / quench
        tb = T_hot + (T_cold - T_hot) * (k + log_every) / quench
        s.step(log_every, T0=ta, T1=tb, ramp=log_every)
        ob = s.observables()
        logs["step"].append(k + log_every)
        logs["T_target"].append(tb)
        logs["pe_per_particle"].append([o["pe"] / n for o in ob])
        logs["T"].append([o["T"] for o in ob])
        logs["msd"].append(s.msd().tolist())
        say(f"quench {k + log_every}/{quench}: T_target {tb:.4f}, "
            f"<PE/N> {np.mean(logs['pe_per_particle'][-1]):.5f}, "
            f"<MSD> {np.mean(logs['msd'][-1]):.4f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["quench_wall_s"] = wall
    out["rate"] = nrep * n * quench / wall if quench else None
    out.update(logs)
    if nve > 0:
        log = s.step(nve, log_every=1)
        out["nve_E_per_particle"] = (log["E"] / n).tolist()
    s.close()
    return out


def one_at_a_time_rate(nrep: int, n: int, *, seed: int = 5, T: float = 2.0, steps: int = 200,
                       dt: float = 0.005, skin: float = 0.3):
    """Particle-steps/s of the same replicas run one after another, each in
    its own context on the plain FP64 path with direct launches (the
    reference point of the batching speedup)."""
    import torch
    import initconf
    eps, sig, rc, mass = initconf.mixture_tables()
    p = md.make_params(eps, sig, rc, mass, skin=skin, dt=dt, precision=md.MD_FP64)
    systems = initconf.batched_systems([n] * nrep, [T] * nrep, seed=seed)
    wall = 0.0
    for sy in systems:
        s = md.System(p, [n], [sy["L"]])
        s.set_state(sy["x"], sy["v"], sy["type"])
        s.step(20, T0=T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, T0=T)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        s.close()
    return nrep * n * steps / wall


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--n", type=int, default=131072)
    ap.add_argument("--equil", type=int, default=10000)
    ap.add_argument("--quench", type=int, default=100000)
    ap.add_argument("--log-every", type=int, default=1000)
    ap.add_argument("--nve", type=int, default=0)
    ap.add_argument("--precision", type=int, default=md.MD_MIXED)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--one-at-a-time-steps", type=int, default=0,
                    help="also time the replicas one at a time on plain FP64 (steps each)")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    res = run_quench(a.replicas, a.n, seed=a.seed, precision=a.precision, equil=a.equil,
                     quench=a.quench, log_every=a.log_every, nve=a.nve,
                     progress=lambda m: print(m, file=sys.stderr, flush=True))
    pe = np.mean(np.asarray(res["pe_per_particle"]), axis=1)
    if len(pe) >= 11:
        _, _, tg, smax, scold = caloric_slope(res["T_target"], pe)
        res["caloric_slope"] = {"T_max_slope": tg, "max_slope": smax, "slope_coldest": scold}
    if a.one_at_a_time_steps > 0:
        r1 = one_at_a_time_rate(a.replicas, a.n, seed=a.seed, steps=a.one_at_a_time_steps)
        res["one_at_a_time_fp64_rate"] = r1
        res["speedup_vs_one_at_a_time_fp64"] = res["rate"] / r1 if res["rate"] else None
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    keys = ("replicas", "n", "precision", "quench", "rate", "quench_wall_s",
            "one_at_a_time_fp64_rate", "speedup_vs_one_at_a_time_fp64", "caloric_slope")
    print(json.dumps({k: res[k] for k in keys if k in res}), flush=True)


if __name__ == "__main__":
    main()
