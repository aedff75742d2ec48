"""Seeded synthetic initial configurations for the binary Lennard-Jones mixture.

This module only draws inputs: lattice sites, jitter, species labels and
Maxwell velocities.  It holds none of the molecular-dynamics arithmetic
(no potential, no force, no temperature definition, no wrap rule); both the
FP64 CPU oracle and the HIP library receive the exact same arrays from here.

Workload shapes follow the paper's test system (binary mixture at number
density 1.2 with species tensors eps/sigma, "The BBMD scaling results"
section) with the Lennard-Jones form of Eq. (1) and the per-pair cutoff
2.5*sigma_ab used by the configurations this repository measures.

Randomness: numpy's Philox4x32-10 counter-based bit generator (Salmon et
al., SC'11) keyed by an integer seed; replica r of a batch uses key
(seed << 20) + r so replicas are independent streams.
"""
from __future__ import annotations

import math

import numpy as np

# Species tensors of the mixture (A = type 0, B = type 1).  Values are the
# ones listed for the paper's benchmark mixture.
MIXTURE = {
    "ntypes": 2,
    "eps": [[1.0, 1.5], [1.5, 0.5]],
    "sig": [[1.0, 0.8], [0.8, 0.88]],
    "mass": [1.0, 1.0],
    "rc_over_sigma": 2.5,
}

DENSITY = 1.2
FRACTION_A = 0.8


def mixture_tables(rc_over_sigma: float = 2.5, global_rc: float | None = None):
    """Return (eps, sig, rc, mass) as nested lists for the two-species mixture.

    rc[a][b] = rc_over_sigma * sig[a][b] unless ``global_rc`` is given.
    """
    eps = [row[:] for row in MIXTURE["eps"]]
    sig = [row[:] for row in MIXTURE["sig"]]
    if global_rc is None:
        rc = [[rc_over_sigma * s for s in row] for row in sig]
    else:
        rc = [[float(global_rc)] * 2 for _ in range(2)]
    return eps, sig, rc, list(MIXTURE["mass"])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def box_length(n: int, rho: float = DENSITY) -> float:
    """Cubic box side for n particles at number density rho."""
    return float((n / rho) ** (1.0 / 3.0))


def fcc_system(n: int, *, rho: float = DENSITY, temperature: float = 2.0,
               seed: int = 1, frac_a: float = FRACTION_A, jitter: float = 0.05,
               sigma_aa: float = 1.0):
    """FCC lattice + uniform jitter, shuffled species, Maxwell velocities.

    Returns dict with x (n,3) float64 in [0, L), v (n,3) float64 with zero
    total momentum (unit masses), type (n,) int32 and L.

    * lattice: m cells per side with m = ceil((n/4)^(1/3)); when 4 m^3 > n
      a seeded subset of n sites is kept (vacancies keep rho exact);
    * jitter: every coordinate += U[-jitter, jitter) * sigma_aa;
    * species: the first round(frac_a*n) particles are A, then a seeded
      permutation of the labels;
    * velocities: each component ~ Normal(0, sqrt(T)) (unit mass), then
      the mean is subtracted.
    """
    if n <= 0:
        raise ValueError("n must be positive")
    rng = _rng(seed)
    L = box_length(n, rho)
    m = int(round((n / 4.0) ** (1.0 / 3.0)))
    if 4 * m ** 3 < n:
        m += 1
    while 4 * (m - 1) ** 3 >= n and m > 1:
        m -= 1
    a = L / m
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0],
                      [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    nsites = 4 * m ** 3
    if nsites == n:
        site = np.arange(n, dtype=np.int64)
    else:
        site = np.sort(rng.permutation(nsites)[:n]).astype(np.int64)
    cell = site // 4
    b = site % 4
    ix = cell % m
    iy = (cell // m) % m
    iz = cell // (m * m)
    x = np.empty((n, 3), dtype=np.float64)
    x[:, 0] = (ix + basis[b, 0]) * a
    x[:, 1] = (iy + basis[b, 1]) * a
    x[:, 2] = (iz + basis[b, 2]) * a
    x += rng.uniform(-jitter, jitter, size=(n, 3)) * sigma_aa
    x = np.mod(x, L)
    x[x >= L] = 0.0
    na = int(round(frac_a * n))
    types = np.ones(n, dtype=np.int32)
    types[:na] = 0
    types = types[rng.permutation(n)].astype(np.int32)
    v = rng.normal(0.0, math.sqrt(temperature), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    return {"x": np.ascontiguousarray(x), "v": np.ascontiguousarray(v),
            "type": np.ascontiguousarray(types), "L": L, "n": n,
            "seed": seed, "temperature": temperature}


def uniform_positions(n: int, L: float, seed: int = 1) -> np.ndarray:
    """n positions drawn uniformly from the cube [0, L)^3 (an ideal gas)."""
    return _rng(seed).random((n, 3)) * L


def replica_sizes(nrep: int, nmin: int = 1000, nmax: int = 65536, seed: int = 4):
    """Log-uniform sizes N_r = round(exp(U[ln nmin, ln nmax]))."""
    rng = _rng(seed)
    u = rng.uniform(math.log(nmin), math.log(nmax), size=nrep)
    return [int(round(math.exp(t))) for t in u]


def replica_temperatures(nrep: int, tmin: float = 0.4, tmax: float = 2.0, seed: int = 4):
    rng = _rng((seed << 20) + 0xFFFFF)
    return [float(t) for t in rng.uniform(tmin, tmax, size=nrep)]


def batched_systems(sizes, temperatures, *, seed: int = 4, rho: float = DENSITY):
    """Independent replicas; replica r is drawn with key (seed<<20)+r."""
    out = []
    for r, (n, t) in enumerate(zip(sizes, temperatures)):
        out.append(fcc_system(int(n), rho=rho, temperature=float(t),
                              seed=(seed << 20) + r))
    return out


def concat_replicas(systems):
    """Stack replicas into the [sum N][3] layout used by the batched calls."""
    x = np.concatenate([s["x"] for s in systems], axis=0)
    v = np.concatenate([s["v"] for s in systems], axis=0)
    t = np.concatenate([s["type"] for s in systems], axis=0)
    return (np.ascontiguousarray(x), np.ascontiguousarray(v),
            np.ascontiguousarray(t.astype(np.int32)),
            [int(s["n"]) for s in systems], [float(s["L"]) for s in systems])


# Named workloads (sizes and settings of the measured configurations).
WORKLOADS = {
    "lj4k_fp64": dict(n=4000, temperature=2.0, dt=0.005, skin=0.3, steps=100, seed=1),
    "lj1m": dict(n=1048576, temperature=2.0, dt=0.005, skin=0.3, steps=1000, seed=2),
    "lj67m_mixed": dict(n=67108864, temperature=2.0, dt=0.005, skin=0.3, steps=200, seed=3),
    "replicas256": dict(nrep=256, nmin=1000, nmax=65536, tmin=0.4, tmax=2.0,
                        dt=0.005, skin=0.3, steps=2000, seed=4),
    "quench64x131k": dict(nrep=64, n=131072, t_hot=2.0, t_cold=0.3, equil=10000,
                          ramp=100000, dt=0.005, skin=0.3, seed=5),
}
