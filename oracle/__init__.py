"""FP64 CPU oracle for the short-range MD hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It is an independent plain implementation of
what the HIP library computes and shares no code with it (see mdref.h for
the passages of arXiv:1105.5613 each function follows).

The C source is compiled with gcc ``-O2 -ffp-contract=off -fopenmp`` into
``oracle/libmdref.so``; ``build()`` (re)compiles it, ``lib()`` loads it and
builds it first when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdref.c")
# MDREF_LIB selects another build of the same source (the sanitizer build)
LIB = os.environ.get("MDREF_LIB") or os.path.join(HERE, "libmdref.so")
SAN_LIB = os.path.join(HERE, "libmdref_san.so")
MAXT = 4

_lib = None


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile libmdref.so with gcc (no FMA contraction, no fast-math).

    sanitize=True builds libmdref_san.so instead, instrumented with
    AddressSanitizer and UndefinedBehaviorSanitizer (every finding fatal);
    a process loads it with the sanitizer runtimes preloaded.
    """
    out = SAN_LIB if sanitize else os.path.join(HERE, "libmdref.so")
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-Werror",
           "-Wno-unused-parameter", *san, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class Params(C.Structure):
    _fields_ = [("ntypes", C.c_int32), ("potential", C.c_int32),
                ("trunc", C.c_int32), ("pad", C.c_int32),
                ("eps", C.c_double * 16), ("sig", C.c_double * 16),
                ("rc", C.c_double * 16), ("mass", C.c_double * 4),
                ("skin", C.c_double)]


class Obs(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("w", C.c_double),
                ("T", C.c_double), ("P", C.c_double), ("E", C.c_double),
                ("max_disp2", C.c_double), ("step", C.c_int64),
                ("rebuilt", C.c_int32), ("pad", C.c_int32)]


def make_params(eps, sig, rc, mass, *, skin=0.3, potential=0, trunc=0) -> Params:
    """Build an oracle parameter block from nested [a][b] tables."""
    p = Params()
    nt = len(eps)
    p.ntypes = nt
    p.potential = potential
    p.trunc = trunc
    for a in range(nt):
        for b in range(nt):
            p.eps[a * MAXT + b] = float(eps[a][b])
            p.sig[a * MAXT + b] = float(sig[a][b])
            p.rc[a * MAXT + b] = float(rc[a][b])
    for a in range(nt):
        p.mass[a] = float(mass[a])
    p.skin = float(skin)
    return p


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        pp = C.POINTER(Params)
        L.mdref_v.restype = C.c_double
        L.mdref_v.argtypes = [pp, C.c_int32, C.c_int32, C.c_double]
        L.mdref_dv.restype = C.c_double
        L.mdref_dv.argtypes = [pp, C.c_int32, C.c_int32, C.c_double]
        L.mdref_pair.argtypes = [pp, C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.mdref_forces_brute.argtypes = [pp, C.c_int64, C.c_double, dp, ip, dp, dp, dp]
        L.mdref_cell_grid.argtypes = [pp, C.c_double, ip, dp]
        L.mdref_build_cells.argtypes = [C.c_int64, C.c_double, C.c_int32, C.c_double,
                                        dp, ip, ip, ip, ip]
        L.mdref_build_nlist.argtypes = [pp, C.c_int64, C.c_double, C.c_int32, dp, ip,
                                        ip, ip, ip, C.c_int32, ip, ip]
        L.mdref_forces_list.argtypes = [pp, C.c_int64, C.c_double, dp, ip, C.c_int32,
                                        ip, ip, dp, dp, dp]
        L.mdref_forces_cells.argtypes = [pp, C.c_int64, C.c_double, C.c_int32, dp, ip,
                                         ip, ip, ip, C.c_int64, lp, dp, dp, dp]
        L.mdref_rdf.argtypes = [C.c_int64, C.c_double, dp, C.c_double, C.c_int32, dp]
        L.mdref_sim_create.restype = C.c_void_p
        L.mdref_sim_create.argtypes = [pp, C.c_int64, C.c_double, C.c_double, C.c_int32]
        L.mdref_sim_destroy.argtypes = [C.c_void_p]
        L.mdref_sim_set_state.argtypes = [C.c_void_p, dp, dp, ip]
        L.mdref_sim_get_state.argtypes = [C.c_void_p, dp, dp, ip]
        L.mdref_sim_get_forces.argtypes = [C.c_void_p, dp, dp, dp]
        L.mdref_sim_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                     C.c_double, C.c_int64, C.POINTER(Obs)]
        L.mdref_sim_rebuilds.restype = C.c_int64
        L.mdref_sim_rebuilds.argtypes = [C.c_void_p]
        L.mdref_set_threads.argtypes = [C.c_int32]
        L.mdref_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops (timing only)."""
    lib().mdref_set_threads(int(n))


def max_threads() -> int:
    return int(lib().mdref_max_threads())


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---- pair functions (Eq. 1-3) ------------------------------------------------
def v(p: Params, a: int, b: int, r: float) -> float:
    return lib().mdref_v(C.byref(p), a, b, r)


def dv(p: Params, a: int, b: int, r: float) -> float:
    return lib().mdref_dv(C.byref(p), a, b, r)


def pair(p: Params, a: int, b: int, r: float):
    vs, f = C.c_double(), C.c_double()
    lib().mdref_pair(C.byref(p), a, b, r, C.byref(vs), C.byref(f))
    return vs.value, f.value


# ---- forces ----------------------------------------------------------------
def forces_brute(p: Params, x, types, L: float):
    x = _f64(x, (-1, 3))
    t = _i32(types)
    n = x.shape[0]
    F = np.zeros((n, 3))
    pe, w = C.c_double(), C.c_double()
    rc = lib().mdref_forces_brute(C.byref(p), n, L, _ptr(x, C.c_double), _ptr(t, C.c_int32),
                                  _ptr(F, C.c_double), C.byref(pe), C.byref(w))
    if rc:
        raise ValueError(f"mdref_forces_brute failed ({rc})")
    return F, pe.value, w.value


def cell_grid(p: Params, L: float):
    nc, inv = C.c_int32(), C.c_double()
    if lib().mdref_cell_grid(C.byref(p), L, C.byref(nc), C.byref(inv)):
        raise ValueError("bad params")
    return nc.value, inv.value


def build_cells(p: Params, x, L: float, img=None):
    """Returns (x_wrapped, img, cell, cell_start, order, nc)."""
    nc, inv = cell_grid(p, L)
    xw = _f64(x, (-1, 3)).copy()
    n = xw.shape[0]
    im = np.zeros((n, 3), np.int32) if img is None else _i32(img).copy()
    cell = np.zeros(n, np.int32)
    cs = np.zeros(nc ** 3 + 1, np.int32)
    order = np.zeros(n, np.int32)
    rc = lib().mdref_build_cells(n, L, nc, inv, _ptr(xw, C.c_double), _ptr(im, C.c_int32),
                                 _ptr(cell, C.c_int32), _ptr(cs, C.c_int32),
                                 _ptr(order, C.c_int32))
    if rc:
        raise ValueError(f"mdref_build_cells failed ({rc})")
    return xw, im, cell, cs, order, nc


def build_nlist(p: Params, xw, types, L: float, cell, cell_start, order, nc: int, cap=None):
    """Full neighbour list on wrapped positions. Returns (count, ids[n][cap])."""
    xw = _f64(xw, (-1, 3))
    t = _i32(types)
    n = xw.shape[0]
    cap = 192 if cap is None else cap
    while True:
        count = np.zeros(n, np.int32)
        ids = np.full((n, cap), -1, np.int32)
        rc = lib().mdref_build_nlist(C.byref(p), n, L, nc, _ptr(xw, C.c_double),
                                     _ptr(t, C.c_int32), _ptr(_i32(cell), C.c_int32),
                                     _ptr(_i32(cell_start), C.c_int32),
                                     _ptr(_i32(order), C.c_int32), cap,
                                     _ptr(count, C.c_int32), _ptr(ids, C.c_int32))
        if rc < 0:
            raise ValueError(f"mdref_build_nlist failed ({rc})")
        if rc == 0:
            return count, ids
        cap = int(count.max()) + 8


def forces_list(p: Params, xw, types, L: float, count, ids):
    xw = _f64(xw, (-1, 3))
    n = xw.shape[0]
    ids = _i32(ids)
    cap = ids.shape[1]
    F = np.zeros((n, 3))
    pe, w = C.c_double(), C.c_double()
    rc = lib().mdref_forces_list(C.byref(p), n, L, _ptr(xw, C.c_double),
                                 _ptr(_i32(types), C.c_int32), cap,
                                 _ptr(_i32(count), C.c_int32), _ptr(ids, C.c_int32),
                                 _ptr(F, C.c_double), C.byref(pe), C.byref(w))
    if rc:
        raise ValueError(f"mdref_forces_list failed ({rc})")
    return F, pe.value, w.value


def forces_cells(p: Params, x, types, L: float, sel=None):
    """Forces (and per-particle PE/W halves) straight from the cell list.

    ``x`` is any in-range state; it is wrapped with the oracle's rule first.
    ``sel``: optional particle ids.  Returns (F[nsel][3], pe_i, w_i).
    """
    xw, _, cell, cs, order, nc = build_cells(p, x, L)
    n = xw.shape[0]
    t = _i32(types)
    if sel is None:
        nsel, sp = n, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        nsel, sp = sel.shape[0], _ptr(sel, C.c_int64)
    F = np.zeros((nsel, 3))
    pe = np.zeros(nsel)
    w = np.zeros(nsel)
    rc = lib().mdref_forces_cells(C.byref(p), n, L, nc, _ptr(xw, C.c_double),
                                  _ptr(t, C.c_int32), _ptr(cell, C.c_int32),
                                  _ptr(cs, C.c_int32), _ptr(order, C.c_int32),
                                  nsel, sp, _ptr(F, C.c_double), _ptr(pe, C.c_double),
                                  _ptr(w, C.c_double))
    if rc:
        raise ValueError(f"mdref_forces_cells failed ({rc})")
    return F, pe, w


def rdf(x, L: float, rmax: float, nbins: int):
    x = _f64(x, (-1, 3))
    g = np.zeros(nbins)
    rc = lib().mdref_rdf(x.shape[0], L, _ptr(x, C.c_double), rmax, nbins, _ptr(g, C.c_double))
    if rc:
        raise ValueError("mdref_rdf failed")
    return g


class Sim:
    """Velocity-Verlet simulation of one periodic box (O(N^2) or list mode)."""

    def __init__(self, p: Params, n: int, L: float, dt: float, brute: bool = False):
        self.p, self.n, self.L, self.dt = p, n, L, dt
        self._h = lib().mdref_sim_create(C.byref(p), n, L, dt, 1 if brute else 0)
        if not self._h:
            raise ValueError("mdref_sim_create failed (box smaller than 2*(rc+skin)?)")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().mdref_sim_destroy(h)
            self._h = None

    def set_state(self, x, v, types):
        x = _f64(x, (-1, 3))
        v = _f64(v, (-1, 3))
        t = _i32(types)
        if lib().mdref_sim_set_state(self._h, _ptr(x, C.c_double), _ptr(v, C.c_double),
                                     _ptr(t, C.c_int32)):
            raise ValueError("bad species")

    def get_state(self):
        x = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        img = np.zeros((self.n, 3), np.int32)
        lib().mdref_sim_get_state(self._h, _ptr(x, C.c_double), _ptr(v, C.c_double),
                                  _ptr(img, C.c_int32))
        return x, v, img

    def forces(self):
        F = np.zeros((self.n, 3))
        pe, w = C.c_double(), C.c_double()
        rc = lib().mdref_sim_get_forces(self._h, _ptr(F, C.c_double), C.byref(pe), C.byref(w))
        if rc:
            raise ValueError(f"forces failed ({rc})")
        return F, pe.value, w.value

    def step(self, nsteps: int, T0=None, T1=None, ramp: int = 0):
        obs = (Obs * max(nsteps, 1))()
        therm = 0 if T0 is None else 1
        t0 = 0.0 if T0 is None else float(T0)
        t1 = t0 if T1 is None else float(T1)
        rc = lib().mdref_sim_step(self._h, nsteps, therm, t0, t1, ramp, obs)
        if rc:
            raise ValueError(f"mdref_sim_step failed ({rc})")
        keys = ["ke", "pe", "w", "T", "P", "E", "max_disp2", "step", "rebuilt"]
        return {k: np.array([getattr(obs[i], k) for i in range(nsteps)]) for k in keys}

    def rebuilds(self) -> int:
        return int(lib().mdref_sim_rebuilds(self._h))


def canonical_lists(count, ids):
    """Per-particle sorted id rows (list order is not part of the contract)."""
    return [np.sort(ids[i, :count[i]]) for i in range(len(count))]
