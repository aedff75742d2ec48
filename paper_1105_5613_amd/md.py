"""ctypes binding of libmd (include/md.h): argument marshalling only.

Every computation runs in the HIP kernels of libmd.so; torch is used only to
own device buffers and to name the HIP stream.  Importing this module does
not need a GPU; creating a context does, and fails loudly when libmd.so has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmd.so")
MAXT = 4

MD_OK, MD_EINVAL, MD_ENOMEM, MD_EBOX, MD_EOVERFLOW, MD_ENONFINITE, MD_EHIP, MD_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
MD_FP64, MD_MIXED = 0, 1
MD_POT_LJ, MD_POT_SOFT = 0, 1
MD_TRUNC_SHIFTED_FORCE, MD_TRUNC_SHIFT = 0, 1
MD_PATH_AUTO, MD_PATH_GATHER, MD_PATH_STAGED, MD_PATH_CELLS = 0, 1, 2, 3

EXPORTS = ["md_init", "md_init_alloc", "md_destroy", "md_last_error", "md_set_state", "md_get_state",
           "md_build_cells", "md_forces", "md_get_forces", "md_step", "md_observables",
           "md_get_cells", "md_get_neighbors", "md_replica_info", "md_profile",
           "md_profile_read", "md_list_stats", "md_autotune", "md_msd_reference", "md_msd",
           "md_rdf", "md_rdf_static"]


class MDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"md error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("ntypes", C.c_int32), ("potential", C.c_int32), ("trunc", C.c_int32),
                ("precision", C.c_int32), ("eps", C.c_double * 16), ("sig", C.c_double * 16),
                ("rc", C.c_double * 16), ("mass", C.c_double * 4), ("skin", C.c_double),
                ("dt", C.c_double), ("max_neighbors", C.c_int32), ("graph_steps", C.c_int32),
                ("tpp", C.c_int32), ("unroll", C.c_int32),
                ("path", C.c_int32), ("tile_cells", C.c_int32), ("stage_slots", C.c_int32),
                ("split_kick", C.c_int32), ("small_box", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("virial", C.c_double),
                ("T", C.c_double), ("P", C.c_double), ("E", C.c_double),
                ("max_disp", C.c_double), ("T_target", C.c_double),
                ("step", C.c_int64), ("n_rebuild", C.c_int64)]


OBS_KEYS = [f[0] for f in Obs._fields_]


class Tune(C.Structure):
    _fields_ = [("tpp", C.c_int32), ("unroll", C.c_int32), ("force_ms", C.c_double),
                ("ntried", C.c_int32), ("tried_tpp", C.c_int32 * 16),
                ("tried_unroll", C.c_int32 * 16), ("tried_ms", C.c_double * 16)]


class Prof(C.Structure):
    _fields_ = [("force_launches", C.c_int64), ("force_ms", C.c_double)]

_lib = None


def lib():
    """Load libmd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1105_5613_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip, lp = C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)
        L.md_init.argtypes = [C.POINTER(C.c_void_p), C.POINTER(Params), C.c_int32,
                              lp, C.POINTER(C.c_double), vp]
        L.md_init_alloc.argtypes = [C.POINTER(C.c_void_p), C.POINTER(Params), C.c_int32,
                                    lp, C.POINTER(C.c_double), vp, C.POINTER(Allocator)]
        L.md_destroy.argtypes = [vp]
        L.md_last_error.argtypes = [vp]
        L.md_last_error.restype = C.c_char_p
        L.md_set_state.argtypes = [vp, dp, dp, ip]
        L.md_get_state.argtypes = [vp, dp, dp, ip]
        L.md_build_cells.argtypes = [vp]
        L.md_forces.argtypes = [vp]
        L.md_get_forces.argtypes = [vp, vp]
        L.md_step.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_int64, C.POINTER(Obs), C.c_int32]
        L.md_observables.argtypes = [vp, C.POINTER(Obs)]
        L.md_get_cells.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.md_get_neighbors.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.c_int32]
        L.md_replica_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double), lp, lp, C.POINTER(C.c_int32)]
        L.md_profile.argtypes = [vp, C.c_int32]
        L.md_profile_read.argtypes = [vp, C.POINTER(Prof)]
        L.md_list_stats.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.md_autotune.argtypes = [vp, C.c_int32, C.POINTER(Tune)]
        L.md_msd_reference.argtypes = [vp]
        L.md_msd.argtypes = [vp, C.POINTER(C.c_double)]
        L.md_rdf.argtypes = [vp, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_double)]
        L.md_rdf_static.argtypes = [vp, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_double)]
        for name in EXPORTS:
            if name != "md_last_error":
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def make_params(eps, sig, rc, mass, *, skin=0.3, dt=0.005, precision=MD_FP64,
                potential=MD_POT_LJ, trunc=MD_TRUNC_SHIFTED_FORCE, max_neighbors=0,
                graph_steps=0, tpp=0, unroll=0, path=MD_PATH_AUTO, tile_cells=0,
                stage_slots=0, split_kick=0, small_box=0) -> Params:
    p = Params()
    nt = len(eps)
    p.ntypes = nt
    p.potential = potential
    p.trunc = trunc
    p.precision = precision
    for a in range(nt):
        for b in range(nt):
            p.eps[a * MAXT + b] = float(eps[a][b])
            p.sig[a * MAXT + b] = float(sig[a][b])
            p.rc[a * MAXT + b] = float(rc[a][b])
        p.mass[a] = float(mass[a])
    p.skin = float(skin)
    p.dt = float(dt)
    p.max_neighbors = int(max_neighbors)
    p.graph_steps = int(graph_steps)
    p.tpp = int(tpp)
    p.unroll = int(unroll)
    p.path = int(path)
    p.tile_cells = int(tile_cells)
    p.stage_slots = int(stage_slots)
    p.split_kick = int(split_kick)
    p.small_box = int(small_box)
    return p


def _obs_dict(o: Obs):
    return {k: getattr(o, k) for k in OBS_KEYS}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """md_allocator: alloc(u, bytes, stream), free(u, ptr, stream), u."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("u", C.c_void_p)]


class TorchAllocator:
    """Device buffers of a context from torch's caching allocator: each block
    is a uint8 CUDA tensor allocated on the context's stream and kept alive
    until the library frees it (after synchronising that stream)."""

    def __init__(self, stream):
        import torch
        self._torch = torch
        self._stream = stream
        self.blocks = {}

        def _alloc(u, nbytes, hip_stream):
            with self._torch.cuda.stream(self._stream):
                t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device="cuda")
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(u, ptr, stream):
            self.blocks.pop(ptr, None)

        self._fns = (ALLOC_FN(_alloc), FREE_FN(_free))  # keep the thunks alive
        self.struct = Allocator(self._fns[0], self._fns[1], None)

    def bytes_held(self):
        return sum(t.numel() for t in self.blocks.values())


class System:
    """One md context: nrep replicas (sizes ``n``, box sides ``L``).  With
    ``allocator="torch"`` the context's device buffers come from torch's
    caching allocator (md_init_alloc), otherwise from hipMalloc."""

    def __init__(self, params: Params, n, L, stream=None, allocator=None):
        import torch
        self._torch = torch
        n = [int(v) for v in (n if hasattr(n, "__len__") else [n])]
        L = [float(v) for v in (L if hasattr(L, "__len__") else [L])]
        self.params = params
        self.n = n
        self.L = L
        self.nrep = len(n)
        self.ntot = sum(n)
        self.device = torch.device("cuda", torch.cuda.current_device())
        st = torch.cuda.current_stream() if stream is None else stream
        self.stream = st
        h = C.c_void_p()
        na = (C.c_int64 * self.nrep)(*n)
        La = (C.c_double * self.nrep)(*L)
        self.allocator = None
        if allocator == "torch":
            self.allocator = TorchAllocator(st)
            rc = lib().md_init_alloc(C.byref(h), C.byref(params), self.nrep, na, La,
                                     C.c_void_p(st.cuda_stream), C.byref(self.allocator.struct))
        elif allocator is None:
            rc = lib().md_init(C.byref(h), C.byref(params), self.nrep, na, La,
                               C.c_void_p(st.cuda_stream))
        else:
            raise ValueError("allocator must be None or 'torch'")
        if rc != MD_OK:
            raise MDError(rc, lib().md_last_error(None).decode())
        self._h = h

    def _check(self, rc):
        if rc != MD_OK:
            raise MDError(rc, lib().md_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().md_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state -------------------------------------------------------------------
    def set_state(self, x, v, types):
        t = self._torch
        x = t.as_tensor(x, dtype=t.float64, device=self.device).contiguous()
        v = t.as_tensor(v, dtype=t.float64, device=self.device).contiguous()
        ty = t.as_tensor(types, dtype=t.int32, device=self.device).contiguous()
        assert x.shape == (self.ntot, 3) and v.shape == (self.ntot, 3) and ty.shape == (self.ntot,)
        self._check(lib().md_set_state(self._h, x.data_ptr(), v.data_ptr(), ty.data_ptr()))

    def get_state(self):
        t = self._torch
        x = t.empty((self.ntot, 3), dtype=t.float64, device=self.device)
        v = t.empty_like(x)
        img = t.empty((self.ntot, 3), dtype=t.int32, device=self.device)
        self._check(lib().md_get_state(self._h, x.data_ptr(), v.data_ptr(), img.data_ptr()))
        return x, v, img

    def build_cells(self):
        self._check(lib().md_build_cells(self._h))

    def forces(self):
        self._check(lib().md_forces(self._h))

    def get_forces(self):
        t = self._torch
        dt = t.float32 if self.params.precision == MD_MIXED else t.float64
        F = t.empty((self.ntot, 3), dtype=dt, device=self.device)
        self._check(lib().md_get_forces(self._h, F.data_ptr()))
        return F

    def step(self, nsteps, T0=None, T1=None, ramp=0, log_every=0):
        """Advance nsteps; returns a dict of [nlog][nrep] arrays when log_every > 0."""
        t0 = t1 = None
        if T0 is not None:
            T0 = list(np.broadcast_to(np.asarray(T0, dtype=np.float64), (self.nrep,)))
            t0 = (C.c_double * self.nrep)(*T0)
            if T1 is not None:
                T1 = list(np.broadcast_to(np.asarray(T1, dtype=np.float64), (self.nrep,)))
                t1 = (C.c_double * self.nrep)(*T1)
        logbuf = None
        nlog = 0
        if log_every > 0:
            nlog = nsteps // log_every
            logbuf = (Obs * max(nlog * self.nrep, 1))()
        self._check(lib().md_step(self._h, int(nsteps), t0, t1, int(ramp), logbuf,
                                  int(log_every)))
        if logbuf is None:
            return None
        out = {}
        for k in OBS_KEYS:
            a = np.array([getattr(logbuf[i], k) for i in range(nlog * self.nrep)])
            out[k] = a.reshape(nlog, self.nrep)
        return out

    def observables(self):
        buf = (Obs * self.nrep)()
        self._check(lib().md_observables(self._h, buf))
        return [_obs_dict(buf[r]) for r in range(self.nrep)]

    # -- parity hooks ----------------------------------------------------------------
    def replica_info(self, rep=0):
        nc, inv = C.c_int32(), C.c_double()
        n, off, cap = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(lib().md_replica_info(self._h, rep, C.byref(nc), C.byref(inv), C.byref(n),
                                          C.byref(off), C.byref(cap)))
        return {"nc": nc.value, "inv_cell": inv.value, "n": n.value, "offset": off.value,
                "max_neighbors": cap.value}

    def get_cells(self, rep=0):
        info = self.replica_info(rep)
        nc, n = info["nc"], info["n"]
        cs = np.zeros(nc ** 3 + 1, np.int32)
        order = np.zeros(n, np.int32)
        self._check(lib().md_get_cells(self._h, rep, cs.ctypes.data_as(C.POINTER(C.c_int32)),
                                       order.ctypes.data_as(C.POINTER(C.c_int32))))
        return cs, order

    def get_neighbors(self, rep=0, cap=None):
        info = self.replica_info(rep)
        n = info["n"]
        cap = info["max_neighbors"] if cap is None else cap
        count = np.zeros(n, np.int32)
        ids = np.full((n, cap), -1, np.int32)
        self._check(lib().md_get_neighbors(self._h, rep,
                                           count.ctypes.data_as(C.POINTER(C.c_int32)),
                                           ids.ctypes.data_as(C.POINTER(C.c_int32)), cap))
        return count, ids

    # -- measurement -------------------------------------------------------------
    def profile(self, every):
        """Bracket the force launch of every ``every``-th step with hipEvents."""
        self._check(lib().md_profile(self._h, int(every)))

    def profile_read(self):
        pr = Prof()
        self._check(lib().md_profile_read(self._h, C.byref(pr)))
        return {"force_launches": pr.force_launches, "force_ms": pr.force_ms}

    def list_stats(self, rep=-1):
        mean, mx = C.c_double(), C.c_int32()
        self._check(lib().md_list_stats(self._h, rep, C.byref(mean), C.byref(mx)))
        return mean.value, mx.value

    def autotune(self, reps=5):
        """Pick the fastest force-kernel variant on the current state (md_autotune)."""
        t = Tune()
        self._check(lib().md_autotune(self._h, int(reps), C.byref(t)))
        return {"tpp": t.tpp, "unroll": t.unroll, "force_ms": t.force_ms,
                "tried": [(t.tried_tpp[k], t.tried_unroll[k], t.tried_ms[k])
                          for k in range(t.ntried)]}

    # -- glass-study observables -------------------------------------------------
    def msd_reference(self):
        self._check(lib().md_msd_reference(self._h))

    def msd(self):
        out = (C.c_double * self.nrep)()
        self._check(lib().md_msd(self._h, out))
        return np.array(out[:])

    def rdf(self, rep=0, rmax=4.0, nbins=400):
        g = np.zeros(nbins)
        self._check(lib().md_rdf(self._h, rep, float(rmax), int(nbins),
                                 g.ctypes.data_as(C.POINTER(C.c_double))))
        return g
