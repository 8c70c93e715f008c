"""ctypes wrapper of the serial CPU oracle (``os_oracle.c``) and of the exact
spatial SSA (``rdme_ssa.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke check
and the CPU-baseline leg of the benchmark.  The product library and its Python
binding never import this module.

The oracle follows the runtime main loop of "Parallel STEPS" (Algorithm 1,
section 2.2) with the window tau of section 2.1; see the header of
``os_oracle.c`` for the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
LIB_PAR_PATH = os.path.join(HERE, "liboracle_par.so")
SOURCES = [os.path.join(HERE, "os_oracle.c"), os.path.join(HERE, "rdme_ssa.c")]
PAR_SOURCES = [os.path.join(HERE, "os_oracle_par.c")]

OS_OK = 0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, fp contraction off), and its all-core
    build (the same source plus an OpenMP window loop)."""
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu99", "-fPIC", "-shared"]
    if force or not os.path.exists(LIB_PATH):
        subprocess.run(["gcc", *flags, "-o", LIB_PATH + ".tmp", *SOURCES, "-lm"], check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    if force or not os.path.exists(LIB_PAR_PATH):
        subprocess.run(["gcc", *flags, "-fopenmp", f"-I{HERE}", "-o", LIB_PAR_PATH + ".tmp", *PAR_SOURCES,
                        "-lm"], check=True)
        os.replace(LIB_PAR_PATH + ".tmp", LIB_PAR_PATH)
    return LIB_PATH


_lib = None
_lib_par = None


def _bind(L):
    p = C.c_void_p
    L.os_philox4x32_10.argtypes = [p, p, p]
    L.os_philox4x32_10.restype = None
    L.os_ln.argtypes = [C.c_double]
    L.os_ln.restype = C.c_double
    L.os_build.argtypes = [C.c_int32, p, C.c_int32, p, p, C.c_int32, C.c_int32, C.c_int32,
                           p, p, p, p, C.c_double, C.POINTER(C.c_void_p)]
    L.os_build.restype = C.c_int
    L.os_destroy.argtypes = [p]
    L.os_destroy.restype = None
    L.os_get_tau.argtypes = [p]
    L.os_get_tau.restype = C.c_double
    L.os_set_rates.argtypes = [p, p]
    L.os_set_rates.restype = C.c_int
    L.os_get_geometry.argtypes = [p] * 9
    L.os_get_geometry.restype = None
    L.os_run.argtypes = [p, C.c_uint64, p, p, C.c_double, p, p]
    L.os_run.restype = C.c_int
    L.os_step.argtypes = [p, C.c_uint64, p, p, C.c_int64, p, p]
    L.os_step.restype = C.c_int
    L.os_window_explicit.argtypes = [p, C.c_uint64, p, C.c_double, C.c_int64, p]
    L.os_window_explicit.restype = C.c_int
    L.os_sample_binom.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, C.c_double,
                                  C.c_int64, p]
    L.os_sample_binom.restype = None
    L.os_sample_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_int64, p, p, p]
    L.os_sample_uniforms.restype = None
    L.os_ssa_only.argtypes = [p, C.c_int32, C.c_double, C.c_uint64, C.c_uint32, p, p]
    L.os_ssa_only.restype = C.c_int64
    if hasattr(L, "rdme_direct"):  # the serial build only
        for f in (L.rdme_direct, L.rdme_tree):
            f.argtypes = [C.c_int32, C.c_int32, C.c_int32, p, p, p, p, p, p, p, p, p,
                          C.c_int32, p, p, C.c_uint64, C.c_int64]
            f.restype = C.c_int64
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def lib_par():
    """The all-core build: the serial oracle's functions plus os_step_par."""
    global _lib_par
    if _lib_par is None:
        if not os.path.exists(LIB_PAR_PATH):
            build(force=True)
        L = _bind(C.CDLL(LIB_PAR_PATH, mode=C.RTLD_LOCAL))
        p = C.c_void_p
        L.os_step_par.argtypes = [p, C.c_uint64, p, p, C.c_int64, p, p, C.c_int]
        L.os_step_par.restype = C.c_int
        L.os_max_threads.argtypes = []
        L.os_max_threads.restype = C.c_int
        _lib_par = L
    return _lib_par


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


class _Tallies(C.Structure):
    _fields_ = [("windows", C.c_int64), ("voxel_steps", C.c_int64),
                ("ssa_events", C.c_int64), ("moves", C.c_int64), ("face_moves", C.c_int64)]


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().os_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def ln(x: float) -> float:
    return lib().os_ln(float(x))


def sample_binom(seed: int, m: int, p: float, n: int, stream_id: int = 1, window: int = 0):
    out = np.zeros(n, np.int64)
    lib().os_sample_binom(seed, stream_id, window, m, p, n, _ptr(out))
    return out


def sample_uniforms(seed: int, n: int, stream_id: int = 0, tet: int = 0, window: int = 0):
    co = np.zeros(n)
    oc = np.zeros(n)
    u32 = np.zeros(n)
    lib().os_sample_uniforms(seed, stream_id, tet, window, n, _ptr(co), _ptr(oc), _ptr(u32))
    return co, oc, u32


@dataclass
class Tallies:
    windows: int = 0
    voxel_steps: int = 0
    ssa_events: int = 0
    moves: int = 0
    face_moves: int = 0   # nonzero (tet, species, face) moves


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class Instance:
    """Mesh + model + tau, and a simulation state (counts, t, window index).

    mesh: dict(verts [V,3] float64 metres, tets [T,4] int32, region [T] uint8 or None)
    model: dict(D [S], lhs [R,S], rhs [R,S], kcst [n_regions,R])
    """

    def __init__(self, mesh: dict, model: dict, seed: int, tau_override: float = 0.0,
                 parallel: bool = False):
        # parallel: the handle lives in the all-core build, whose step_parallel
        # runs the tet loop on several threads (same results bit for bit)
        L = lib_par() if parallel else lib()
        self._L = L
        self.verts = np.ascontiguousarray(mesh["verts"], np.float64)
        self.tets = np.ascontiguousarray(mesh["tets"], np.int32)
        reg = mesh.get("region")
        self.region = None if reg is None else np.ascontiguousarray(reg, np.uint8)
        self.D = np.ascontiguousarray(model["D"], np.float64)
        self.S = int(self.D.shape[0])
        self.lhs = np.ascontiguousarray(model["lhs"], np.int32).reshape(-1, self.S)
        self.rhs = np.ascontiguousarray(model["rhs"], np.int32).reshape(-1, self.S)
        self.R = int(self.lhs.shape[0])
        kc = np.ascontiguousarray(model["kcst"], np.float64)
        if self.R:
            self.kcst = kc.reshape(-1, self.R)
            self.n_regions = int(self.kcst.shape[0])
        else:
            self.n_regions = int(kc.shape[0]) if kc.ndim == 2 else int(model.get("n_regions", 1))
            self.kcst = np.zeros((self.n_regions, 0))
        self.T = int(self.tets.shape[0])
        self.seed = int(seed)
        h = C.c_void_p()
        kc = np.ascontiguousarray(self.kcst, np.float64)
        st = L.os_build(self.verts.shape[0], _ptr(self.verts), self.T, _ptr(self.tets),
                        _ptr(self.region), self.S, self.R, self.n_regions, _ptr(self.D),
                        _ptr(self.lhs), _ptr(self.rhs), _ptr(kc), float(tau_override),
                        C.byref(h))
        if st != OS_OK:
            raise OracleError(st, "build")
        self._h = h
        self.tau = L.os_get_tau(h)
        self.counts = np.zeros((self.S, self.T), np.int32)
        self.t = 0.0
        self.window = 0
        self.tallies = Tallies()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.os_destroy(h)
            self._h = None

    def geometry(self) -> dict:
        T = self.T
        out = dict(nbr=np.zeros((T, 4), np.int32), vol=np.zeros(T), area=np.zeros((T, 4)),
                   dist=np.zeros((T, 4)), g=np.zeros((T, 4)), G=np.zeros(T),
                   cum=np.zeros((T, 4)), nav=np.zeros(T))
        self._L.os_get_geometry(self._h, *[_ptr(out[k]) for k in
                                         ("nbr", "vol", "area", "dist", "g", "G", "cum", "nav")])
        return out

    def set_counts(self, counts: np.ndarray):
        c = np.ascontiguousarray(counts, np.int32).reshape(self.S, self.T)
        self.counts = c.copy()

    def set_rates(self, kcst: np.ndarray):
        """Piecewise-constant forcing: new rate constants [n_regions, R] from
        the next window on (the influx of section 3.2 changes every 1 ms)."""
        kc = np.ascontiguousarray(kcst, np.float64).reshape(self.n_regions, self.R)
        if self._L.os_set_rates(self._h, _ptr(kc)) != OS_OK:
            raise OracleError(-1, "set_rates: rate constants must be finite and >= 0")
        self.kcst = kc.copy()

    def region_counts(self) -> np.ndarray:
        """Recording (section 3.2 records per-region counts every 0.02 ms): the
        molecules of each species summed over the tets of each region, as
        int64 [n_regions, S], straight from the definition."""
        reg = np.zeros(self.T, np.int64) if self.region is None else self.region.astype(np.int64)
        out = np.zeros((self.n_regions, self.S), np.int64)
        for g in range(self.n_regions):
            out[g] = self.counts[:, reg == g].astype(np.int64).sum(axis=1)
        return out

    def reset(self, counts: np.ndarray, seed: int | None = None):
        """New realisation: counts at t = 0, window 0, optionally a new seed."""
        self.set_counts(counts)
        if seed is not None:
            self.seed = int(seed)
        self.t = 0.0
        self.window = 0
        self.tallies = Tallies()

    def _tally(self, tal: _Tallies):
        self.tallies.windows += tal.windows
        self.tallies.voxel_steps += tal.voxel_steps
        self.tallies.ssa_events += tal.ssa_events
        self.tallies.moves += tal.moves
        self.tallies.face_moves += tal.face_moves

    def run(self, t_end: float):
        t = C.c_double(self.t)
        w = C.c_int64(self.window)
        tal = _Tallies()
        st = self._L.os_run(self._h, self.seed, _ptr(self.counts), C.byref(t), float(t_end),
                          C.byref(w), C.byref(tal))
        self.t, self.window = t.value, w.value
        self._tally(tal)
        if st != OS_OK:
            raise OracleError(st, "run")
        return self.counts

    def step(self, n_windows: int):
        t = C.c_double(self.t)
        w = C.c_int64(self.window)
        tal = _Tallies()
        st = self._L.os_step(self._h, self.seed, _ptr(self.counts), C.byref(t), int(n_windows),
                           C.byref(w), C.byref(tal))
        self.t, self.window = t.value, w.value
        self._tally(tal)
        if st != OS_OK:
            raise OracleError(st, "step")
        return self.counts

    def step_parallel(self, n_windows: int, threads: int = 0):
        """As step(), the tet loop on `threads` host threads (0: all); needs
        parallel=True at construction."""
        if not hasattr(self._L, "os_step_par"):
            raise RuntimeError("step_parallel needs Instance(..., parallel=True)")
        t = C.c_double(self.t)
        w = C.c_int64(self.window)
        tal = _Tallies()
        nt = int(threads) if threads else int(self._L.os_max_threads())
        st = self._L.os_step_par(self._h, self.seed, _ptr(self.counts), C.byref(t), int(n_windows),
                                 C.byref(w), C.byref(tal), nt)
        self.t, self.window = t.value, w.value
        self._tally(tal)
        if st != OS_OK:
            raise OracleError(st, "step_parallel")
        return self.counts

    def window_explicit(self, tau_k: float, window: int):
        tal = _Tallies()
        st = self._L.os_window_explicit(self._h, self.seed, _ptr(self.counts), float(tau_k),
                                      int(window), C.byref(tal))
        self._tally(tal)
        if st != OS_OK:
            raise OracleError(st, "window")
        return self.counts

    def ssa_only(self, tet: int, tau_k: float, window: int, N: np.ndarray):
        n = np.ascontiguousarray(N, np.int32).copy()
        nbar = np.zeros(self.S)
        ev = self._L.os_ssa_only(self._h, int(tet), float(tau_k), self.seed, int(window),
                               _ptr(n), _ptr(nbar))
        return n, nbar, ev


def rdme_direct(inst: Instance, counts: np.ndarray, t_rec, seed: int,
                max_events: int = 10**9, method: str = "direct", return_events: bool = False):
    """Exact spatial SSA from ``counts`` (at t=0); returns counts at each time of
    t_rec (and the number of events with return_events).  method "direct"
    recomputes every channel per event (tiny meshes); "tree" selects through
    a sum tree of per-tet totals (same law, for timing larger meshes)."""
    geo = inst.geometry()
    c = np.ascontiguousarray(counts, np.int32).reshape(inst.S, inst.T).copy()
    t_rec = np.ascontiguousarray(t_rec, np.float64)
    rec = np.zeros((len(t_rec), inst.S, inst.T), np.int32)
    kc = np.ascontiguousarray(inst.kcst, np.float64)
    fn = {"direct": lib().rdme_direct, "tree": lib().rdme_tree}[method]
    ev = fn(inst.T, inst.S, inst.R, _ptr(geo["nbr"]), _ptr(geo["g"]),
            _ptr(inst.D), _ptr(inst.lhs), _ptr(inst.rhs), _ptr(kc),
            _ptr(inst.region), _ptr(geo["nav"]), _ptr(c), len(t_rec),
            _ptr(t_rec), _ptr(rec), seed, max_events)
    if ev < 0:
        raise OracleError(int(ev), "rdme_" + method)
    return (rec, int(ev)) if return_events else rec
