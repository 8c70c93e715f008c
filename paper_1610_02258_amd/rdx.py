"""Thin ctypes binding of the C ABI in ``include/rdx.h`` (``librdx.so``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  NumPy arrays are passed as host pointers; torch tensors on a
GPU are passed as device pointers together with torch's current stream.
Importing this module never falls back to anything: if ``librdx.so`` is
missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librdx.so")

STATUS = {0: "RDX_OK", -1: "RDX_EINVAL", -2: "RDX_EMESH", -3: "RDX_ENODIFF", -4: "RDX_ENOMEM",
          -5: "RDX_EOVERFLOW", -6: "RDX_EHIP", -7: "RDX_EBUDGET", -8: "RDX_ECANCELLED",
          -9: "RDX_EEVENTS", -10: "RDX_ESTATE"}

# Every function the header declares, with its ctypes signature.
_p = C.c_void_p
SIGNATURES = {
    "rdx_create": ([_p, _p, C.c_uint64, C.c_double, C.POINTER(C.c_void_p)], C.c_int),
    "rdx_destroy": ([_p], None),
    "rdx_set_counts": ([_p, _p, C.c_int, _p], C.c_int),
    "rdx_get_counts": ([_p, _p, C.c_int, _p], C.c_int),
    "rdx_set_rate_constants": ([_p, _p, C.c_int64, _p], C.c_int),
    "rdx_region_counts": ([_p, _p, C.c_int, _p], C.c_int),
    "rdx_region_counts_static": ([_p, _p, _p], C.c_int),
    "rdx_step_recorded": ([_p, C.c_int64, C.c_int64, _p, C.c_int64, C.POINTER(C.c_int64), _p], C.c_int),
    "rdx_batch_set_rate_constants": ([_p, C.c_int32, _p, C.c_int64, _p], C.c_int),
    "rdx_batch_region_counts": ([_p, C.c_int32, _p, C.c_int, _p], C.c_int),
    "rdx_run": ([_p, C.c_double, _p], C.c_int),
    "rdx_step": ([_p, C.c_int64, _p], C.c_int),
    "rdx_sync": ([_p, _p], C.c_int),
    "rdx_get_stats": ([_p, _p, _p], C.c_int),
    "rdx_get_tau": ([_p, C.POINTER(C.c_double)], C.c_int),
    "rdx_get_sizes": ([_p, _p, _p, _p], C.c_int),
    "rdx_get_geometry": ([_p, _p, _p, _p, _p, _p], C.c_int),
    "rdx_setup_geometry": ([_p, _p, C.c_double, _p, _p, _p, _p, _p, C.POINTER(C.c_double)], C.c_int),
    "rdx_save": ([_p, _p, C.POINTER(C.c_size_t), _p], C.c_int),
    "rdx_load": ([_p, _p, C.c_size_t, _p], C.c_int),
    "rdx_set_kernel_timing": ([_p, C.c_int], C.c_int),
    "rdx_get_kernel_times": ([_p, _p, C.c_int], C.c_int),
    "rdx_last_error": ([], C.c_char_p),
    "rdx_version": ([], C.c_int32),
    "rdx_selftest_philox": ([_p, _p, C.c_int64], C.c_int),
    "rdx_selftest_ln": ([_p, _p, C.c_int64], C.c_int),
    "rdx_selftest_binom": ([C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, C.c_double, C.c_int64,
                            _p], C.c_int),
    "rdx_selftest_copy": ([C.c_int64, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "rdx_set_exec_options": ([_p, _p], C.c_int),
    "rdx_get_exec_options": ([_p, _p], C.c_int),
    "rdx_batch_create": ([C.c_int32, _p, _p, _p, _p, C.POINTER(C.c_void_p)], C.c_int),
    "rdx_batch_destroy": ([_p], None),
    "rdx_batch_size": ([_p, C.POINTER(C.c_int32)], C.c_int),
    "rdx_batch_get_run_info": ([_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
    "rdx_batch_set_counts": ([_p, C.c_int32, _p, C.c_int, _p], C.c_int),
    "rdx_batch_get_counts": ([_p, C.c_int32, _p, C.c_int, _p], C.c_int),
    "rdx_batch_set_counts_all": ([_p, _p, _p], C.c_int),
    "rdx_batch_run": ([_p, _p, _p], C.c_int),
    "rdx_batch_step": ([_p, C.c_int64, _p], C.c_int),
    "rdx_batch_sync": ([_p, _p], C.c_int),
    "rdx_batch_get_stats": ([_p, C.c_int32, _p, _p], C.c_int),
    "rdx_batch_set_exec_options": ([_p, _p], C.c_int),
    "rdx_batch_get_exec_options": ([_p, _p], C.c_int),
    "rdx_server_create": ([_p, _p, C.POINTER(C.c_void_p)], C.c_int),
    "rdx_server_destroy": ([_p], None),
    "rdx_server_submit": ([_p, _p, _p, C.c_uint64, _p, C.c_double, C.c_double, C.POINTER(C.c_int64)],
                          C.c_int),
    "rdx_server_poll": ([_p, C.c_int64, _p], C.c_int),
    "rdx_server_wait": ([_p, C.c_int64, C.c_double, _p, _p], C.c_int),
    "rdx_server_cancel": ([_p, C.c_int64], C.c_int),
    "rdx_server_get_stats": ([_p, _p], C.c_int),
}


class RdxError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Loads librdx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1610_02258_amd.build` (needs hipcc)")
        # PyTorch-ROCm ships its own HIP and HSA runtimes; loading torch first
        # makes librdx.so bind to those (same sonames), so that the library, torch
        # tensors and torch streams share one runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise RdxError(status, where, lib().rdx_last_error().decode(errors="replace"))


class _Mesh(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("verts", _p), ("tets", _p),
                ("region", _p)]


class _Model(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32), ("n_regions", C.c_int32),
                ("diff_coef", _p), ("lhs", _p), ("rhs", _p), ("kcst", _p)]


class _Stats(C.Structure):
    _fields_ = [("windows", C.c_int64), ("voxel_steps", C.c_int64), ("ssa_events", C.c_int64),
                ("moves", C.c_int64), ("t", C.c_double), ("window_index", C.c_int64),
                ("face_moves", C.c_int64)]


class _ExecOptions(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("fast_grid_div", C.c_int32), ("graph_windows", C.c_int32),
                ("event_group", C.c_int32), ("event_bins", C.c_int32), ("tile_claim", C.c_int32)]


class _ServerOptions(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_runs", C.c_int32), ("tick_windows", C.c_int32),
                ("graph_windows", C.c_int32)]


class _RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("n_tets", C.c_int32), ("n_species", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("stats", _Stats)]


class _ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "cancelled", "queued",
                                         "running", "ticks", "voxel_steps", "ssa_events", "moves")] + \
               [(n, C.c_double) for n in ("busy_s", "uptime_s", "latency_p50_s", "latency_p99_s")] + \
               [("capacity_tets", C.c_int64), ("worker_s", C.c_double)]


REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class _KernelTimes(C.Structure):
    _fields_ = [("windows", C.c_int64), ("detect_ms", C.c_double), ("main_ms", C.c_double)]


@dataclass
class Stats:
    windows: int
    voxel_steps: int
    ssa_events: int
    moves: int
    t: float
    window_index: int
    face_moves: int = 0   # nonzero (tet, species, face) moves


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _stream_ptr(stream):
    """hipStream_t from None (default stream), an int, or a torch stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


def _current_device():
    """The HIP device current in torch (the one a new handle binds to), or
    None without a usable torch."""
    try:
        import torch
        return torch.cuda.current_device() if torch.cuda.is_available() else None
    except Exception:  # noqa: BLE001
        return None


def _check_device_tensor(t, dtype: str, numel: int, what: str, device=None):
    """Raises unless t is a contiguous CUDA tensor of `dtype` with `numel`
    elements on `device` (the library writes or reads exactly that many
    through its device pointer)."""
    if not _is_torch_cuda(t):
        raise TypeError(f"{what} must be a CUDA tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what} is on cuda:{t.device.index}, the handle on cuda:{device}")
    if str(t.dtype) != f"torch.{dtype}":
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")


def _marshal(mesh: dict, model: dict):
    verts = np.ascontiguousarray(mesh["verts"], np.float64)
    tets = np.ascontiguousarray(mesh["tets"], np.int32)
    region = mesh.get("region")
    region = None if region is None else np.ascontiguousarray(region, np.uint8)
    D = np.ascontiguousarray(model["D"], np.float64)
    S = D.shape[0]
    lhs = np.ascontiguousarray(model["lhs"], np.int32).reshape(-1, S)
    rhs = np.ascontiguousarray(model["rhs"], np.int32).reshape(-1, S)
    R = lhs.shape[0]
    kcst = np.ascontiguousarray(model["kcst"], np.float64)
    if R:
        kcst = kcst.reshape(-1, R)
        n_regions = kcst.shape[0]
    else:
        n_regions = kcst.shape[0] if kcst.ndim == 2 else int(model.get("n_regions", 1))
        kcst = np.zeros((n_regions, 0))
    m = _Mesh(verts.shape[0], tets.shape[0], _np_ptr(verts), _np_ptr(tets), _np_ptr(region))
    md = _Model(S, R, n_regions, _np_ptr(D), _np_ptr(lhs), _np_ptr(rhs), _np_ptr(kcst))
    keep = (verts, tets, region, D, lhs, rhs, kcst)
    return m, md, keep, int(tets.shape[0]), int(S), int(R)


def setup_geometry(mesh: dict, model: dict, tau_override: float = 0.0) -> dict:
    """Host-only set-up arrays (adjacency, couplings, tau); no GPU needed."""
    m, md, keep, T, S, R = _marshal(mesh, model)
    out = dict(nbr=np.zeros((T, 4), np.int32), g=np.zeros((T, 4)), G=np.zeros(T),
               cum=np.zeros((T, 4)), nav=np.zeros(T))
    tau = C.c_double()
    _check(lib().rdx_setup_geometry(C.byref(m), C.byref(md), float(tau_override),
                                    *[_np_ptr(out[k]) for k in ("nbr", "g", "G", "cum", "nav")],
                                    C.byref(tau)), "rdx_setup_geometry")
    out["tau"] = tau.value
    return out


class Sim:
    """One simulation: mesh + model + seed, device-resident counts.

    mesh: dict(verts [V,3] float64 m, tets [T,4] int32, region [T] uint8 | None)
    model: dict(D [S], lhs [R,S], rhs [R,S], kcst [n_regions,R])
    """

    def __init__(self, mesh: dict, model: dict, seed: int, tau_override: float = 0.0):
        L = lib()
        m, md, keep, T, S, R = _marshal(mesh, model)
        h = C.c_void_p()
        _check(L.rdx_create(C.byref(m), C.byref(md), int(seed) & (2**64 - 1), float(tau_override),
                            C.byref(h)), "rdx_create")
        self._h = h
        self.device = _current_device()
        self.T, self.S, self.R = T, S, R
        self.n_regions = int(md.n_regions)
        tau = C.c_double()
        _check(L.rdx_get_tau(h, C.byref(tau)), "rdx_get_tau")
        self.tau = tau.value
        self.seed = int(seed)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rdx_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ---------------------------------------------------------------
    def set_counts(self, counts, stream=None):
        if _is_torch_cuda(counts):
            _check_device_tensor(counts, "int32", self.S * self.T, "counts", self.device)
            _check(lib().rdx_set_counts(self._h, counts.data_ptr(), 1, _stream_ptr(stream)),
                   "rdx_set_counts")
        else:
            c = np.ascontiguousarray(counts, np.int32).reshape(self.S, self.T)
            _check(lib().rdx_set_counts(self._h, _np_ptr(c), 0, _stream_ptr(stream)), "rdx_set_counts")

    def get_counts(self, out=None, stream=None):
        if out is not None and _is_torch_cuda(out):
            _check_device_tensor(out, "int32", self.S * self.T, "out", self.device)
            _check(lib().rdx_get_counts(self._h, out.data_ptr(), 1, _stream_ptr(stream)), "rdx_get_counts")
            return out
        c = np.zeros((self.S, self.T), np.int32)
        _check(lib().rdx_get_counts(self._h, _np_ptr(c), 0, _stream_ptr(stream)), "rdx_get_counts")
        return c

    def set_rate_constants(self, kcst, stream=None):
        """Rate constants [n_regions, R] for the windows enqueued after this
        call (piecewise-constant forcing); waits for `stream`."""
        k = np.ascontiguousarray(kcst, np.float64).reshape(-1)
        _check(lib().rdx_set_rate_constants(self._h, _np_ptr(k), k.size, _stream_ptr(stream)),
               "rdx_set_rate_constants")

    def region_counts(self, out=None, stream=None):
        """Per-region molecule sums, int64 [n_regions, S].  With `out` a CUDA
        int64 tensor (e.g. one slot of a recording ring) the sums are written
        on `stream` without waiting."""
        if out is not None and _is_torch_cuda(out):
            _check_device_tensor(out, "int64", self.n_regions * self.S, "out", self.device)
            _check(lib().rdx_region_counts(self._h, out.data_ptr(), 1, _stream_ptr(stream)), "rdx_region_counts")
            return out
        c = np.zeros((self.n_regions, self.S), np.int64)
        _check(lib().rdx_region_counts(self._h, _np_ptr(c), 0, _stream_ptr(stream)), "rdx_region_counts")
        return c

    def region_counts_static(self, out, stream=None):
        """As region_counts into the CUDA int64 tensor `out` [n_regions, S],
        through the entry point that allocates nothing (a static device
        array holds the partial sums; calls on one GPU must not overlap)."""
        _check_device_tensor(out, "int64", self.n_regions * self.S, "out", self.device)
        _check(lib().rdx_region_counts_static(self._h, out.data_ptr(), _stream_ptr(stream)),
               "rdx_region_counts_static")
        return out

    def step_recorded(self, n_windows: int, every: int, ring, stream=None) -> int:
        """n_windows windows, recording per-region sums after every `every`
        of them into the CUDA int64 ring [slots, n_regions, S] (slot j mod
        slots); returns the number of records.  Does not wait."""
        if not _is_torch_cuda(ring):
            raise TypeError("the recording ring must be a CUDA tensor")
        if ring.dtype != __import__("torch").int64 or not ring.is_contiguous() or \
                tuple(ring.shape[1:]) != (self.n_regions, self.S):
            raise ValueError(f"the ring must be contiguous int64 [slots, {self.n_regions}, {self.S}]")
        if self.device is not None and ring.device.index != self.device:
            raise ValueError(f"the ring is on cuda:{ring.device.index}, the handle on cuda:{self.device}")
        n = C.c_int64()
        _check(lib().rdx_step_recorded(self._h, int(n_windows), int(every), ring.data_ptr(), int(ring.shape[0]),
                                       C.byref(n), _stream_ptr(stream)), "rdx_step_recorded")
        return n.value

    def run(self, t_end: float, stream=None):
        _check(lib().rdx_run(self._h, float(t_end), _stream_ptr(stream)), "rdx_run")

    def step(self, n_windows: int, stream=None):
        _check(lib().rdx_step(self._h, int(n_windows), _stream_ptr(stream)), "rdx_step")

    def sync(self, stream=None):
        _check(lib().rdx_sync(self._h, _stream_ptr(stream)), "rdx_sync")

    def stats(self, stream=None) -> Stats:
        st = _Stats()
        _check(lib().rdx_get_stats(self._h, C.byref(st), _stream_ptr(stream)), "rdx_get_stats")
        return Stats(st.windows, st.voxel_steps, st.ssa_events, st.moves, st.t, st.window_index, st.face_moves)

    def set_kernel_timing(self, enable: bool):
        _check(lib().rdx_set_kernel_timing(self._h, int(bool(enable))), "rdx_set_kernel_timing")

    def set_exec_options(self, autotune: bool = False, fast_grid_div: int = 1, graph_windows: int = 1,
                         event_group: int = 0, event_bins: int = 1, tile_claim: int = 0):
        o = _ExecOptions(int(bool(autotune)), int(fast_grid_div), int(graph_windows), int(event_group),
                         int(event_bins), int(tile_claim))
        _check(lib().rdx_set_exec_options(self._h, C.byref(o)), "rdx_set_exec_options")

    def exec_options(self) -> dict:
        o = _ExecOptions()
        _check(lib().rdx_get_exec_options(self._h, C.byref(o)), "rdx_get_exec_options")
        return dict(autotune=o.autotune, fast_grid_div=o.fast_grid_div, graph_windows=o.graph_windows,
                    event_group=o.event_group, event_bins=o.event_bins, tile_claim=o.tile_claim)

    def kernel_times(self, reset: bool = False) -> dict:
        kt = _KernelTimes()
        _check(lib().rdx_get_kernel_times(self._h, C.byref(kt), int(bool(reset))), "rdx_get_kernel_times")
        return dict(windows=kt.windows, detect_ms=kt.detect_ms, main_ms=kt.main_ms)

    def geometry(self) -> dict:
        T = self.T
        out = dict(nbr=np.zeros((T, 4), np.int32), g=np.zeros((T, 4)), G=np.zeros(T),
                   cum=np.zeros((T, 4)), nav=np.zeros(T))
        _check(lib().rdx_get_geometry(self._h, *[_np_ptr(out[k]) for k in ("nbr", "g", "G", "cum", "nav")]),
               "rdx_get_geometry")
        return out

    def save(self, stream=None) -> bytes:
        n = C.c_size_t(0)
        _check(lib().rdx_save(self._h, None, C.byref(n), _stream_ptr(stream)), "rdx_save")
        buf = C.create_string_buffer(n.value)
        _check(lib().rdx_save(self._h, buf, C.byref(n), _stream_ptr(stream)), "rdx_save")
        return buf.raw[: n.value]

    def load(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().rdx_load(self._h, buf, len(blob), _stream_ptr(stream)), "rdx_load")


class Batch:
    """Many independent runs advanced by the same window launches.

    runs: sequence of (mesh, model, seed) or (mesh, model, seed, tau_override);
    every model shares the species/reaction structure of the first.
    """

    def __init__(self, runs):
        L = lib()
        runs = list(runs)
        n = len(runs)
        meshes = (_Mesh * n)()
        models = (_Model * n)()
        seeds = (C.c_uint64 * n)()
        taus = (C.c_double * n)()
        self._keep = []
        self.T, self.S, self.R = [], None, None
        self.n_regions = []
        for i, r in enumerate(runs):
            mesh, model, seed = r[0], r[1], r[2]
            m, md, keep, T, S, R = _marshal(mesh, model)
            meshes[i], models[i] = m, md
            seeds[i] = int(seed) & (2**64 - 1)
            taus[i] = float(r[3]) if len(r) > 3 else 0.0
            self._keep.append(keep)
            self.T.append(T)
            self.n_regions.append(int(md.n_regions))
            self.S, self.R = S, R
        h = C.c_void_p()
        _check(L.rdx_batch_create(n, meshes, models, seeds, taus, C.byref(h)), "rdx_batch_create")
        self._h = h
        self.device = _current_device()
        self._keep = None  # the library copied the inputs
        self.n = n
        self.tau = []
        for i in range(n):
            tau = C.c_double()
            _check(L.rdx_batch_get_run_info(h, i, None, C.byref(tau)), "rdx_batch_get_run_info")
            self.tau.append(tau.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rdx_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_counts(self, i: int, counts, stream=None):
        if _is_torch_cuda(counts):
            _check_device_tensor(counts, "int32", self.S * self.T[i], "counts", self.device)
            _check(lib().rdx_batch_set_counts(self._h, i, counts.data_ptr(), 1, _stream_ptr(stream)),
                   "rdx_batch_set_counts")
        else:
            c = np.ascontiguousarray(counts, np.int32).reshape(self.S, self.T[i])
            _check(lib().rdx_batch_set_counts(self._h, i, _np_ptr(c), 0, _stream_ptr(stream)),
                   "rdx_batch_set_counts")

    def set_counts_all(self, counts, stream=None):
        """Every run's counts from device tensors (one per run), in one launch."""
        if len(counts) != len(self.T):
            raise ValueError(f"one counts tensor per run: {len(self.T)} expected, got {len(counts)}")
        for j, (c, T) in enumerate(zip(counts, self.T)):
            _check_device_tensor(c, "int32", self.S * T, f"counts[{j}]", self.device)
        ptrs = (C.c_void_p * len(counts))(*[c.data_ptr() for c in counts])
        _check(lib().rdx_batch_set_counts_all(self._h, ptrs, _stream_ptr(stream)), "rdx_batch_set_counts_all")

    def get_counts(self, i: int, out=None, stream=None):
        if out is not None and _is_torch_cuda(out):
            _check_device_tensor(out, "int32", self.S * self.T[i], "out", self.device)
            _check(lib().rdx_batch_get_counts(self._h, i, out.data_ptr(), 1, _stream_ptr(stream)),
                   "rdx_batch_get_counts")
            return out
        c = np.zeros((self.S, self.T[i]), np.int32)
        _check(lib().rdx_batch_get_counts(self._h, i, _np_ptr(c), 0, _stream_ptr(stream)), "rdx_batch_get_counts")
        return c

    def set_rate_constants(self, i: int, kcst, stream=None):
        k = np.ascontiguousarray(kcst, np.float64).reshape(-1)
        _check(lib().rdx_batch_set_rate_constants(self._h, i, _np_ptr(k), k.size, _stream_ptr(stream)),
               "rdx_batch_set_rate_constants")

    def region_counts(self, i: int, out=None, stream=None):
        if out is not None and _is_torch_cuda(out):
            _check_device_tensor(out, "int64", self.n_regions[i] * self.S, "out", self.device)
            _check(lib().rdx_batch_region_counts(self._h, i, out.data_ptr(), 1, _stream_ptr(stream)),
                   "rdx_batch_region_counts")
            return out
        c = np.zeros((self.n_regions[i], self.S), np.int64)
        _check(lib().rdx_batch_region_counts(self._h, i, _np_ptr(c), 0, _stream_ptr(stream)),
               "rdx_batch_region_counts")
        return c

    def run(self, t_end, stream=None):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t_end, np.float64), (self.n,)))
        _check(lib().rdx_batch_run(self._h, _np_ptr(t), _stream_ptr(stream)), "rdx_batch_run")

    def step(self, n_windows: int, stream=None):
        _check(lib().rdx_batch_step(self._h, int(n_windows), _stream_ptr(stream)), "rdx_batch_step")

    def sync(self, stream=None):
        _check(lib().rdx_batch_sync(self._h, _stream_ptr(stream)), "rdx_batch_sync")

    def stats(self, i: int, stream=None) -> Stats:
        st = _Stats()
        _check(lib().rdx_batch_get_stats(self._h, i, C.byref(st), _stream_ptr(stream)), "rdx_batch_get_stats")
        return Stats(st.windows, st.voxel_steps, st.ssa_events, st.moves, st.t, st.window_index, st.face_moves)

    def set_exec_options(self, autotune: bool = False, fast_grid_div: int = 1, graph_windows: int = 1,
                         event_group: int = 0, event_bins: int = 1, tile_claim: int = 0):
        o = _ExecOptions(int(bool(autotune)), int(fast_grid_div), int(graph_windows), int(event_group),
                         int(event_bins), int(tile_claim))
        _check(lib().rdx_batch_set_exec_options(self._h, C.byref(o)), "rdx_batch_set_exec_options")

    def exec_options(self) -> dict:
        o = _ExecOptions()
        _check(lib().rdx_batch_get_exec_options(self._h, C.byref(o)), "rdx_batch_get_exec_options")
        return dict(autotune=o.autotune, fast_grid_div=o.fast_grid_div, graph_windows=o.graph_windows,
                    event_group=o.event_group, event_bins=o.event_bins, tile_claim=o.tile_claim)


def _info(ri: _RequestInfo) -> dict:
    st = ri.stats
    return dict(state=REQ_STATES.get(ri.state, ri.state), status=ri.status, n_tets=ri.n_tets,
                t_submit=ri.t_submit, t_admit=ri.t_admit, t_done=ri.t_done,
                latency_s=ri.t_done - ri.t_submit,
                stats=Stats(st.windows, st.voxel_steps, st.ssa_events, st.moves, st.t, st.window_index, st.face_moves))


class Server:
    """Request loop with continuous batching over a device-memory budget.

    structure: a model dict fixing the species/reaction structure shared by
    every request."""

    def __init__(self, structure: dict, hbm_budget_bytes: int, max_runs: int = 0, tick_windows: int = 0,
                 graph_windows: int = 0):
        L = lib()
        m, md, keep, T, S, R = _marshal(_ONE_TET, structure)
        o = _ServerOptions(int(hbm_budget_bytes), int(max_runs), int(tick_windows), int(graph_windows))
        h = C.c_void_p()
        _check(L.rdx_server_create(C.byref(md), C.byref(o), C.byref(h)), "rdx_server_create")
        self._h = h
        self.S = S
        self._sizes = {}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rdx_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, mesh: dict, model: dict, seed: int, counts, t_end: float, tau_override: float = 0.0) -> int:
        m, md, keep, T, S, R = _marshal(mesh, model)
        c = np.ascontiguousarray(counts, np.int32).reshape(S, T)
        tk = C.c_int64()
        _check(lib().rdx_server_submit(self._h, C.byref(m), C.byref(md), int(seed) & (2**64 - 1), _np_ptr(c),
                                       float(t_end), float(tau_override), C.byref(tk)), "rdx_server_submit")
        self._sizes[tk.value] = (S, T)
        return tk.value

    def poll(self, ticket: int) -> dict:
        ri = _RequestInfo()
        _check(lib().rdx_server_poll(self._h, int(ticket), C.byref(ri)), "rdx_server_poll")
        return _info(ri)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        """(counts [S, T], info); raises RdxError for failed or cancelled requests."""
        S, T = self._sizes[ticket]
        out = np.zeros((S, T), np.int32)
        ri = _RequestInfo()
        _check(lib().rdx_server_wait(self._h, int(ticket), float(timeout_s), _np_ptr(out), C.byref(ri)),
               "rdx_server_wait")
        self._sizes.pop(ticket, None)
        return out, _info(ri)

    def cancel(self, ticket: int):
        _check(lib().rdx_server_cancel(self._h, int(ticket)), "rdx_server_cancel")

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().rdx_server_get_stats(self._h, C.byref(st)), "rdx_server_get_stats")
        return {n: getattr(st, n) for n, _ in _ServerStats._fields_}


_ONE_TET = dict(verts=np.array([[0, 0, 0], [1e-6, 0, 0], [0, 1e-6, 0], [0, 0, 1e-6]], np.float64),
                tets=np.array([[0, 1, 2, 3]], np.int32))


# -- device self-tests of the random layer ------------------------------------
def selftest_philox(ctr_key: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(ctr_key, np.uint32).reshape(-1, 6)
    out = np.zeros((a.shape[0], 4), np.uint32)
    _check(lib().rdx_selftest_philox(_np_ptr(a), _np_ptr(out), a.shape[0]), "rdx_selftest_philox")
    return out


def selftest_ln(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros_like(x)
    _check(lib().rdx_selftest_ln(_np_ptr(x), _np_ptr(y), x.size), "rdx_selftest_ln")
    return y


def selftest_binom(seed: int, m: int, p: float, n: int, stream_id: int = 1, window: int = 0) -> np.ndarray:
    out = np.zeros(n, np.int64)
    _check(lib().rdx_selftest_binom(seed, stream_id, window, m, p, n, _np_ptr(out)), "rdx_selftest_binom")
    return out


def selftest_copy(nbytes: int, reps: int = 20) -> float:
    """Device copy bandwidth in GB/s (read + write bytes over time)."""
    g = C.c_double()
    _check(lib().rdx_selftest_copy(int(nbytes), int(reps), C.byref(g)), "rdx_selftest_copy")
    return g.value


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "copy":
        nbytes = int(float(sys.argv[2])) if len(sys.argv) > 2 else 1 << 30
        print(f"copy {nbytes} B: {selftest_copy(nbytes):.1f} GB/s", flush=True)
