"""Python binding of libmgx.so (ctypes; argument marshalling only).

Every step of the radiative transfer path runs in the library's HIP kernels.
PyTorch, when present, supplies the HIP stream (torch's current stream) and
device tensors may be passed wherever the C ABI accepts host or device
pointers.  There is no fallback: if the library is missing this module
raises on import of the library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgx.so")

MGX_OK, MGX_EINVAL, MGX_ESTATE, MGX_ENOMEM, MGX_EHIP = 0, -1, -2, -3, -4
MGX_ENOCONV, MGX_ESINGULAR, MGX_ENONFINITE, MGX_EPENDING = -5, -6, -7, -8
FP64, FP32 = 0, 1
NG_NONE, NG_CLASSICAL, NG_ADAPTIVE = 0, 1, 2
# or'ed into an Ng mode: after a used prediction only later regular iterates
# are stored
NG_FRESH = 0x10

_STATUS = {0: "MGX_OK", -1: "MGX_EINVAL", -2: "MGX_ESTATE", -3: "MGX_ENOMEM", -4: "MGX_EHIP",
           -5: "MGX_ENOCONV", -6: "MGX_ESINGULAR", -7: "MGX_ENONFINITE", -8: "MGX_EPENDING"}
REQ_CONVERGE, REQ_RENDER = 0, 1


class MgxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("branch_threshold", C.c_double),
                ("tau_floor", C.c_double), ("chi_min", C.c_double), ("pop_floor", C.c_double),
                ("trace_slot_min_bytes", C.c_int64)]


class ModelStruct(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("npoints", C.c_int), ("pos", C.c_void_p), ("vel", C.c_void_p),
        ("nbs_off", C.c_void_p), ("nbs", C.c_void_p), ("bdy", C.c_void_p), ("T", C.c_void_p),
        ("vturb2", C.c_void_p), ("nspec", C.c_void_p), ("ncoll", C.c_void_p),
        ("nrays", C.c_int), ("ray_dir", C.c_void_p), ("ray_w", C.c_void_p),
        ("antipode", C.c_void_p), ("mass", C.c_double), ("nlev", C.c_int), ("E", C.c_void_p),
        ("g", C.c_void_p), ("nlines", C.c_int), ("up", C.c_void_p), ("lo", C.c_void_p),
        ("A", C.c_void_p), ("nu", C.c_void_p), ("ncoll_tr", C.c_int), ("cu", C.c_void_p),
        ("cl", C.c_void_p), ("K0", C.c_void_p), ("nbins", C.c_int), ("xmax", C.c_double),
        ("Tcmb", C.c_double),
    ]


class BatchStats(C.Structure):
    _fields_ = [("models", C.c_int), ("active", C.c_int), ("iterations", C.c_int),
                ("lane_classes", C.c_int), ("work_items", C.c_int64),
                ("class_items", C.c_int * 16), ("class_threads", C.c_int * 16),
                ("class_chunk", C.c_int * 16), ("class_order", C.c_int * 16),
                ("tune_seconds", C.c_double),
                ("iterate_seconds", C.c_double), ("last_converged_seconds", C.c_double),
                ("updates_per_iteration", C.c_int64),
                ("lane_records", C.c_int64), ("lane_semi", C.c_int64),
                ("lane_origin_pairs", C.c_int64), ("fs_launches", C.c_int64),
                ("fs_ms_total", C.c_double), ("fs_ms_last", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("id", C.c_int64), ("kind", C.c_int), ("model", C.c_int), ("status", C.c_int),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("iterations", C.c_int), ("change", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("models", C.c_int), ("render_slots", C.c_int), ("submitted", C.c_int64),
                ("completed", C.c_int64), ("failed", C.c_int64), ("replays", C.c_int64),
                ("updates", C.c_int64), ("iterate_busy_s", C.c_double),
                ("render_busy_s", C.c_double), ("hbm_budget", C.c_uint64),
                ("hbm_resident", C.c_uint64), ("hbm_render_peak", C.c_uint64)]


class Counters(C.Structure):
    _fields_ = [("total_records", C.c_int64), ("holes", C.c_int64),
                ("semi_segments", C.c_int64), ("masing", C.c_int64), ("singular", C.c_int64),
                ("iterations", C.c_int), ("ng_applied", C.c_int), ("ng_rejected", C.c_int),
                ("last_change", C.c_double), ("fs_launches", C.c_int64),
                ("fs_ms_total", C.c_double), ("fs_ms_last", C.c_double)]


_lib = None


def lib():
    """Load libmgx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    # torch ships its own HIP runtime; loading it first lets libmgx.so bind to
    # that same runtime (same soname) so one process never holds two.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I, D, I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
    sig = {
        "mgx_default_options": (None, [P]),
        "mgx_create": (I, [P, I, P, P]),
        "mgx_destroy": (None, [P]),
        "mgx_last_error": (C.c_char_p, [P]),
        "mgx_load_model": (I, [P, P]),
        "mgx_trace_rays": (I, [P, P]),
        "mgx_get_trace": (I, [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P]),
        "mgx_get_trace_offsets": (I, [P, P]),
        "mgx_get_trace_records": (I, [P, I64, I64, P, P, P, P]),
        "mgx_set_populations": (I, [P, P]),
        "mgx_get_populations": (I, [P, P]),
        "mgx_set_lte_populations": (I, [P]),
        "mgx_formal_solve": (I, [P, P, P]),
        "mgx_set_radiation": (I, [P, P, P]),
        "mgx_formal_solve_shape": (I, [I, I, I, P, P, P]),
        "mgx_update_populations": (I, [P, P]),
        "mgx_ng_reset": (I, [P, I]),
        "mgx_ng_accelerate": (I, [P, I, I, P]),
        "mgx_ng_predict": (I, [P, I, P, P, P]),
        "mgx_ng_push": (I, [P]),
        "mgx_ng_predict_noalloc": (I, [I, P, P, I, I64, P, P, P]),
        "mgx_iterate": (I, [P, D, I, I, I, P, P]),
        "mgx_get_counters": (I, [P, P]),
        "mgx_reset_timers": (I, [P]),
        "mgx_render_image": (I, [P, P, I, I, D, D, I, P]),
        "mgx_batch_create": (I, [P, I, P, P]),
        "mgx_batch_destroy": (None, [P]),
        "mgx_batch_last_error": (C.c_char_p, [P]),
        "mgx_batch_add_model": (I, [P, P, P]),
        "mgx_batch_prepare": (I, [P]),
        "mgx_batch_set_lte_populations": (I, [P]),
        "mgx_batch_set_populations": (I, [P, I, P]),
        "mgx_batch_get_populations": (I, [P, I, P]),
        "mgx_batch_iterate": (I, [P, D, I, I, P, P, P]),
        "mgx_batch_get_stats": (I, [P, P]),
        "mgx_server_create": (I, [P, I, P, C.c_uint64, I]),
        "mgx_server_destroy": (None, [P]),
        "mgx_server_last_error": (C.c_char_p, [P]),
        "mgx_server_add_model": (I, [P, P, P]),
        "mgx_server_start": (I, [P]),
        "mgx_server_clock": (D, [P]),
        "mgx_server_submit_converge": (I, [P, I, D, I, I, P]),
        "mgx_server_submit_render": (I, [P, I, P, I, I, D, D, I, P, P]),
        "mgx_server_wait": (I, [P, I64, D, P]),
        "mgx_server_get_populations": (I, [P, I, P]),
        "mgx_server_get_stats": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a) -> int:
    """Address of a contiguous numpy array or torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous()
        return a.data_ptr()
    raise TypeError(type(a))


def _host_image(npy: int, npx: int, nfreq: int) -> np.ndarray:
    """Host array for an image: page-locked when torch can provide it (the
    device-to-host copy then runs at DMA speed, and torch's caching host
    allocator reuses freed buffers), else plain memory."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.empty((npy, npx, nfreq), dtype=torch.float32,
                               pin_memory=True).numpy()
    except ImportError:
        pass
    return np.empty((npy, npx, nfreq), np.float32)


def _torch_stream(device: int):
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream(device).cuda_stream


def _options(precision, branch_threshold, tau_floor, chi_min, pop_floor,
             trace_slot_min_bytes=None) -> Options:
    opt = Options()
    lib().mgx_default_options(C.byref(opt))
    opt.precision = precision
    opt.branch_threshold = branch_threshold
    opt.tau_floor = tau_floor
    opt.chi_min = chi_min
    opt.pop_floor = pop_floor
    if trace_slot_min_bytes is not None:
        opt.trace_slot_min_bytes = int(trace_slot_min_bytes)
    return opt


def _model_struct(m):
    """mgx_model view of a synthetic model; the arrays must outlive the call."""
    a = m.arrays()
    s = ModelStruct()
    s.dim, s.npoints = m.dim, m.npoints
    for k in ("pos", "vel", "nbs_off", "nbs", "bdy", "T", "vturb2", "nspec", "ncoll",
              "ray_dir", "ray_w", "antipode", "E", "g", "up", "lo", "A", "nu", "cu", "cl",
              "K0"):
        setattr(s, k, a[k].ctypes.data)
    s.nrays, s.mass, s.nlev, s.nlines = m.nrays, m.mass, m.nlev, m.nlines
    s.ncoll_tr = int(a["K0"].size)
    s.nbins, s.xmax, s.Tcmb = m.nbins, m.xmax, m.Tcmb
    return s, a


class Context:
    """One model on one GPU.  Mirrors the C ABI entry points by name."""

    def __init__(self, device: int = 0, precision: int = FP32, stream: Optional[int] = None,
                 use_torch_stream: bool = True, branch_threshold: float = 0.35,
                 tau_floor: float = 1e-15, chi_min: float = 1e-30, pop_floor: float = 1e-12,
                 trace_slot_min_bytes: Optional[int] = None):
        L = lib()
        opt = _options(precision, branch_threshold, tau_floor, chi_min, pop_floor,
                       trace_slot_min_bytes)
        if stream is None and use_torch_stream:
            stream = _torch_stream(device)
        h = C.c_void_p()
        st = L.mgx_create(C.byref(h), device, stream, C.byref(opt))
        if st != MGX_OK:
            raise MgxError(st, L.mgx_last_error(None).decode())
        self._h = h
        self.precision = precision
        self.model = None
        self._keep = None

    # -- plumbing -------------------------------------------------------------
    def _check(self, st: int):
        if st != MGX_OK:
            raise MgxError(st, lib().mgx_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().mgx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- model ------------------------------------------------------------------
    def load_model(self, m) -> None:
        s, keep = _model_struct(m)
        self._check(lib().mgx_load_model(self._h, C.byref(s)))
        del keep
        self.model = m

    def trace_rays(self) -> int:
        n = C.c_int64()
        self._check(lib().mgx_trace_rays(self._h, C.byref(n)))
        return n.value

    def get_trace(self, origin: int, ray: int):
        n = C.c_int32()
        self._check(lib().mgx_get_trace(self._h, origin, ray, 0, None, None, None, None,
                                        C.byref(n)))
        cap = max(n.value, 1)
        idx = np.zeros(cap, np.int32)
        Z = np.zeros(cap)
        dv = np.zeros(cap)
        semi = np.zeros(cap, np.uint8)
        self._check(lib().mgx_get_trace(self._h, origin, ray, cap, _ptr(idx), _ptr(Z), _ptr(dv),
                                        _ptr(semi), C.byref(n)))
        k = n.value
        return idx[:k], Z[:k], dv[:k], semi[:k]

    def get_trace_offsets(self) -> np.ndarray:
        m = self.model
        off = np.zeros(m.npoints * m.nrays + 1, np.int64)
        self._check(lib().mgx_get_trace_offsets(self._h, _ptr(off)))
        return off

    def get_trace_records(self, first: int, count: int):
        idx = np.zeros(count, np.int32)
        Z = np.zeros(count)
        dv = np.zeros(count)
        semi = np.zeros(count, np.uint8)
        self._check(lib().mgx_get_trace_records(self._h, first, count, _ptr(idx), _ptr(Z),
                                                _ptr(dv), _ptr(semi)))
        return idx, Z, dv, semi

    # -- populations / radiation ---------------------------------------------------
    def set_populations(self, pops) -> None:
        if isinstance(pops, np.ndarray):
            pops = np.ascontiguousarray(pops, np.float64)
        self._check(lib().mgx_set_populations(self._h, _ptr(pops)))

    def get_populations(self, out=None):
        m = self.model
        if out is None:
            out = np.zeros((m.npoints, m.nlev))
        self._check(lib().mgx_get_populations(self._h, _ptr(out)))
        return out

    def set_lte_populations(self) -> None:
        self._check(lib().mgx_set_lte_populations(self._h))

    def formal_solve(self, J=None, L=None, copy: bool = True):
        m = self.model
        if copy and J is None:
            J = np.zeros((m.npoints, m.nlines))
            L = np.zeros((m.npoints, m.nlines))
        self._check(lib().mgx_formal_solve(self._h, _ptr(J), _ptr(L)))
        return J, L

    def set_radiation(self, J, L) -> None:
        J = np.ascontiguousarray(J, np.float64) if isinstance(J, np.ndarray) else J
        L = np.ascontiguousarray(L, np.float64) if isinstance(L, np.ndarray) else L
        self._check(lib().mgx_set_radiation(self._h, _ptr(J), _ptr(L)))

    def update_populations(self) -> float:
        ch = C.c_double()
        self._check(lib().mgx_update_populations(self._h, C.byref(ch)))
        return ch.value

    def ng_reset(self, capacity: int) -> None:
        self._check(lib().mgx_ng_reset(self._h, capacity))

    def ng_push(self) -> None:
        self._check(lib().mgx_ng_push(self._h))

    def ng_accelerate(self, mode: int, param: int) -> bool:
        """One decision of the classical / adaptive Ng schedule; True if a
        prediction replaced the populations."""
        ap = C.c_int()
        self._check(lib().mgx_ng_accelerate(self._h, int(mode), int(param), C.byref(ap)))
        return bool(ap.value)

    def ng_predict(self, apply: bool = False):
        """(valid, change against the previous prediction, coefficients)."""
        st, pc = C.c_int(), C.c_double()
        coef = np.zeros(32)
        self._check(lib().mgx_ng_predict(self._h, int(apply), C.byref(st), C.byref(pc),
                                         _ptr(coef)))
        return bool(st.value), pc.value, coef

    def iterate(self, tol: float = 1e-10, max_iter: int = 500, ng_mode: int = NG_NONE,
                ng_param: int = 4, raise_on_noconv: bool = True):
        it, ch = C.c_int(), C.c_double()
        st = lib().mgx_iterate(self._h, tol, max_iter, ng_mode, ng_param, C.byref(it),
                               C.byref(ch))
        if st == MGX_ENOCONV and not raise_on_noconv:
            return it.value, ch.value, False
        self._check(st)
        return it.value, ch.value, True

    def counters(self) -> dict:
        c = Counters()
        self._check(lib().mgx_get_counters(self._h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    def reset_timers(self) -> None:
        self._check(lib().mgx_reset_timers(self._h))

    def render_image(self, direction, npx: int, npy: int, f_min: float, f_max: float,
                     nfreq: int, out=None):
        d = (C.c_double * 3)(*[float(x) for x in direction])
        if out is None:
            out = _host_image(npy, npx, nfreq)
        self._check(lib().mgx_render_image(self._h, d, npx, npy, f_min, f_max, nfreq,
                                           _ptr(out)))
        return out


class Batch:
    """Many models iterated together on one GPU (mgx_batch_* entry points)."""

    def __init__(self, device: int = 0, precision: int = FP32, stream: Optional[int] = None,
                 branch_threshold: float = 0.35, tau_floor: float = 1e-15,
                 chi_min: float = 1e-30, pop_floor: float = 1e-12):
        # stream None: the library creates its own (graph capture cannot use
        # the legacy default stream)
        L = lib()
        opt = _options(precision, branch_threshold, tau_floor, chi_min, pop_floor)
        h = C.c_void_p()
        st = L.mgx_batch_create(C.byref(h), device, stream, C.byref(opt))
        if st != MGX_OK:
            raise MgxError(st, L.mgx_batch_last_error(None).decode())
        self._h = h
        self.precision = precision
        self.models = []

    def _check(self, st: int):
        if st != MGX_OK:
            raise MgxError(st, lib().mgx_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().mgx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_model(self, m) -> int:
        s, keep = _model_struct(m)
        i = C.c_int()
        self._check(lib().mgx_batch_add_model(self._h, C.byref(s), C.byref(i)))
        del keep
        self.models.append(m)
        return i.value

    def prepare(self) -> None:
        self._check(lib().mgx_batch_prepare(self._h))

    def set_lte_populations(self) -> None:
        self._check(lib().mgx_batch_set_lte_populations(self._h))

    def set_populations(self, i: int, pops) -> None:
        pops = np.ascontiguousarray(pops, np.float64) if isinstance(pops, np.ndarray) else pops
        self._check(lib().mgx_batch_set_populations(self._h, i, _ptr(pops)))

    def get_populations(self, i: int, out=None):
        m = self.models[i]
        if out is None:
            out = np.empty((m.npoints, m.nlev), np.float64)
        self._check(lib().mgx_batch_get_populations(self._h, i, _ptr(out)))
        return out

    def iterate(self, tol: float = 1e-10, max_iter: int = 500, ng_order: int = 0,
                raise_on_noconv: bool = True):
        M = len(self.models)
        its = np.zeros(M, np.int32)
        chg = np.zeros(M, np.float64)
        nconv = C.c_int()
        st = lib().mgx_batch_iterate(self._h, tol, max_iter, ng_order, _ptr(its), _ptr(chg),
                                     C.byref(nconv))
        if st == MGX_ENOCONV and not raise_on_noconv:
            return its, chg, nconv.value
        self._check(st)
        return its, chg, nconv.value

    def stats(self) -> dict:
        s = BatchStats()
        self._check(lib().mgx_batch_get_stats(self._h, C.byref(s)))
        out = {}
        for k, _ in BatchStats._fields_:
            v = getattr(s, k)
            out[k] = list(v) if not isinstance(v, (int, float)) else v
        return out


class Server:
    """Resident models answering converge and render requests (mgx_server_*)."""

    def __init__(self, device: int = 0, precision: int = FP32, hbm_budget: int = 0,
                 render_slots: int = 2, branch_threshold: float = 0.35,
                 tau_floor: float = 1e-15, chi_min: float = 1e-30, pop_floor: float = 1e-12):
        L = lib()
        opt = _options(precision, branch_threshold, tau_floor, chi_min, pop_floor)
        h = C.c_void_p()
        st = L.mgx_server_create(C.byref(h), device, C.byref(opt), int(hbm_budget), render_slots)
        if st != MGX_OK:
            raise MgxError(st, L.mgx_server_last_error(None).decode())
        self._h = h
        self.models = []
        self._images = {}   # request id -> image array (kept alive until finished)

    def _check(self, st: int):
        if st != MGX_OK:
            raise MgxError(st, lib().mgx_server_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().mgx_server_destroy(self._h)
            self._h = None
            self._images.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_model(self, m) -> int:
        s, keep = _model_struct(m)
        i = C.c_int()
        self._check(lib().mgx_server_add_model(self._h, C.byref(s), C.byref(i)))
        del keep
        self.models.append(m)
        return i.value

    def start(self) -> None:
        self._check(lib().mgx_server_start(self._h))

    def clock(self) -> float:
        return lib().mgx_server_clock(self._h)

    def submit_converge(self, model: int, tol: float = 1e-6, max_iter: int = 200,
                        ng_order: int = 4) -> int:
        rid = C.c_int64()
        self._check(lib().mgx_server_submit_converge(self._h, model, tol, max_iter, ng_order,
                                                     C.byref(rid)))
        return rid.value

    def submit_render(self, model: int, direction, npx: int, npy: int, f_min: float,
                      f_max: float, nfreq: int, out=None) -> int:
        d = (C.c_double * 3)(*[float(x) for x in direction])
        if out is None:
            # pageable: many requests may be in flight at once, and page-locked
            # memory is a scarce host resource
            out = np.empty((npy, npx, nfreq), np.float32)
        rid = C.c_int64()
        self._check(lib().mgx_server_submit_render(self._h, model, d, npx, npy, f_min, f_max,
                                                   nfreq, _ptr(out), C.byref(rid)))
        self._images[rid.value] = out
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0, raise_on_error: bool = True) -> dict:
        info = RequestInfo()
        st = lib().mgx_server_wait(self._h, rid, timeout, C.byref(info))
        out = {k: getattr(info, k) for k, _ in RequestInfo._fields_}
        if st != MGX_EPENDING:
            out["image"] = self._images.pop(rid, None)
        if raise_on_error and st not in (MGX_OK, MGX_EPENDING):
            raise MgxError(st, lib().mgx_server_last_error(self._h).decode())
        return out

    def get_populations(self, model: int, out=None):
        m = self.models[model]
        if out is None:
            out = np.empty((m.npoints, m.nlev), np.float64)
        self._check(lib().mgx_server_get_populations(self._h, model, _ptr(out)))
        return out

    def stats(self) -> dict:
        s = ServerStats()
        self._check(lib().mgx_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def ng_predict_noalloc(iterates, prediction, coef, status, device: int = 0,
                       stream: Optional[int] = None) -> None:
    """Ng prediction from device iterates without allocation (see the C
    header): iterates is a sequence of contiguous device tensors of equal
    length, prediction / coef / status device tensors (float64, float64,
    int32).  Enqueued on torch's current stream unless stream is given."""
    nh = len(iterates)
    table = (C.c_void_p * max(nh, 1))(*[_ptr(t) for t in iterates])
    n = int(iterates[0].numel()) if nh else 0
    s = _torch_stream(device) if stream is None else stream
    st = lib().mgx_ng_predict_noalloc(device, s, table, nh, n, _ptr(prediction), _ptr(coef),
                                      _ptr(status))
    if st != MGX_OK:
        raise MgxError(st, lib().mgx_last_error(None).decode())


def formal_solve_shape(precision: int, nlines: int, nbins: int):
    """(lines per chunk, threads per workgroup, LDS bytes) of the formal
    solution's launch for such a model (host-only query)."""
    nlc, nth, lds = C.c_int(), C.c_int(), C.c_int64()
    st = lib().mgx_formal_solve_shape(precision, nlines, nbins, C.byref(nlc), C.byref(nth),
                                      C.byref(lds))
    if st != MGX_OK:
        raise MgxError(st, "invalid formal-solution shape query")
    return nlc.value, nth.value, lds.value


def header_functions(header_path: Optional[str] = None):
    """Names of the functions declared in include/mgx.h."""
    import re
    if header_path is None:
        header_path = os.path.join(os.path.dirname(HERE), "include", "mgx.h")
    text = open(header_path).read()
    return sorted(set(re.findall(r"\b(mgx_[a-z_]+)\s*\(", text)))
