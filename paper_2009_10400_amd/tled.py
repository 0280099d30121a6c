"""Thin ctypes binding of ``libtled.so`` (C-ABI in ``include/tled.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch is used for device memory (optional caching-allocator
callback) and streams.  There is no fallback: if the library is missing this
module raises on import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "csrc", "libtled.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2009_10400_amd.build`")


def _share_torch_hip_runtime():
    """Bind the library to PyTorch's bundled HIP runtime when PyTorch is installed.

    PyTorch ships its own ``libamdhip64`` (same soname as the system one).  If the
    system copy were loaded first, importing torch later would bring a second HIP
    runtime into the process and torch would find no device.  Loading torch's copy
    (by path, without importing torch) before the library keeps one runtime.
    """
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    for base in spec.submodule_search_locations:
        path = os.path.join(base, "lib", "libamdhip64.so")
        if os.path.exists(path):
            ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
            return


_share_torch_hip_runtime()
_lib = ctypes.CDLL(LIB_PATH)

OK, E_ARG, E_MESH, E_STATE, E_HIP, E_OOM, E_UNSTABLE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
T4, H8 = 4, 8
FLAG_NONFINITE, FLAG_INVERTED = 1, 2

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class Material(ctypes.Structure):
    _fields_ = [
        ("rho", _d), ("mu", _d), ("kappa", _d), ("eta", _d), ("alpha", _d), ("alpha_m", _d),
        ("alpha_n", _d), ("T0", _d), ("k", _d), ("k_m", _d), ("c", _d), ("wbcb", _d), ("T_art", _d), ("Q_met", _d),
        ("g", _d * 4), ("tau", _d * 4),
        ("muT_lo", _d), ("muT_hi", _d), ("muT_drop", _d),
        ("shrink_T", _d), ("shrink_width", _d), ("shrink_eps", _d),
        ("ckT_lo", _d), ("ckT_hi", _d), ("c_hi", _d), ("k_hi", _d), ("hg_coef", _d),
        ("n_prony", _i32), ("expan_mode", _i32), ("cond_mode", _i32), ("muT_on", _i32),
        ("shrink_on", _i32), ("ckT_on", _i32),
    ]


class Options(ctypes.Structure):
    _fields_ = [("graph_steps", _i32), ("kernel_variant", _i32), ("reorder", _i32),
                ("block_size", _i32), ("patch_elems", _i32), ("ablation_T", _d),
                ("batch_schedule", _i32), ("shared_update", _i32)]


class Monitors(ctypes.Structure):
    _fields_ = [("step", _i64), ("t", _d), ("kinetic", _d), ("strain", _d), ("T_max", _d),
                ("T_min", _d), ("ablated_volume", _d), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_scenarios", _i32), ("n_patches", _i32), ("n_elems", _i64), ("n_nodes", _i64),
                ("n_shared_nodes", _i64), ("max_steps", _i64), ("step", _i64), ("device_bytes", _i64),
                ("kernel_variant", _i32), ("reserved", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", _i64), ("n_elems", _i64), ("elem_type", _i32), ("n_prony", _i32),
                ("n_swapped", _i64), ("kernel_variant", _i32), ("n_patches", _i32),
                ("n_shared_nodes", _i64), ("patch_max_nodes", _i32), ("patch_lds_bytes", _i32),
                ("device_bytes", _i64), ("dt", _d), ("dt_critical", _d), ("patch_wgs_per_cu", _i32),
                ("shared_update", _i32), ("dt_thermal", _d)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_P = ctypes.c_void_p
_dp = ctypes.POINTER(_d)
_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "tled_create": ([ctypes.POINTER(_P), ctypes.c_int], ctypes.c_int),
    "tled_destroy": ([_P], None),
    "tled_set_allocator": ([_P, _ALLOC, _FREE, _P], ctypes.c_int),
    "tled_set_stream": ([_P, _P], ctypes.c_int),
    "tled_set_options": ([_P, ctypes.POINTER(Options)], ctypes.c_int),
    "tled_set_mesh": ([_P, ctypes.c_int, _i64, _dp, _i64, ctypes.POINTER(_i32)], ctypes.c_int),
    "tled_set_material": ([_P, ctypes.POINTER(Material)], ctypes.c_int),
    "tled_set_fibres": ([_P, _dp], ctypes.c_int),
    "tled_set_expansion_axes": ([_P, _dp], ctypes.c_int),
    "tled_set_conductivity": ([_P, _dp], ctypes.c_int),
    "tled_set_fixed_dofs": ([_P, _i64, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_uint8)], ctypes.c_int),
    "tled_set_fixed_temperature": ([_P, _i64, ctypes.POINTER(_i32), _dp], ctypes.c_int),
    "tled_set_heat_source": ([_P, _dp, _d, _d], ctypes.c_int),
    "tled_set_time": ([_P, _d, _d], ctypes.c_int),
    "tled_critical_dt": ([_P, _dp], ctypes.c_int),
    "tled_finalize": ([_P], ctypes.c_int),
    "tled_step": ([_P, _i64], ctypes.c_int),
    "tled_stream_copy": ([ctypes.c_int, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tled_prepare_steps": ([_P, _i64], ctypes.c_int),
    "tled_sync": ([_P], ctypes.c_int),
    "tled_read_u": ([_P, _dp], ctypes.c_int),
    "tled_read_T": ([_P, _dp], ctypes.c_int),
    "tled_set_thermal_dose": ([_P, _d, _d], ctypes.c_int),
    "tled_read_thermal_dose": ([_P, _dp, _dp], ctypes.c_int),
    "tled_copy_fields_device": ([_P, _P, _P], ctypes.c_int),
    "tled_get_monitors": ([_P, ctypes.POINTER(Monitors)], ctypes.c_int),
    "tled_get_info": ([_P, ctypes.POINTER(Info)], ctypes.c_int),
    "tled_get_lumped": ([_P, _dp, _dp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "tled_read_state": ([_P, _dp, _dp, _dp, _dp, ctypes.POINTER(_i64)], ctypes.c_int),
    "tled_write_state": ([_P, _dp, _dp, _dp, _dp, _i64], ctypes.c_int),
    "tled_state_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tled_get_state": ([_P, _P], ctypes.c_int),
    "tled_set_state": ([_P, _P], ctypes.c_int),
    "tled_kernel_times": ([_P, _i64, _dp], ctypes.c_int),
    "tled_batch_create": ([ctypes.POINTER(_P), ctypes.c_int], ctypes.c_int),
    "tled_batch_destroy": ([_P], None),
    "tled_batch_add": ([_P, ctypes.c_int, _i64, _dp, _i64, ctypes.POINTER(_i32), ctypes.POINTER(Material), _dp, _dp,
                        _d, _d, _i64, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_uint8), _d, _d, _i64, _i32,
                        ctypes.POINTER(_i32)], ctypes.c_int),
    "tled_batch_set_duration": ([_P, _i32, _d, _d], ctypes.c_int),
    "tled_batch_finalize": ([_P], ctypes.c_int),
    "tled_batch_scenario_steps": ([_P, _i32, _dp, ctypes.POINTER(_i64)], ctypes.c_int),
    "tled_batch_run": ([_P], ctypes.c_int),
    "tled_batch_read": ([_P, _i32, _dp, _dp], ctypes.c_int),
    "tled_batch_read_all": ([_P, _dp, _dp], ctypes.c_int),
    "tled_batch_monitors": ([_P, _d, _dp, _dp], ctypes.c_int),
    "tled_batch_get_info": ([_P, ctypes.POINTER(BatchInfo)], ctypes.c_int),
    "tled_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "tled_last_error": ([_P], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class TledError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_lib.tled_status_string(status).decode()} ({status}): {message}")
        self.status = status


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def material(params: dict) -> Material:
    """Material struct from a dict of field names (missing fields are zero / off)."""
    m = Material()
    ints = ("n_prony", "expan_mode", "cond_mode", "muT_on", "shrink_on", "ckT_on")
    for name, _ in Material._fields_:
        if name not in params:
            continue
        v = params[name]
        if name in ("g", "tau"):
            setattr(m, name, (_d * 4)(*([float(x) for x in v] + [0.0] * (4 - len(v)))))
        elif name in ints:
            setattr(m, name, int(v))
        else:
            setattr(m, name, float(v))
    if "n_prony" not in params and "g" in params:
        m.n_prony = len(params["g"])
    return m


class Sim:
    """One problem on one device (``device=-1``: host-only set-up)."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = False):
        h = _P()
        st = _lib.tled_create(ctypes.byref(h), int(device))
        if st != OK:
            raise TledError(st, f"tled_create(device={device}) failed")
        self._h = h
        self.device = device
        self._cb = None
        if use_torch_allocator and device >= 0:
            self._torch_allocator(device)
        if stream is not None:
            self._check(_lib.tled_set_stream(h, _P(int(stream))))

    def _torch_allocator(self, device: int):
        """Route the library's device allocations through torch's caching allocator."""
        import sys

        import torch
        torch.cuda.init()
        dev = torch.device("cuda", device)

        def _alloc(nbytes, ctx):
            try:
                with torch.cuda.device(dev):
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev))
            except Exception as exc:  # noqa: BLE001 - reported, then NULL (TLED_E_OOM)
                print(f"tled: torch allocator failed for {nbytes} bytes: {exc!r}", file=sys.stderr)
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._cb = (_ALLOC(_alloc), _FREE(_free))
        self._check(_lib.tled_set_allocator(self._h, self._cb[0], self._cb[1], None))

    # ------------------------------------------------------------------ helpers
    def _check(self, st):
        if st != OK:
            raise TledError(st, _lib.tled_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tled_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    # ------------------------------------------------------------------ set-up
    def set_options(self, **kw):
        o = Options()
        for k, v in kw.items():
            setattr(o, k, v)
        self._check(_lib.tled_set_options(self._h, ctypes.byref(o)))

    def set_mesh(self, elem_type, X, conn):
        X = _f64(X)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.nn, self.ne, self.npe = X.shape[0], conn.shape[0], int(elem_type)
        self._check(_lib.tled_set_mesh(self._h, int(elem_type), self.nn, _ptr(X), self.ne,
                                       conn.ctypes.data_as(ctypes.POINTER(_i32))))

    def set_material(self, params: dict):
        self.params = dict(params)
        self._mat = material(params)
        self.n_prony = self._mat.n_prony
        self._check(_lib.tled_set_material(self._h, ctypes.byref(self._mat)))

    def set_fibres(self, a0):
        self._check(_lib.tled_set_fibres(self._h, _ptr(_f64(a0))))

    def set_expansion_axes(self, n0):
        """Second axis of the orthotropic expansion per element (n_elems x 3)."""
        if n0 is not None:
            n0 = _f64(n0)
            if n0.shape != (self.ne, 3):
                raise ValueError(f"expansion axes must be ({self.ne}, 3), got {n0.shape}")
        self._check(_lib.tled_set_expansion_axes(self._h, _ptr(n0)))

    def set_conductivity(self, D):
        """Conductivity tensor per element: n_elems x 3 x 3 (symmetric) or n_elems x 6 (xx yy zz xy yz xz)."""
        if D is None:
            self._check(_lib.tled_set_conductivity(self._h, None))
            return
        D = np.asarray(D, dtype=np.float64)
        if D.ndim == 3 and D.shape[1:] == (3, 3):
            D = np.stack([D[:, 0, 0], D[:, 1, 1], D[:, 2, 2], D[:, 0, 1], D[:, 1, 2], D[:, 0, 2]], 1)
        D = _f64(D)
        if D.shape != (self.ne, 6):
            raise ValueError(f"conductivity tensors must be ({self.ne}, 3, 3) or ({self.ne}, 6), got {D.shape}")
        self._check(_lib.tled_set_conductivity(self._h, _ptr(D)))

    def set_fixed_dofs(self, nodes, masks):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        masks = np.ascontiguousarray(masks, dtype=np.uint8)
        self._check(_lib.tled_set_fixed_dofs(self._h, len(nodes), nodes.ctypes.data_as(ctypes.POINTER(_i32)),
                                             masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))

    def set_fixed_temperature(self, nodes, T):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        T = _f64(T)
        self._check(_lib.tled_set_fixed_temperature(self._h, len(nodes),
                                                    nodes.ctypes.data_as(ctypes.POINTER(_i32)), _ptr(T)))

    def set_heat_source(self, q_elem, t_on=0.0, t_off=float("inf")):
        self._check(_lib.tled_set_heat_source(self._h, _ptr(_f64(q_elem)), float(t_on), float(t_off)))

    def set_time(self, dt, gamma):
        self.dt = float(dt)
        self._check(_lib.tled_set_time(self._h, float(dt), float(gamma)))

    def critical_dt(self) -> float:
        v = _d()
        self._check(_lib.tled_critical_dt(self._h, ctypes.byref(v)))
        return v.value

    def finalize(self):
        self._check(_lib.tled_finalize(self._h))

    # ------------------------------------------------------------------ run
    def step(self, n: int):
        self._check(_lib.tled_step(self._h, int(n)))

    def prepare(self, n: int):
        """Capture the hipGraphs a following step(n) replays, without running anything."""
        self._check(_lib.tled_prepare_steps(self._h, int(n)))

    def sync(self):
        self._check(_lib.tled_sync(self._h))

    def read_u(self):
        out = np.zeros((self.nn, 3))
        self._check(_lib.tled_read_u(self._h, _ptr(out)))
        return out

    def read_T(self):
        out = np.zeros(self.nn)
        self._check(_lib.tled_read_T(self._h, _ptr(out)))
        return out

    def set_thermal_dose(self, arrhenius_A: float = 0.0, arrhenius_Ea: float = 0.0):
        """Accumulate CEM43 and the Arrhenius damage integral per node (before finalize)."""
        self._check(_lib.tled_set_thermal_dose(self._h, float(arrhenius_A), float(arrhenius_Ea)))

    def read_thermal_dose(self):
        """(CEM43 minutes, Arrhenius integral) per node, caller numbering."""
        cem, om = np.zeros(self.nn), np.zeros(self.nn)
        self._check(_lib.tled_read_thermal_dose(self._h, _ptr(cem), _ptr(om)))
        return cem, om

    def damage_volumes(self, cem43_min: float = 240.0, omega_min: float = 1.0) -> dict:
        """Lumped reference volume (m^3) of the nodes whose CEM43 reaches cem43_min minutes and of
        those whose Arrhenius integral reaches omega_min."""
        cem, om = self.read_thermal_dose()
        Vl = self.lumped()["Vl"]
        return {"cem43": float(Vl[cem >= cem43_min].sum()), "arrhenius": float(Vl[om >= omega_min].sum())}

    def copy_fields_device(self, u_dst=None, T_dst=None):
        """Write u (nn x 3) and T (nn) as float32 into device tensors (caller numbering)."""
        import torch
        n = self.info()["n_nodes"]
        for t, shape, name in ((u_dst, (n, 3), "u_dst"), (T_dst, (n,), "T_dst")):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
                                  or not t.is_contiguous() or tuple(t.shape) != shape):
                raise ValueError(f"{name}: expected a contiguous float32 device tensor of shape {shape}")
        up = None if u_dst is None else _P(u_dst.data_ptr())
        tp = None if T_dst is None else _P(T_dst.data_ptr())
        self._check(_lib.tled_copy_fields_device(self._h, up, tp))

    def monitors(self) -> dict:
        m = Monitors()
        self._check(_lib.tled_get_monitors(self._h, ctypes.byref(m)))
        return m.as_dict()

    def info(self) -> dict:
        i = Info()
        self._check(_lib.tled_get_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def lumped(self) -> dict:
        out = {k: np.zeros(self.nn) for k in ("Vl", "M", "C", "Kb", "Qm", "Qr")}
        self._check(_lib.tled_get_lumped(self._h, *(_ptr(out[k]) for k in ("Vl", "M", "C", "Kb", "Qm", "Qr"))))
        return out

    def read_state(self) -> dict:
        u = np.zeros((self.nn, 3)); v = np.zeros((self.nn, 3)); T = np.zeros(self.nn)
        th = np.zeros((self.ne, self.n_prony, 6))
        step = _i64()
        self._check(_lib.tled_read_state(self._h, _ptr(u), _ptr(v), _ptr(T), _ptr(th) if th.size else None,
                                         ctypes.byref(step)))
        return {"u": u, "v": v, "T": T, "theta": th, "step": step.value}

    def write_state(self, u=None, v=None, T=None, theta=None, step=0):
        self._check(_lib.tled_write_state(self._h, _ptr(_f64(u)), _ptr(_f64(v)), _ptr(_f64(T)),
                                          _ptr(_f64(theta)) if theta is not None and np.size(theta) else None,
                                          int(step)))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(_lib.tled_state_size(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(_lib.tled_get_state(self._h, buf))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(_lib.tled_set_state(self._h, buf))

    def kernel_times(self, n_steps: int):
        ms = (_d * 3)()
        self._check(_lib.tled_kernel_times(self._h, int(n_steps), ms))
        return {"element_ms": ms[0], "node_ms": ms[1], "finish_ms": ms[2]}


def stream_copy(dst, src, stream=None):
    """The library's plain streaming copy of one device tensor into another of the same size."""
    import torch
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("stream_copy needs contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or dst.device != src.device:
        raise ValueError("stream_copy needs tensors of one size on one device")
    st = _lib.tled_stream_copy(int(src.device.index), _P(dst.data_ptr()), _P(src.data_ptr()), nbytes,
                               _P(int(stream) if stream is not None else torch.cuda.current_stream(src.device).cuda_stream))
    if st != OK:
        raise TledError(st, "tled_stream_copy failed")


def from_problem(problem, dt=None, device: int = 0, stream=None, finalize: bool = True,
                 use_torch_allocator: bool = False, **options) -> Sim:
    """Set up a :class:`Sim` from a :class:`workloads.Problem` (dt defaults to cfl * critical step)."""
    s = Sim(device, stream=stream, use_torch_allocator=use_torch_allocator)
    if options:
        s.set_options(**options)
    s.set_mesh(problem.npe, problem.X, problem.conn)
    s.set_material(problem.params)
    if problem.a0 is not None:
        s.set_fibres(problem.a0)
    if problem.n0 is not None:
        s.set_expansion_axes(problem.n0)
    if problem.D is not None:
        s.set_conductivity(problem.D)
    if problem.fix is not None:
        nodes = np.nonzero(problem.fix & 7)[0]
        if len(nodes):
            s.set_fixed_dofs(nodes, problem.fix[nodes] & 7)
        tn = np.nonzero(problem.fix & 8)[0]
        if len(tn):
            s.set_fixed_temperature(tn, problem.Tfix[tn])
    if problem.q is not None:
        s.set_heat_source(problem.q, problem.t_on, problem.t_off)
    if dt is None:
        dt = problem.cfl * s.critical_dt()
    s.set_time(dt, problem.gamma)
    if finalize:
        s.finalize()
    return s


class Batch(Sim):
    """Many independent scenarios advanced together by the fused kernels."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = False):
        h = _P()
        st = _lib.tled_batch_create(ctypes.byref(h), int(device))
        if st != OK:
            raise TledError(st, f"tled_batch_create(device={device}) failed")
        self._h = h
        self.device = device
        self._cb = None
        self.sizes = []
        if use_torch_allocator and device >= 0:
            self._torch_allocator(device)
        if stream is not None:
            self._check(_lib.tled_set_stream(h, _P(int(stream))))

    def add(self, problem, dt: float = 0.0, n_steps: int = 0, patch_elems: int = 0, cfl: float = 0.0,
            t_end: float = 0.0) -> int:
        """Adds a scenario: either an explicit dt and n_steps, or cfl > 0 and t_end, in which case
        finalize picks dt = cfl x the scenario's critical step and n_steps = round(t_end / dt)."""
        k = self._add(problem, dt, n_steps, patch_elems)
        if cfl > 0.0:
            self._check(_lib.tled_batch_set_duration(self._h, k, float(cfl), float(t_end)))
        return k

    def scenario_steps(self, k: int):
        """(dt, n_steps) of scenario k after finalize."""
        dt = _d()
        n = _i64()
        self._check(_lib.tled_batch_scenario_steps(self._h, int(k), ctypes.byref(dt), ctypes.byref(n)))
        return dt.value, n.value

    def _add(self, problem, dt: float, n_steps: int, patch_elems: int) -> int:
        X = _f64(problem.X)
        conn = np.ascontiguousarray(problem.conn, dtype=np.int32)
        m = material(problem.params)
        self.n_prony = m.n_prony
        fix = problem.fix if problem.fix is not None else np.zeros(len(X), np.uint8)
        nodes = np.ascontiguousarray(np.nonzero(fix & 7)[0], dtype=np.int32)
        masks = np.ascontiguousarray(fix[nodes] & 7, dtype=np.uint8)
        idx = _i32()
        self._check(_lib.tled_batch_add(
            self._h, int(problem.npe), len(X), _ptr(X), len(conn), conn.ctypes.data_as(ctypes.POINTER(_i32)),
            ctypes.byref(m), _ptr(_f64(problem.a0)), _ptr(_f64(problem.q)), float(problem.t_on),
            float(problem.t_off), len(nodes), nodes.ctypes.data_as(ctypes.POINTER(_i32)),
            masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), float(dt), float(problem.gamma), int(n_steps),
            int(patch_elems), ctypes.byref(idx)))
        self.sizes.append(len(X))
        return idx.value

    def finalize(self):
        self._check(_lib.tled_batch_finalize(self._h))

    def run(self):
        self._check(_lib.tled_batch_run(self._h))

    def read(self, k: int):
        n = self.sizes[k]
        u = np.zeros((n, 3))
        T = np.zeros(n)
        self._check(_lib.tled_batch_read(self._h, int(k), _ptr(u), _ptr(T)))
        return u, T

    def read_all(self):
        """[(u, T)] of every scenario, from one device-to-host copy."""
        n = sum(self.sizes)
        u = np.zeros((n, 3))
        T = np.zeros(n)
        self._check(_lib.tled_batch_read_all(self._h, _ptr(u), _ptr(T)))
        out, o = [], 0
        for s in self.sizes:
            out.append((u[o:o + s], T[o:o + s]))
            o += s
        return out

    def scenario_monitors(self, ablation_T: float = 333.15, strict: bool = True):
        """Per-scenario maximum temperature and volume at or above ablation_T.  With strict=False a
        device-raised instability does not raise: (T_max, volume, status) is returned, and the
        scenarios that went unstable show a non-finite T_max."""
        S = len(self.sizes)
        tmax = np.zeros(S)
        vol = np.zeros(S)
        st = _lib.tled_batch_monitors(self._h, float(ablation_T), _ptr(tmax), _ptr(vol))
        if strict:
            self._check(st)
            return tmax, vol
        if st not in (OK, E_UNSTABLE):
            self._check(st)
        return tmax, vol, st

    def batch_info(self) -> dict:
        i = BatchInfo()
        self._check(_lib.tled_batch_get_info(self._h, ctypes.byref(i)))
        return i.as_dict()
