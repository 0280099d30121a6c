"""FP64 CPU oracle of the coupled TLED + Pennes time step (arXiv 2009.10400).

TEST INFRASTRUCTURE.  Only the tests, the smoke check of ``__graft_entry__`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It loads
``liborc.so`` built from ``tled_oracle.c`` with gcc and shares no code with the
GPU library (``paper_2009_10400_amd``): it never imports it, and the library
never imports this.

Material parameters are passed as a plain ``dict`` whose keys are the field
names of :class:`Material`; missing keys default to zero (flags off).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tled_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


class Material(ctypes.Structure):
    """Mirror of ``orc_material`` in tled_oracle.c (same field order)."""

    _fields_ = [
        ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("kappa", ctypes.c_double),
        ("eta", ctypes.c_double), ("alpha", ctypes.c_double), ("alpha_m", ctypes.c_double),
        ("alpha_n", ctypes.c_double), ("T0", ctypes.c_double), ("k", ctypes.c_double), ("k_m", ctypes.c_double),
        ("c", ctypes.c_double), ("wbcb", ctypes.c_double), ("T_art", ctypes.c_double),
        ("Q_met", ctypes.c_double), ("g", ctypes.c_double * 4), ("tau", ctypes.c_double * 4),
        ("muT_lo", ctypes.c_double), ("muT_hi", ctypes.c_double), ("muT_drop", ctypes.c_double),
        ("shrink_T", ctypes.c_double), ("shrink_width", ctypes.c_double),
        ("shrink_eps", ctypes.c_double),
        ("ckT_lo", ctypes.c_double), ("ckT_hi", ctypes.c_double), ("c_hi", ctypes.c_double),
        ("k_hi", ctypes.c_double), ("hg_coef", ctypes.c_double),
        ("n_prony", ctypes.c_int32), ("expan_mode", ctypes.c_int32),
        ("cond_mode", ctypes.c_int32), ("muT_on", ctypes.c_int32),
        ("shrink_on", ctypes.c_int32), ("ckT_on", ctypes.c_int32),
    ]


def material(params: dict) -> Material:
    m = Material()
    for name, _ in Material._fields_:
        if name in params:
            v = params[name]
            if name in ("g", "tau"):
                arr = (ctypes.c_double * 4)(*([float(x) for x in v] + [0.0] * (4 - len(v))))
                setattr(m, name, arr)
            elif name in ("n_prony", "expan_mode", "cond_mode", "muT_on", "shrink_on", "ckT_on"):
                setattr(m, name, int(v))
            else:
                setattr(m, name, float(v))
    if "n_prony" not in params and "g" in params:
        m.n_prony = len(params["g"])
    return m


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


def _load(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_create.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.c_int64, dp, ctypes.c_int64,
                             ctypes.POINTER(ctypes.c_int32), dp, dp, dp, dp, ctypes.POINTER(ctypes.c_uint8), dp,
                             ctypes.POINTER(Material), ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double]
    L.orc_create.restype = ctypes.c_int
    L.orc_destroy.argtypes = [P]
    L.orc_critical_dt.argtypes = [P]
    L.orc_critical_dt.restype = ctypes.c_double
    L.orc_n_swapped.argtypes = [P]
    L.orc_n_swapped.restype = ctypes.c_int64
    L.orc_lumped.argtypes = [P, dp, dp, dp, dp, dp]
    L.orc_geometry.argtypes = [P, ctypes.POINTER(ctypes.c_int32), dp, dp]
    L.orc_run.argtypes = [P, ctypes.c_int64, ctypes.c_int64, dp, dp, dp, dp, dp]
    L.orc_run.restype = ctypes.c_int
    L.orc_loads.argtypes = [P, dp, dp, dp, dp]
    L.orc_loads.restype = ctypes.c_int
    L.orc_stress.argtypes = [ctypes.POINTER(Material), dp, dp, dp, ctypes.c_double, dp, dp]
    L.orc_stress.restype = ctypes.c_double
    L.orc_element.argtypes = [ctypes.POINTER(Material), ctypes.c_int32, dp, dp, dp, dp, dp, dp, dp,
                              ctypes.c_double, dp, dp, dp]
    L.orc_element.restype = ctypes.c_int
    L.orc_thermal_dose.argtypes = [ctypes.c_int64, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
    L.orc_thermal_dose.restype = None
    return L


@contextlib.contextmanager
def using_library(path: str):
    """Route every oracle call through another build of the oracle source for the
    duration of the block (the tests use it to show that the pins catch planted
    mistakes in a copy of the oracle)."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def build_variant(src_text: str, out_dir: str, name: str) -> str:
    """Compile oracle source text (e.g. a copy with one planted mistake) into out_dir."""
    src = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, src, "-lm"])
    return so


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def stress(params: dict, F, a0, Te: float, n0=None):
    """Total pulled-back stress S0 (3x3) and energy density det(Fth) Psi.  n0: the second
    thermal-expansion axis of the orthotropic mode (expan_mode 2)."""
    m = material(params)
    F = _f64(np.asarray(F).reshape(9))
    a0 = _f64(np.asarray(a0).reshape(3))
    n0 = None if n0 is None else _f64(np.asarray(n0, dtype=np.float64).reshape(3))
    S = np.zeros(9)
    psi = np.zeros(1)
    lib().orc_stress(ctypes.byref(m), _dp(F), _dp(a0), _dp(n0), float(Te), _dp(S), _dp(psi))
    return S.reshape(3, 3), float(psi[0])


def element(params: dict, Xe, ue, Te, a0=(1.0, 0.0, 0.0), theta=None, dt: float = 0.0, n0=None, D=None):
    """One element: nodal forces (npe x 3), conduction loads (npe), energy; theta updated in place.
    n0: second expansion axis (expan_mode 2); D: conductivity tensor, 3x3 or (xx yy zz xy yz xz)
    (cond_mode 2)."""
    m = material(params)
    Xe = _f64(Xe)
    npe = Xe.shape[0]
    ue = _f64(ue)
    Te = _f64(np.broadcast_to(np.asarray(Te, dtype=np.float64), (npe,)).copy())
    a0 = _f64(np.asarray(a0, dtype=np.float64).reshape(3))
    f = np.zeros((npe, 3))
    h = np.zeros(npe)
    en = np.zeros(1)
    n0 = None if n0 is None else _f64(np.asarray(n0, dtype=np.float64).reshape(3))
    D = None if D is None else _f64(sym6(D).reshape(6))
    rc = lib().orc_element(ctypes.byref(m), npe, _dp(Xe), _dp(ue), _dp(Te), _dp(a0), _dp(n0), _dp(D),
                           _dp(theta) if theta is not None else None, float(dt), _dp(f), _dp(h), _dp(en))
    if rc != 0:
        raise ValueError(f"orc_element failed ({rc})")
    return f, h, float(en[0])


def sym6(D):
    """Symmetric tensors as (xx yy zz xy yz xz): accepts (..., 3, 3) or (..., 6)."""
    D = np.asarray(D, dtype=np.float64)
    if D.shape[-2:] == (3, 3):
        return np.stack([D[..., 0, 0], D[..., 1, 1], D[..., 2, 2], D[..., 0, 1], D[..., 1, 2], D[..., 0, 2]], -1)
    return D


class OracleSim:
    """A problem set up in the oracle: geometry and lumped matrices in FP64.  n0 (ne x 3): second
    thermal-expansion axis per element (expan_mode 2); D (ne x 3 x 3 or ne x 6): conductivity
    tensor per element (cond_mode 2)."""

    def __init__(self, npe, X, conn, params: dict, a0=None, q=None, fix=None, Tfix=None,
                 t_on=0.0, t_off=float("inf"), dt=0.0, gamma=0.0, n0=None, D=None):
        self.X = _f64(X)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.nn = self.X.shape[0]
        self.ne = self.conn.shape[0]
        self.npe = int(npe)
        self.params = dict(params)
        self.n_prony = int(params.get("n_prony", len(params.get("g", []))))
        self._m = material(params)
        a0 = _f64(a0)
        n0 = _f64(n0)
        D = None if D is None else _f64(sym6(D))
        q = _f64(q)
        fix = None if fix is None else np.ascontiguousarray(fix, dtype=np.uint8)
        Tfix = _f64(Tfix)
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.orc_create(ctypes.byref(h), self.npe, self.nn, _dp(self.X), self.ne,
                              self.conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(a0), _dp(n0),
                              _dp(D), _dp(q),
                              fix.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if fix is not None else None,
                              _dp(Tfix), ctypes.byref(self._m), float(t_on), float(t_off),
                              float(dt), float(gamma))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self._h = h
        self.dt = float(dt)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.orc_destroy(h)
            self._h = None

    @property
    def critical_dt(self) -> float:
        return self._L.orc_critical_dt(self._h)

    @property
    def n_swapped(self) -> int:
        return self._L.orc_n_swapped(self._h)

    def lumped(self):
        out = {k: np.zeros(self.nn) for k in ("Vl", "M", "Kb", "Qm", "Qr")}
        self._L.orc_lumped(self._h, *(_dp(out[k]) for k in ("Vl", "M", "Kb", "Qm", "Qr")))
        return out

    def geometry(self):
        conn = np.zeros((self.ne, self.npe), dtype=np.int32)
        dhdx = np.zeros((self.ne, self.npe, 3))
        V0 = np.zeros(self.ne)
        self._L.orc_geometry(self._h, conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(dhdx), _dp(V0))
        return conn, dhdx, V0

    def initial_state(self, T0: float):
        return {
            "u": np.zeros((self.nn, 3)), "u_prev": np.zeros((self.nn, 3)),
            "T": np.full(self.nn, float(T0)),
            "theta": np.zeros((self.ne, self.n_prony, 6)), "step": 0,
        }

    def run(self, state: dict, nsteps: int, monitors: bool = False):
        """Advance ``state`` in place by ``nsteps``; returns the per-step monitors (nsteps x 6)."""
        for k in ("u", "u_prev", "T", "theta"):
            state[k] = _f64(state[k])
        mon = np.zeros((nsteps, 6)) if monitors else None
        rc = self._L.orc_run(self._h, int(nsteps), int(state["step"]), _dp(state["u"]), _dp(state["u_prev"]),
                           _dp(state["T"]), _dp(state["theta"]) if state["theta"].size else
                           _dp(np.zeros(1)), _dp(mon))
        if rc != 0:
            raise RuntimeError(f"orc_run failed ({rc})")
        state["step"] = int(state["step"]) + int(nsteps)
        return mon

    def run_with_dose(self, state: dict, nsteps: int, A: float, Ea: float):
        """Advance ``state`` by ``nsteps`` one step at a time and add each step's thermal dose at
        the temperatures it ends at to ``state["cem43"]`` and ``state["omega"]`` (created as
        zeros when absent); see ``thermal_dose``."""
        for k in ("cem43", "omega"):
            if k not in state:
                state[k] = np.zeros(self.nn)
        for _ in range(int(nsteps)):
            self.run(state, 1)
            thermal_dose(state["T"], self.dt, A, Ea, state["cem43"], state["omega"])

    def loads(self, u, T):
        """Internal forces (nn x 3) and conduction loads (nn) for a state, without a Prony update."""
        F = np.zeros((self.nn, 3))
        H = np.zeros(self.nn)
        self._L.orc_loads(self._h, _dp(_f64(u)), _dp(_f64(T)), _dp(F), _dp(H))
        return F, H


def thermal_dose(T, dt: float, A: float, Ea: float, cem43, omega):
    """One time step's thermal dose at nodal temperatures T (kelvin), added in place: CEM43
    (Sapareto and Dewey) += (dt/60) R^(43 - T_C), R = 0.5 at T_C >= 43 C and 0.25 below;
    Arrhenius damage (Henriques and Moritz) += dt A exp(-Ea / (R_gas T)) (nothing when A <= 0)."""
    L = lib()
    T = _f64(T)
    assert cem43.dtype == np.float64 and omega.dtype == np.float64
    assert cem43.flags.c_contiguous and omega.flags.c_contiguous
    L.orc_thermal_dose(int(T.size), _dp(T), float(dt), float(A), float(Ea), _dp(cem43), _dp(omega))
