"""Learned surrogate of the solver: binding of the BF16 MFMA network and its workflow.

The network (``include/tled_surrogate.h``) maps a node's coordinates relative to
the probe (random Fourier features) and its scenario's parameters to the node's
temperature rise and displacement at the end of the heating.  It is trained on
the library's own batched solver runs (:func:`make_dataset`) by the library's
forward/backward MFMA kernels (:meth:`MLP.train_step`).  An ensemble of members
trained from different seeds estimates its own uncertainty: a scenario whose
members disagree by more than a threshold on temperature is handed back to the
solver (:func:`plan`).

Every array operation of the network runs in the library's kernels; this module
marshals arguments and runs the training loop.  PyTorch holds device memory.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass

import numpy as np

from . import tled
from .tled import TledError, _lib

_P = ctypes.c_void_p
_f = ctypes.c_float
_fp = ctypes.POINTER(ctypes.c_float)


class MLPConfig(ctypes.Structure):
    _fields_ = [("n_param", ctypes.c_int32), ("n_freq", ctypes.c_int32), ("width", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("n_out", ctypes.c_int32), ("layerwise", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("init_scale", ctypes.c_float), ("seed", ctypes.c_uint64)]


_SIGS = {
    "tled_mlp_create": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(MLPConfig)], ctypes.c_int),
    "tled_mlp_destroy": ([_P], None),
    "tled_mlp_set_stream": ([_P, _P], ctypes.c_int),
    "tled_mlp_param_count": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "tled_mlp_get_params": ([_P, _fp], ctypes.c_int),
    "tled_mlp_set_params": ([_P, _fp], ctypes.c_int),
    "tled_mlp_get_frequencies": ([_P, _fp], ctypes.c_int),
    "tled_mlp_forward": ([_P, ctypes.c_int64, _P, _P, _P], ctypes.c_int),
    "tled_mlp_train_step": ([_P, ctypes.c_int64, _P, _P, _P, _f, _fp], ctypes.c_int),
    "tled_mlp_gradient": ([_P, ctypes.c_int64, _P, _P, _P, _fp, _fp], ctypes.c_int),
    "tled_mlp_gemm": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "tled_mlp_gemm_static": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "tled_mlp_ensemble_stats": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P], ctypes.c_int),
    "tled_mlp_scenario_inputs": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_double,
                                  _P, _P, _P, _P], ctypes.c_int),
    "tled_mlp_scenario_outputs": ([ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
                                  ctypes.c_int),
    "tled_mlp_set_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "tled_mlp_last_timing": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                             ctypes.c_int),
    "tled_mlp_last_error": ([_P], ctypes.c_char_p),
}
for _name, (_a, _r) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _a
    _fn.restype = _r

EXPORTED = tuple(_SIGS)

# Inputs.  Coordinates: node position relative to the probe in units of
# XI_SCALE element sizes (the source is 1/r^2 with core radius h, so the field near
# the probe has a shape common to all resolutions in these units).  Scenario
# parameters (normalised): node position (3, /0.05 m), probe position (3, /0.05 m),
# power (/50 W), heating time (/t_ref), Young's modulus (/4 kPa), element size
# (/2 mm), body (0 cube, 1 ellipsoid).
N_PARAM = 11
XI_SCALE = 8.0
R_REF = 0.02            # m: length in the temperature scale below


def _dp(t):
    return _P(t.data_ptr())


def _need(t, rows, cols, dtype, name):
    """Refuse a tensor the kernels would misread (they take plain row-major device pointers)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: a CUDA/HIP device tensor is required")
    if t.dtype != dtype or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != cols or \
            (rows is not None and t.shape[0] != rows):
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of shape "
                         f"({rows if rows is not None else 'n'}, {cols}), got {tuple(t.shape)} {t.dtype}")


class MLP:
    """One network on one device (device tensors via torch)."""

    def __init__(self, device: int = 0, n_param: int = N_PARAM, n_freq: int = 64, width: int = 256, depth: int = 5,
                 n_out: int = 4, sigma: float = 1.0, seed: int = 0, init_scale: float = 1.0, stream=None,
                 layerwise: bool = False):
        self.cfg = dict(n_param=n_param, n_freq=n_freq, width=width, depth=depth, n_out=n_out)
        c = MLPConfig(n_param, n_freq, width, depth, n_out, int(layerwise), sigma, init_scale, seed)
        h = _P()
        st = _lib.tled_mlp_create(ctypes.byref(h), int(device), ctypes.byref(c))
        if st != 0:
            raise TledError(st, "tled_mlp_create failed")
        self._h = h
        self.device = device
        # The library runs on this stream; every call that takes or returns torch
        # tensors orders it after torch's current stream and torch's current stream
        # after it, so tensors may be made and read on torch's stream as usual.
        import torch
        if stream is None:
            self._stream = torch.cuda.Stream(device=device)
        else:
            self._stream = torch.cuda.ExternalStream(int(stream), device=device)
        self._check(_lib.tled_mlp_set_stream(h, _P(self._stream.cuda_stream)))
        n = ctypes.c_int64()
        self._check(_lib.tled_mlp_param_count(h, ctypes.byref(n)))
        self.n_params = n.value

    def _check(self, st):
        if st != 0:
            raise TledError(st, _lib.tled_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tled_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        self._check(_lib.tled_mlp_get_params(self._h, out.ctypes.data_as(_fp)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, np.float32)
        self._check(_lib.tled_mlp_set_params(self._h, theta.ctypes.data_as(_fp)))

    def frequencies(self) -> np.ndarray:
        out = np.zeros((self.cfg["n_freq"], 3), np.float32)
        self._check(_lib.tled_mlp_get_frequencies(self._h, out.ctypes.data_as(_fp)))
        return out

    def _call(self, fn, *args):
        import torch
        cur = torch.cuda.current_stream(self.device)
        self._stream.wait_stream(cur)
        self._check(fn(self._h, *args))
        cur.wait_stream(self._stream)

    def _inputs(self, x, p, y=None):
        import torch
        _need(x, None, 3, torch.float32, "coords")
        n = x.shape[0]
        if self.cfg["n_param"] > 0:
            _need(p, n, self.cfg["n_param"], torch.float32, "params")
        if y is not None:
            _need(y, n, self.cfg["n_out"], torch.float32, "target")
        for t in (p, y):
            if t is not None and t.device != x.device:
                raise ValueError("all tensors must be on the same device")
        if x.device.index != self.device:
            raise ValueError(f"tensors are on {x.device}, the network on device {self.device}")

    def forward(self, x, p, out=None):
        import torch
        self._inputs(x, p)
        if out is None:
            out = torch.empty((x.shape[0], self.cfg["n_out"]), dtype=torch.float32, device=x.device)
        else:
            _need(out, x.shape[0], self.cfg["n_out"], torch.float32, "out")
        self._call(_lib.tled_mlp_forward, x.shape[0], _dp(x), _dp(p), _dp(out))
        return out

    def train_step(self, x, p, y, lr: float, want_loss: bool = False):
        self._inputs(x, p, y)
        loss = _f(0.0)
        self._call(_lib.tled_mlp_train_step, x.shape[0], _dp(x), _dp(p), _dp(y), float(lr),
                   ctypes.byref(loss) if want_loss else None)
        return loss.value if want_loss else None

    def gradient(self, x, p, y):
        self._inputs(x, p, y)
        g = np.zeros(self.n_params, np.float32)
        loss = _f(0.0)
        self._call(_lib.tled_mlp_gradient, x.shape[0], _dp(x), _dp(p), _dp(y), g.ctypes.data_as(_fp),
                   ctypes.byref(loss))
        return loss.value, g

    def gemm(self, A_bits, B_bits, C):
        """C = A B on the matrix cores; A, B int16 tensors of bfloat16 bits, C float32."""
        import torch
        m, k = A_bits.shape
        n = B_bits.shape[1]
        _need(A_bits, m, k, torch.int16, "A")
        _need(B_bits, k, n, torch.int16, "B")
        _need(C, m, n, torch.float32, "C")
        self._call(_lib.tled_mlp_gemm, m, n, k, _dp(A_bits), _dp(B_bits), _dp(C))

    def gemm_static(self, A_bits, B_bits, C):
        """gemm() through the allocation-free entry point (split-K partials in the library's static
        device scratch array)."""
        import torch
        m, k = A_bits.shape
        n = B_bits.shape[1]
        _need(A_bits, m, k, torch.int16, "A")
        _need(B_bits, k, n, torch.int16, "B")
        _need(C, m, n, torch.float32, "C")
        self._call(_lib.tled_mlp_gemm_static, m, n, k, _dp(A_bits), _dp(B_bits), _dp(C))

    def set_timing(self, on: bool):
        self._check(_lib.tled_mlp_set_timing(self._h, int(on)))

    def timing(self):
        """{"gemm_ms", "gemm_flops", "fused_ms", "fused_flops"} since timing was switched on."""
        ms = (ctypes.c_double * 2)()
        fl = (ctypes.c_double * 2)()
        self._check(_lib.tled_mlp_last_timing(self._h, ms, fl))
        return {"gemm_ms": ms[0], "gemm_flops": fl[0], "fused_ms": ms[1], "fused_flops": fl[1]}


# --------------------------------------------------------------------------- data

def temperature_scale(problem, duration: float) -> float:
    """K: P t / (rho c h^2 R_REF).  The temperature rise near the probe is this
    scale times a shape of order one (energy P t deposited by a 1/r^2 source of
    core radius h, before conduction spreads it)."""
    m = problem.params
    return problem.meta["power"] * duration / (m["rho"] * m["c"] * problem.h ** 2 * R_REF)


def _scenario_params(problem, duration: float, t_ref: float):
    probe = np.asarray(problem.meta["probe"])
    prm = np.array([*(probe / 0.05), problem.meta["power"] / 50.0, duration / t_ref,
                    problem.meta["E"] / 4000.0, problem.h / 2e-3,
                    1.0 if problem.meta["kind"] == "ellipsoid" else 0.0])
    return probe, prm


def fill_inputs(problem, duration: float, t_ref: float, x_out, p_out):
    """Write one scenario's network inputs into preallocated float32 rows (nn x 3, nn x N_PARAM)."""
    probe, prm = _scenario_params(problem, duration, t_ref)
    np.multiply(problem.X - probe, 1.0 / (XI_SCALE * problem.h), out=x_out, casting="same_kind")
    np.multiply(problem.X, 1.0 / 0.05, out=p_out[:, :3], casting="same_kind")
    p_out[:, 3:] = prm


def scenario_inputs(problem, duration: float, t_ref: float):
    x = np.empty((problem.nn, 3), np.float32)
    p = np.empty((problem.nn, N_PARAM), np.float32)
    fill_inputs(problem, duration, t_ref, x, p)
    return x, p


def scaled_targets(problem, duration: float, u, T):
    """Network targets before standardisation: temperature rise / s_T and
    displacement / (alpha s_T h), s_T = temperature_scale."""
    sT = temperature_scale(problem, duration)
    su = problem.params["alpha"] * sT * problem.h
    return np.concatenate([((T - problem.params["T0"]) / sT)[:, None], u / su], axis=1)


def unscale(problem, duration: float, y):
    sT = temperature_scale(problem, duration)
    su = problem.params["alpha"] * sT * problem.h
    return problem.params["T0"] + sT * y[..., 0], su * y[..., 1:]


def solve_snapshots(scenarios, n_snap: int = 5, device: int = 0, stream=None, graph_steps: int = 0, log=None,
                    batch_schedule: int = 0, progress_steps: int = 50000):
    """Runs scenarios [(Problem, duration)] in one batch, each to the end of its heating,
    and reads every scenario's fields at n_snap evenly spaced batch steps.  A snapshot
    of a scenario at heating time t is the solution of the same scenario with
    duration t (the source is on from t = 0 and the past does not depend on a later
    switch-off).  Returns (list of (scenario index, duration, u, T), solver seconds)."""
    b = tled.Batch(device, stream=stream)
    b.set_options(graph_steps=graph_steps, batch_schedule=batch_schedule)
    for p, dur in scenarios:
        b.add(p, cfl=p.cfl, t_end=dur)
    b.finalize()
    dts, steps = zip(*(b.scenario_steps(k) for k in range(len(scenarios))))
    S = max(steps)
    marks = sorted(set(max(1, int(round(S * j / n_snap))) for j in range(1, n_snap + 1)))
    snaps, last, done, el = [], [0] * len(scenarios), 0, 0.0
    for k in marks:
        b.sync()
        while done < k:                      # in slices, with a progress line each (long runs)
            c = min(k - done, progress_steps)
            t0 = time.perf_counter()
            b.step(c)
            b.sync()
            el += time.perf_counter() - t0
            done += c
            if log and done < k:
                log(f"[surrogate] batch step {done}/{S}, {el:.1f}s")
        fields = b.read_all()
        for s, (u, T) in enumerate(fields):
            n = min(k, steps[s])
            if n > last[s]:
                snaps.append((s, n * dts[s], u.copy(), T.copy()))
                last[s] = n
        if log:
            log(f"[surrogate] snapshot at batch step {k}/{S}: {len(snaps)} fields")
    b.close()
    return snaps, el


def solve(scenarios, device: int = 0, stream=None, graph_steps: int = 0, torch_allocator: bool = False,
          batch_schedule: int = 0, log=None, progress_steps: int = 200000):
    """Solver alone: one batch, every scenario to the end of its heating.
    Returns ([(u, T)], {"setup": s, "run": s, "total": s}): set-up = host precompute and
    upload, run = GPU stepping and the read-back of every field.  With `log`, the steps
    run in slices of progress_steps with a progress line after each (long runs)."""
    t0 = time.perf_counter()
    b = tled.Batch(device, stream=stream, use_torch_allocator=torch_allocator)
    b.set_options(graph_steps=graph_steps, batch_schedule=batch_schedule)
    for p, dur in scenarios:
        b.add(p, cfl=p.cfl, t_end=dur)
    b.finalize()
    b.sync()
    t1 = time.perf_counter()
    if log:
        total = b.batch_info()["max_steps"]
        done = 0
        while done < total:
            c = min(progress_steps, total - done)
            b.step(c)
            b.sync()
            done += c
            log(f"[surrogate] solver batch step {done}/{total}, {time.perf_counter() - t1:.1f}s")
    else:
        b.run()
    out = [(u.copy(), T.copy()) for u, T in b.read_all()]
    t2 = time.perf_counter()
    b.close()
    return out, {"setup": t1 - t0, "run": t2 - t1, "total": t2 - t0}


@dataclass
class Dataset:
    x: np.ndarray        # samples x 3
    p: np.ndarray        # samples x N_PARAM
    y: np.ndarray        # samples x 4 (scaled targets)
    field: np.ndarray    # snapshot index per sample


def make_dataset(scenarios, snaps, t_ref: float) -> Dataset:
    xs, ps, ys, fs = [], [], [], []
    for j, (s, dur, u, T) in enumerate(snaps):
        prob = scenarios[s][0]
        x, p = scenario_inputs(prob, dur, t_ref)
        xs.append(x)
        ps.append(p)
        ys.append(scaled_targets(prob, dur, u, T).astype(np.float32))
        fs.append(np.full(len(x), j, np.int32))
    return Dataset(np.concatenate(xs), np.concatenate(ps), np.concatenate(ys), np.concatenate(fs))


def _shard_nodes(nn: int, scenario: int, ordinal: int, per_field: int, seed: int):
    """Node subsample of one stored field: a seeded draw from (seed, scenario, snapshot ordinal)."""
    rng = np.random.default_rng([seed, scenario, ordinal])
    return np.sort(rng.choice(nn, size=min(nn, per_field), replace=False))


def write_shard(path: str, scenarios, first: int, snaps, per_field: int = 2048, seed: int = 17):
    """Stores a node subsample of every snapshot field of scenarios[first:first + len] (solver runs
    of the training set), so that data made in separate runs can be combined: per field the global
    scenario index, its snapshot ordinal and duration, and the scaled targets (temperature in
    float32, displacement in float16) at nodes drawn by _shard_nodes (not stored: they are drawn
    again when the shard is read, as are the coordinates, from the seeded scenario generator)."""
    meta, yT, yu, ordinal = [], [], [], {}
    for s, dur, u, T in snaps:                 # s: position in the slice that starts at `first`
        prob = scenarios[first + s][0]
        j = ordinal.get(s, 0)
        ordinal[s] = j + 1
        idx = _shard_nodes(prob.nn, first + s, j, per_field, seed)
        y = scaled_targets(prob, dur, u[idx], T[idx])
        meta.append((first + s, j, dur, len(idx)))
        yT.append(y[:, 0].astype(np.float32))
        yu.append(y[:, 1:].astype(np.float16))
    m = np.array(meta, dtype=[("scenario", "i4"), ("ordinal", "i4"), ("duration", "f8"), ("n", "i4")])
    np.savez_compressed(path, scenario=m["scenario"], ordinal=m["ordinal"], duration=m["duration"], n=m["n"],
                        yT=np.concatenate(yT), yu=np.concatenate(yu), per_field=per_field, seed=seed)


def dataset_from_shards(paths, scenarios, t_ref: float) -> Dataset:
    """Training set from shards written by write_shard for the scenario list `scenarios` (indices
    are global positions in it)."""
    xs, ps, ys, fs, field = [], [], [], [], 0
    for path in paths:
        z = np.load(path, allow_pickle=False)
        per, seed = int(z["per_field"]), int(z["seed"])
        yT, yu = z["yT"], z["yu"]              # each access to the archive decompresses the array
        off = 0
        for s, j, dur, n in zip(z["scenario"], z["ordinal"], z["duration"], z["n"]):
            prob = scenarios[int(s)][0]
            idx = _shard_nodes(prob.nn, int(s), int(j), per, seed)
            if len(idx) != n:
                raise ValueError(f"shard {path}: field of scenario {s} does not match the scenario list")
            x, p = scenario_inputs(prob, float(dur), t_ref)
            xs.append(x[idx])
            ps.append(p[idx])
            ys.append(np.concatenate([yT[off:off + n, None], yu[off:off + n].astype(np.float32)], 1))
            fs.append(np.full(n, field, np.int32))
            field += 1
            off += n
    return Dataset(np.concatenate(xs), np.concatenate(ps), np.concatenate(ys), np.concatenate(fs))


class Ensemble:
    """K networks trained from different seeds on standardised targets; the
    spread of their temperature predictions, times a factor calibrated on
    held-back solver runs, is the disagreement estimate."""

    def __init__(self, k: int = 4, device: int = 0, t_ref: float = 0.3, stream=None, **net):
        self.models = [MLP(device, seed=1000 + i, stream=stream, **net) for i in range(k)]
        self.device = device
        self.t_ref = t_ref
        self.y_std = np.ones(4, np.float32)
        self.calib = 1.0
        self.last_forward_s = 0.0

    def fit(self, data: Dataset, epochs: int, batch: int = 16384, lr: float = 2e-3, log=None):
        self.y_std = data.y.std(0).astype(np.float32) + np.float32(1e-12)
        d = Dataset(data.x, data.p, (data.y / self.y_std).astype(np.float32), data.field)
        t0 = time.perf_counter()
        hist = [train(m, d, epochs, batch=batch, lr=lr, seed=i, log=log) for i, m in enumerate(self.models)]
        return hist, time.perf_counter() - t0

    def _forward_device(self, X, Pm):
        """Member outputs (device inputs) into one K x n x 4 device array, then the library's
        ensemble statistics kernel: device (mean of the scaled targets n x 4, spread of target 0)."""
        import torch
        dev = torch.device("cuda", self.device)
        n, K = X.shape[0], len(self.models)
        outs = torch.empty((K, n, 4), dtype=torch.float32, device=dev)
        mean = torch.empty((n, 4), dtype=torch.float32, device=dev)
        spread = torch.empty(n, dtype=torch.float32, device=dev)
        scale = torch.from_numpy(self.y_std).to(dev)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for k, m in enumerate(self.models):
            m.forward(X, Pm, out=outs[k])
        st = _lib.tled_mlp_ensemble_stats(n, K, 4, _dp(outs), _dp(scale), _dp(mean), _dp(spread),
                                          _P(torch.cuda.current_stream(dev).cuda_stream))
        if st != 0:
            raise TledError(st, "tled_mlp_ensemble_stats failed")
        torch.cuda.synchronize(dev)
        self.last_forward_s = time.perf_counter() - t0
        return mean, spread

    def predict_many(self, items):
        """items [(Problem, duration)] -> [(T mean, u mean, T spread)] (FP32).  The nodes of all
        scenarios go to the device once (FP64 coordinates and a few constants per scenario); the
        library assembles the network inputs there (bitwise those of fill_inputs), the members
        run, and the library turns the ensemble statistics into physical fields (bitwise those of
        unscale), which come back in one copy."""
        import torch
        dev = torch.device("cuda", self.device)
        S = len(items)
        sizes = np.array([p.nn for p, _ in items], np.int64)
        offs = np.zeros(S + 1, np.int64)
        np.cumsum(sizes, out=offs[1:])
        n = int(offs[-1])
        probe = np.empty((S, 3))
        xi = np.empty(S)
        prm = np.empty((S, N_PARAM - 3), np.float32)
        T0 = np.empty(S, np.float32)
        sT = np.empty(S, np.float32)
        su = np.empty(S, np.float32)
        for k, (p, d) in enumerate(items):
            probe[k], prm[k] = _scenario_params(p, d, self.t_ref)
            xi[k] = 1.0 / (XI_SCALE * p.h)
            s_t = temperature_scale(p, d)
            T0[k], sT[k], su[k] = p.params["T0"], s_t, p.params["alpha"] * s_t * p.h
        Xd = torch.from_numpy(np.concatenate([np.asarray(p.X, np.float64) for p, _ in items])).to(dev)
        tab = {name: torch.from_numpy(a).to(dev) for name, a in
               (("offs", offs), ("probe", probe), ("xi", xi), ("prm", prm), ("T0", T0), ("sT", sT), ("su", su))}
        x_in = torch.empty((n, 3), dtype=torch.float32, device=dev)
        p_in = torch.empty((n, N_PARAM), dtype=torch.float32, device=dev)
        stream = _P(torch.cuda.current_stream(dev).cuda_stream)
        st = _lib.tled_mlp_scenario_inputs(S, N_PARAM - 3, n, _dp(tab["offs"]), _dp(Xd), _dp(tab["probe"]),
                                           _dp(tab["xi"]), 1.0 / 0.05, _dp(tab["prm"]), _dp(x_in), _dp(p_in), stream)
        if st != 0:
            raise TledError(st, "tled_mlp_scenario_inputs failed")
        mean, spread = self._forward_device(x_in, p_in)
        out_d = torch.empty(5 * n, dtype=torch.float32, device=dev)      # T | u | spread
        st = _lib.tled_mlp_scenario_outputs(S, n, _dp(tab["offs"]), _dp(mean), _dp(spread), _dp(tab["T0"]),
                                            _dp(tab["sT"]), _dp(tab["su"]), _dp(out_d[:n]), _dp(out_d[n:4 * n]),
                                            _dp(out_d[4 * n:]), stream)
        if st != 0:
            raise TledError(st, "tled_mlp_scenario_outputs failed")
        host = out_d.cpu().numpy()
        T, u, sp = host[:n], host[n:4 * n].reshape(n, 3), host[4 * n:]
        return [(T[a:b], u[a:b], sp[a:b]) for a, b in zip(offs[:-1], offs[1:])]

    def calibrate(self, items, fields):
        """Factor c with max|T - T_solver| <= c * max spread on every calibration field."""
        preds = self.predict_many(items)
        r = [np.abs(Tm - T).max() / max(sp.max(), 1e-12) for (Tm, _, sp), (_, T) in zip(preds, fields)]
        self.calib = float(max(r)) if r else 1.0
        return self.calib

    def disagreement(self, spread):
        return self.calib * float(spread.max())


def train(model: MLP, data: Dataset, epochs: int, batch: int = 16384, lr: float = 2e-3, seed: int = 0, log=None):
    """Minibatch Adam over the dataset (device-resident); cosine learning-rate decay."""
    import torch
    dev = torch.device("cuda", model.device)
    X = torch.from_numpy(data.x).to(dev)
    Pm = torch.from_numpy(data.p).to(dev)
    Y = torch.from_numpy(data.y).to(dev)
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    it = 0
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb, pb, yb = X[idx].contiguous(), Pm[idx].contiguous(), Y[idx].contiguous()
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * it / total))
            want = (s == steps_per_epoch - 1)
            loss = model.train_step(xb, pb, yb, lr_t, want_loss=want)
            if want:
                losses.append(loss)
            it += 1
        if log and (ep % max(1, epochs // 5) == 0 or ep == epochs - 1):
            log(f"[surrogate] seed {seed} epoch {ep + 1}/{epochs} loss {losses[-1]:.4g}")
    return losses


def plan(ens: Ensemble, items, threshold_K: float = 0.5, device: int = 0, stream=None, log=None,
         batch_schedule: int = 0, graph_steps: int = 0):
    """Surrogate-first planning of items [(Problem, duration)]: every scenario is
    predicted by the ensemble; those whose disagreement estimate exceeds
    threshold_K are run by the solver instead.  Returns results and timings
    (t_surrogate: input assembly on the host + ensemble inference + read-back;
    t_surrogate_gpu: the inference calls alone)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preds = ens.predict_many(items)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    est = [ens.disagreement(sp) for _, _, sp in preds]
    reject = [k for k, e in enumerate(est) if e > threshold_K]
    t_fb, fallback = {"setup": 0.0, "run": 0.0, "total": 0.0}, {}
    if reject:
        fields, t_fb = solve([items[k] for k in reject], device=device, stream=stream, log=log,
                             batch_schedule=batch_schedule, graph_steps=graph_steps)
        fallback = dict(zip(reject, fields))
    results = []
    for k, (Tm, um, _) in enumerate(preds):
        if k in fallback:
            u, T = fallback[k]
            results.append(("solver", u, T))
        else:
            results.append(("surrogate", um, Tm))
    return {"results": results, "t_surrogate": t_sur, "t_surrogate_gpu": ens.last_forward_s, "t_fallback": t_fb,
            "rejected": reject, "estimate": est}
