"""CPU-side checks of the library: it loads, exports every symbol the C header declares, and its
host-only set-up (validation, FP64 precompute, reordering, patch partition) agrees with the
oracle's independent precompute.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2009_10400_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tled.h")
SURROGATE_HEADER = os.path.join(ROOT, "include", "tled_surrogate.h")


def declared_symbols(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tled_[A-Za-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2009_10400_amd import tled
    lib = ctypes.CDLL(tled.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(tled.EXPORTED)


def test_library_exports_every_surrogate_symbol():
    from paper_2009_10400_amd import surrogate, tled
    lib = ctypes.CDLL(tled.LIB_PATH)
    syms = declared_symbols(SURROGATE_HEADER)
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(surrogate.EXPORTED)


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    """The product path fails loudly when the HIP library is missing (no CPU fallback)."""
    import importlib.util
    import shutil
    pkg = tmp_path / "pkg"
    (pkg / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "paper_2009_10400_amd", "tled.py"), pkg / "tled.py")
    spec = importlib.util.spec_from_file_location("tled_missing", pkg / "tled.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def host_sim(problem, dt=None, **opts):
    from paper_2009_10400_amd import tled
    return tled.from_problem(problem, dt=dt if dt is not None else 1e-5, device=-1, **opts)


def default_patch_elems(npe, ne):
    """The documented default: H8 256; T4 the smallest multiple of 8 (at least 128) that
    fills the fewest whole rounds of 1024 resident workgroups with patches of at most 504."""
    if npe == 8:
        return 256
    k = 1
    while True:
        pe = -(-(-(-ne // (1024 * k))) // 8) * 8
        if pe <= 504:
            return max(pe, 128)
        k += 1


def test_default_patch_size_fills_whole_rounds():
    assert default_patch_elems(4, 6000) == 128
    assert default_patch_elems(4, 1_001_328) == 496          # 2019 patches: two rounds of 1024
    assert default_patch_elems(4, 2_002_566) == 496          # 4038 patches: four rounds
    assert default_patch_elems(4, 1024 * 504 + 1) == 256     # one element too many for one round
    for n in (30000, 500_000):
        p = W.ellipsoid_t4(n)
        info = host_sim(p).info()
        pe = default_patch_elems(4, p.ne)
        assert info["n_patches"] == -(-p.ne // pe)
        rounds = -(-info["n_patches"] // 1024)
        if pe > 128:      # the next smaller size would need another round
            assert -(-p.ne // (pe - 8)) > rounds * 1024
        assert info["n_patches"] <= rounds * 1024
    # 512-thread workgroups: two per CU, patches of at most 704 elements (one workgroup's LDS)
    p = W.ellipsoid_t4(500_000)
    info = host_sim(p, block_size=512).info()
    pe = -(-(-(-p.ne // 1024)) // 8) * 8      # one round of 512 would need 984: two rounds
    assert pe <= 704 and info["n_patches"] == -(-p.ne // pe)
    assert info["patch_lds_bytes"] <= 65536 - 1024


@pytest.mark.parametrize("name", ["cube_t4", "cube_h8", "ellipsoid"])
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_host_precompute_matches_oracle(name, variant):
    p = {"cube_t4": lambda: W.cube_t4(), "cube_h8": lambda: W.cube_h8(n=10),
         "ellipsoid": lambda: W.ellipsoid_t4(20000)}[name]()
    s = host_sim(p, kernel_variant=variant)
    o = oracle.OracleSim(p.npe, p.X, p.conn, p.params, a0=p.a0, q=p.q, fix=p.fix, dt=1e-5)
    assert s.critical_dt() == pytest.approx(o.critical_dt, rel=1e-12)
    L, Lo = s.lumped(), o.lumped()
    for k in ("Vl", "M", "Kb", "Qm", "Qr"):
        scale = max(np.abs(Lo[k]).max(), 1e-300)
        assert np.abs(L[k] - Lo[k]).max() <= 1e-12 * scale, k
    assert L["C"] == pytest.approx(p.params["rho"] * p.params["c"] * Lo["Vl"], rel=1e-12)
    info = s.info()
    assert info["kernel_variant"] == variant
    assert info["n_nodes"] == p.nn and info["n_elems"] == p.ne
    if variant >= 2:
        assert info["n_patches"] == -(-p.ne // default_patch_elems(p.npe, p.ne))
        assert 0 < info["n_shared_nodes"] < p.nn


def test_orientation_repair_counted():
    p = W.cube_t4(n=4, L=0.016)
    rng = np.random.default_rng(1)
    flip = rng.random(p.ne) < 0.4
    p.conn[flip] = p.conn[flip][:, [0, 1, 3, 2]]
    s = host_sim(p)
    assert s.info()["n_swapped"] == flip.sum()


def test_setup_errors():
    from paper_2009_10400_amd import tled
    p = W.cube_t4(n=2, L=0.01)
    s = tled.Sim(-1)
    with pytest.raises(tled.TledError) as e:
        s.set_mesh(5, p.X, p.conn)
    assert e.value.status == tled.E_ARG
    bad = p.conn.copy(); bad[0, 0] = p.nn + 3
    s.set_mesh(4, p.X, bad)
    s.set_material(p.params)
    s.set_time(1e-6, 0.0)
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_MESH
    s = tled.Sim(-1)
    s.set_mesh(4, p.X, p.conn)
    s.set_material(dict(p.params, g=[0.6, 0.5], tau=[1, 1], n_prony=2))
    s.set_time(1e-6, 0.0)
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_ARG and "Prony" in str(e.value)
    s = tled.Sim(-1)
    s.set_mesh(4, p.X, p.conn)
    s.set_material(p.params)
    s.set_time(1.0, 0.0)            # far above the critical step
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_ARG
    # inverted H8
    X, conn, h = W.box_mesh("h8", 2, 0.01)
    conn = conn.copy(); conn[0] = conn[0][[4, 5, 6, 7, 0, 1, 2, 3]]
    s = tled.Sim(-1)
    s.set_mesh(8, X, conn)
    s.set_material(p.params)
    s.set_time(1e-6, 0.0)
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_MESH
    # orphan node
    X2 = np.vstack([p.X, [[1.0, 1.0, 1.0]]])
    s = tled.Sim(-1)
    s.set_mesh(4, X2, p.conn)
    s.set_material(p.params)
    s.set_time(1e-6, 0.0)
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_MESH


def test_host_handle_refuses_stepping():
    from paper_2009_10400_amd import tled
    s = host_sim(W.cube_t4(n=2, L=0.01))
    with pytest.raises(tled.TledError) as e:
        s.step(1)
    assert e.value.status == tled.E_STATE
    with pytest.raises(tled.TledError) as e:
        s.read_u()
    assert e.value.status == tled.E_STATE


def test_batch_host_setup_and_errors():
    from paper_2009_10400_amd import tled
    sc = W.planning_scenarios(4, seed=5, lo=1000, hi=4000)
    b = tled.Batch(-1)
    ne = nn = 0
    for p, _ in sc:
        b.add(p, 1e-5, 10)
        ne += p.ne
        nn += p.nn
    b.finalize()
    info = b.batch_info()
    assert info["n_scenarios"] == 4 and info["n_elems"] == ne and info["n_nodes"] == nn
    assert info["max_steps"] == 10 and info["n_patches"] >= 4
    # mixed element types and a too-large dt are refused
    b2 = tled.Batch(-1)
    b2.add(sc[0][0], 1e-5, 10)
    with pytest.raises(tled.TledError) as e:
        b2.add(W.cube_h8(n=3), 1e-5, 10)
    assert e.value.status == tled.E_ARG
    b3 = tled.Batch(-1)
    b3.add(sc[0][0], 0.01, 10)          # above the critical step (~1e-3 s)
    with pytest.raises(tled.TledError) as e:
        b3.finalize()
    assert e.value.status == tled.E_ARG
    # the single-problem calls refuse a batch handle
    with pytest.raises(tled.TledError) as e:
        b.set_time(1e-5, 0.0)
    assert e.value.status == tled.E_STATE


def test_batch_duration_picks_fraction_of_critical_step():
    """tled_batch_set_duration: dt = cfl x the scenario's critical step, n = round(t_end / dt)."""
    from paper_2009_10400_amd import tled
    sc = W.planning_scenarios(3, seed=8, lo=1000, hi=4000, duration_scale=1e-3)
    b = tled.Batch(-1)
    b.add(sc[0][0], 1e-5, 7)                               # explicit
    for p, dur in sc[1:]:
        b.add(p, cfl=0.8, t_end=dur)                       # chosen at finalize
    with pytest.raises(tled.TledError):
        b.scenario_steps(0)                                # not finalized yet
    b.finalize()
    assert b.scenario_steps(0) == (1e-5, 7)
    for k, (p, dur) in enumerate(sc[1:], start=1):
        s = host_sim(p)
        dt, n = b.scenario_steps(k)
        assert dt == pytest.approx(0.8 * s.critical_dt(), rel=1e-14)
        assert n == max(1, round(dur / dt))
    # dt 0 without a duration, or a cfl outside (0, 1], is refused
    b2 = tled.Batch(-1)
    b2.add(sc[0][0], 0.0, 10)
    with pytest.raises(tled.TledError) as e:
        b2.finalize()
    assert e.value.status == tled.E_ARG
    with pytest.raises(tled.TledError) as e:
        b2.add(sc[0][0], cfl=1.5, t_end=1.0)
    assert e.value.status == tled.E_ARG


def test_batch_setup_is_independent_of_host_threads(monkeypatch):
    """The per-scenario precompute runs on a thread pool; results do not depend on its size."""
    from paper_2009_10400_amd import tled
    sc = W.planning_scenarios(5, seed=9, lo=1000, hi=6000, duration_scale=1e-3)
    infos = []
    for n in ("1", "3"):
        monkeypatch.setenv("TLED_HOST_THREADS", n)
        b = tled.Batch(-1)
        for p, dur in sc:
            b.add(p, cfl=0.8, t_end=dur)
        b.finalize()
        infos.append((b.batch_info(), [b.scenario_steps(k) for k in range(len(sc))]))
        b.close()
    assert infos[0] == infos[1]


def _tet_gradients(X, conn):
    """Shape-function gradients (ne x 4 x 3) and volumes of linear tets (numpy, FP64)."""
    D = np.stack([X[conn[:, k]] - X[conn[:, 0]] for k in (1, 2, 3)], axis=2)   # columns X_k - X_0
    Di = np.linalg.inv(D)
    g = np.concatenate([-Di.sum(axis=1, keepdims=True), Di], axis=1)
    return g, np.abs(np.linalg.det(D)) / 6.0


def test_thermal_stability_bound():
    """dt_thermal = 2 min_a C_a / (sum_b |K_ab| bound + K_b,a) on the reference geometry; it bounds
    the true largest eigenvalue of C^-1 (K + K_b), and finalize refuses a larger dt."""
    from paper_2009_10400_amd import tled
    p = W.cube_t4(n=3, L=0.01)
    info = host_sim(p).info()
    m = p.params
    g, V = _tet_gradients(p.X, p.conn)
    gn = np.linalg.norm(g, axis=2)                                           # |dh_a/dX|
    nn = len(p.X)
    rows = np.zeros(nn)
    Vl = np.zeros(nn)
    K = np.zeros((nn, nn))
    kmax = m["k"] * max(1.0, m["k_hi"] / m["k"]) if m.get("ckT_on") else m["k"]
    for e, c in enumerate(p.conn):
        rows[c] += V[e] * kmax * gn[e] * gn[e].sum()
        Vl[c] += V[e] / 4
        K[np.ix_(c, c)] += V[e] * kmax * g[e] @ g[e].T
    cmin = min(m["c"], m["c_hi"]) if m.get("ckT_on") else m["c"]
    C = m["rho"] * cmin * Vl
    expect = 2.0 * np.min(C / (rows + m["wbcb"] * Vl))
    assert info["dt_thermal"] == pytest.approx(expect, rel=1e-12)
    lam = np.max(np.linalg.eigvals((K + np.diag(m["wbcb"] * Vl)) / C[:, None]).real)
    assert 2.0 / lam >= info["dt_thermal"] * (1 - 1e-12)          # the bound is conservative
    assert info["dt_thermal"] > info["dt_critical"]                # mechanics sets the step here
    # a conductivity high enough to make the thermal bound binding is refused at finalize
    hot = W.cube_t4(n=3, L=0.01)
    hot.params = dict(hot.params, k=1e6, k_hi=1e6)
    s = tled.from_problem(hot, dt=1e-5, device=-1, finalize=False)
    with pytest.raises(tled.TledError) as e:
        s.finalize()
    assert e.value.status == tled.E_ARG and "thermal" in str(e.value)


def test_bisection_patches_on_a_regular_grid():
    # 16^3 hexahedra in patches of 256: every cut is a grid plane, so the patches
    # are 4x8x8 boxes (in some orientation) and the shared nodes are those on the
    # internal planes -- three planes across one axis, one across each other:
    # 17^3 - (17 - 3)(17 - 1)(17 - 1)
    p = W.cube_h8(n=16)
    for r in (0, 1, 2):
        info = host_sim(p, reorder=r).info()
        assert info["n_patches"] == 16
        assert info["n_shared_nodes"] == 17 ** 3 - 14 * 16 * 16


def test_bisection_patches_beat_morton_runs_on_tetrahedra():
    from paper_2009_10400_amd import tled
    p = W.ellipsoid_t4(100_000)
    bis, runs = host_sim(p, reorder=1, patch_elems=448).info(), host_sim(p, reorder=2, patch_elems=448).info()
    assert bis["n_patches"] == runs["n_patches"]
    assert bis["n_shared_nodes"] < 0.95 * runs["n_shared_nodes"]
    assert bis["patch_max_nodes"] < runs["patch_max_nodes"]
    assert bis["patch_lds_bytes"] < runs["patch_lds_bytes"]
    assert host_sim(p, patch_elems=448).info() == bis     # the default order, and deterministic
    with pytest.raises(tled.TledError) as e:
        host_sim(W.cube_t4(n=2, L=0.01), reorder=3)
    assert e.value.status == tled.E_ARG


def test_single_setup_is_independent_of_host_threads(monkeypatch):
    """The element pass and the bisection of one problem run on several host threads; the
    layout and the first reported mesh error do not depend on how many."""
    from paper_2009_10400_amd import tled
    p = W.ellipsoid_t4(200_000)
    bad = p.conn.copy()
    for e in (150_000, 40_000):                 # two zero-volume elements: the lower one is reported
        bad[e, 3] = bad[e, 2]
    out = []
    for n in ("1", "8"):
        monkeypatch.setenv("TLED_HOST_THREADS", n)
        s = host_sim(p)
        out.append((s.info(), s.lumped()["M"].tobytes()))
        s = tled.Sim(-1)
        s.set_mesh(4, p.X, bad)
        s.set_material(p.params)
        s.set_time(1e-6, 0.0)
        with pytest.raises(tled.TledError) as e:
            s.finalize()
        out.append(str(e.value))
    assert out[0] == out[2] and out[1] == out[3]
    assert "element 40000 " in out[1]


def _spread3(q):
    q = q.astype(np.uint64) & np.uint64(0x1FFFFF)
    for sh, m in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                  (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        q = (q | (q << np.uint64(sh))) & np.uint64(m)
    return q


def _bisection_patches(X, conn, P):
    """Recursive coordinate bisection written independently of the library: Morton keys of the
    element centroids over the bounding cube; a set of M > P elements (q = ceil(M/P) patches) is
    cut across the longest centroid extent into floor(q/2) P elements and the rest (ties by
    element number, equal extents to the lower axis); leaves in (key, element) order.  Only sets
    matter, so full sorts give the same patches as partial ones."""
    ne, npe = conn.shape
    c = X[conn[:, 0]].copy()
    for a in range(1, npe):
        c += X[conn[:, a]]
    c /= npe
    lo, span = X.min(0), max((X.max(0) - X.min(0)).max(), 1e-300)
    t = np.clip((c - lo) / span * 2097151.0, 0.0, 2097151.0).astype(np.uint64)
    key = _spread3(t[:, 0]) | (_spread3(t[:, 1]) << np.uint64(1)) | (_spread3(t[:, 2]) << np.uint64(2))
    order = np.arange(ne)
    todo = [(0, ne)]
    while todo:
        a, b = todo.pop()
        sub = order[a:b]
        if b - a <= P:
            order[a:b] = sub[np.lexsort((sub, key[sub]))]
            continue
        ext = c[sub].max(0) - c[sub].min(0)
        ax = 0
        for i in (1, 2):
            if ext[i] > ext[ax] * (1.0 + 1e-9):
                ax = i
        order[a:b] = sub[np.lexsort((sub, c[sub, ax]))]
        left = (-(-(b - a) // P) // 2) * P
        todo += [(a + left, b), (a, a + left)]
    pid = np.empty(ne, np.int64)
    pid[order] = np.arange(ne) // P
    pairs = np.unique(np.stack([np.repeat(pid, npe), conn.reshape(-1)], 1), axis=0)
    touched = np.bincount(pairs[:, 1], minlength=len(X))
    return int((touched > 1).sum()), int(np.bincount(pairs[:, 0]).max())


@pytest.mark.parametrize("n, P", [(30_000, 448), (30_000, 128), (100_000, 496)])
def test_bisection_patches_match_an_independent_implementation(n, P):
    p = W.ellipsoid_t4(n)
    n_shared, max_nodes = _bisection_patches(np.asarray(p.X, np.float64), np.asarray(p.conn), P)
    info = host_sim(p, patch_elems=P).info()
    assert info["n_patches"] == -(-p.ne // P)
    assert info["n_shared_nodes"] == n_shared
    assert info["patch_max_nodes"] == max_nodes


def test_anisotropic_setup_errors_and_thermal_bound():
    """Orthotropic expansion (Eq. 11) and element conductivity tensors (Eqs. 15-16) at set-up: a
    missing second axis or tensor, an axis parallel to the fibre and a tensor that is not positive
    semi-definite are refused with TLED_E_ARG; batches refuse both modes; the explicit thermal bound
    with a tensor k I is no larger than with the scalar k (its Frobenius norm bounds the largest
    eigenvalue)."""
    from paper_2009_10400_amd import tled
    cases = ((dict(expan_mode=2), None, None), (dict(cond_mode=2), None, None),
             (dict(expan_mode=2), lambda ne: np.tile([2.0, 0.0, 0.0], (ne, 1)), None),
             (dict(cond_mode=2), None, lambda ne: np.tile(np.diag([1.0, -0.5, 1.0]), (ne, 1, 1))),
             (dict(cond_mode=2), None, lambda ne: np.tile([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]],
                                                          (ne, 1, 1))))
    for params, n0, D in cases:
        q = W.cube_t4(n=2, L=0.01)
        q.params = dict(q.params, **params)
        q.n0 = n0(q.ne) if n0 else None
        q.D = D(q.ne) if D else None
        with pytest.raises(tled.TledError) as ei:
            host_sim(q)
        assert ei.value.status == tled.E_ARG, params
    p = W.cube_t4(n=3, L=0.012)
    ok = W.cube_t4(n=3, L=0.012)
    ok.params = dict(ok.params, cond_mode=2, expan_mode=2, alpha_m=3e-4, alpha_n=-1e-4)
    ok.D = np.tile(ok.params["k"] * np.eye(3), (ok.ne, 1, 1))
    ok.n0 = np.tile([0.2, 1.0, 0.0], (ok.ne, 1))
    dt_iso, dt_ten = host_sim(p).info()["dt_thermal"], host_sim(ok).info()["dt_thermal"]
    assert 0.0 < dt_ten <= dt_iso
    b = tled.Batch(-1)
    with pytest.raises(tled.TledError) as ei:
        b.add(ok, dt=1e-5, n_steps=1)
    assert ei.value.status == tled.E_UNSUPPORTED
    s = tled.Sim(-1)
    s.set_mesh(4, p.X, p.conn)
    with pytest.raises(ValueError):
        s.set_expansion_axes(np.zeros((p.ne + 1, 3)))
    with pytest.raises(ValueError):
        s.set_conductivity(np.zeros((p.ne, 5)))


def test_shared_update_option():
    """Where the shared nodes are advanced: by a kernel of their own unless asked otherwise;
    inside the next step's patch kernel when asked, for single problems with kernel variant 2,
    256 threads and no anisotropy plane; nothing to report without patches.  Set before
    finalize only."""
    from paper_2009_10400_amd import tled
    t4, h8 = W.cube_t4(), W.cube_h8(n=8)
    assert host_sim(t4).info()["shared_update"] == 2                     # default: a kernel of their own
    assert host_sim(h8).info()["shared_update"] == 2
    assert host_sim(h8, shared_update=1).info()["shared_update"] == 2    # H8 default: variant 3
    assert host_sim(h8, kernel_variant=2, shared_update=1).info()["shared_update"] == 1
    assert host_sim(t4, shared_update=1).info()["shared_update"] == 1
    assert host_sim(t4, shared_update=2).info()["shared_update"] == 2
    assert host_sim(t4, kernel_variant=3, shared_update=1).info()["shared_update"] == 2
    assert host_sim(t4, block_size=512, shared_update=1).info()["shared_update"] == 2
    assert host_sim(t4, kernel_variant=1).info()["shared_update"] == 0
    ortho = W.cube_t4()
    ortho.params = dict(ortho.params, cond_mode=2)
    ortho.D = np.tile(np.array([0.5, 0.6, 0.7, 0.0, 0.0, 0.0]), (ortho.ne, 1))
    assert host_sim(ortho, shared_update=1).info()["shared_update"] == 2
    s = host_sim(t4)
    with pytest.raises(tled.TledError) as e:
        s.set_options(shared_update=1)
    assert e.value.status == tled.E_STATE
    with pytest.raises(tled.TledError) as e:
        host_sim(t4, shared_update=3)
    assert e.value.status == tled.E_ARG
    # one patch: no shared node
    assert host_sim(W.cube_h8(n=6)).info()["shared_update"] == 0


def test_thermal_dose_setup_errors():
    """tled_set_thermal_dose: before finalize, single problems only, finite non-negative
    Arrhenius parameters; reading needs a device handle with the dose enabled."""
    from paper_2009_10400_amd import tled
    p = W.cube_t4(n=2, L=0.01)
    s = tled.from_problem(p, dt=1e-5, device=-1, finalize=False)
    for A, Ea in ((-1.0, 1e5), (1e10, -1.0), (float("inf"), 1e5), (1e10, float("nan"))):
        with pytest.raises(tled.TledError) as e:
            s.set_thermal_dose(A, Ea)
        assert e.value.status == tled.E_ARG
    s.set_thermal_dose(7.39e39, 2.577e5)
    s.finalize()
    f = tled.from_problem(W.cube_t4(), dt=1e-5, device=-1, finalize=False, shared_update=1)
    f.set_thermal_dose(0.0, 0.0)
    f.finalize()
    assert f.info()["shared_update"] == 2          # the dose kernel needs every node after each step
    with pytest.raises(tled.TledError) as e:
        s.set_thermal_dose(0.0, 0.0)
    assert e.value.status == tled.E_STATE
    with pytest.raises(tled.TledError) as e:
        s.read_thermal_dose()
    assert e.value.status == tled.E_STATE          # host-only handle: no device state
    b = tled.Batch(-1)
    with pytest.raises(tled.TledError) as e:
        b.set_thermal_dose(0.0, 0.0)
    assert e.value.status == tled.E_UNSUPPORTED
