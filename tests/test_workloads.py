"""Seeded input generators: meshes conform, volumes are positive and add up, sources carry
their stated power, presets reproduce the paper's printed material values (tests/golden)."""
import os

import numpy as np
import pytest

import oracle
from paper_2009_10400_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_material_tables.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out


def tet_volumes(X, conn):
    d = X[conn[:, 1:]] - X[conn[:, :1]]
    return np.linalg.det(d.transpose(0, 2, 1)) / 6.0


def faces_shared_ok(conn, X, L=None):
    faces = np.concatenate([np.sort(conn[:, f], axis=1) for f in ([0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3])])
    uniq, cnt = np.unique(faces, axis=0, return_counts=True)
    assert cnt.max() == 2
    return uniq[cnt == 1]


def test_paper_presets_match_tables():
    g = golden()
    mu, kappa = W.youngs_to_lame(g["table1.E"], g["table1.nu"])
    assert mu == pytest.approx(g["table1.mu"], abs=1e-3)
    assert kappa == pytest.approx(g["table1.kappa"], abs=1e-3)
    t1 = W.paper_table1_material()
    assert (t1["rho"], t1["c"], t1["k"]) == (g["table1.rho"], g["table1.c"], g["table1.k"])
    t5 = W.paper_table5_material()
    assert t5["eta"] == pytest.approx(g["table5.eta_over_mu"] * g["table5.mu"])
    assert (t5["c"], t5["c_hi"], t5["k"], t5["k_hi"]) == (g["table5.c_lo"], g["table5.c_hi"],
                                                          g["table5.k_lo"], g["table5.k_hi"])
    assert t5["wbcb"] == pytest.approx(g["table5.wb"] * g["table5.cb"])
    assert t5["Q_met"] == g["table5.Qm"]
    assert g["table5.rho"] * g["table5.SAR"] == pytest.approx(g["table5.Qr"], rel=1e-12)
    assert t5["ckT_hi"] - t5["ckT_lo"] == pytest.approx(90 - 37)
    assert g["table1.dt"] * g["table1.steps"] == pytest.approx(5.0)
    assert g["table5.dt"] * g["table5.steps"] == pytest.approx(25.0)


def test_cube_t4_conforming():
    p = W.cube_t4()
    assert (p.ne, p.nn) == (6000, 1331)
    V = tet_volumes(p.X, p.conn)
    assert V.min() > 0 and V.sum() == pytest.approx(0.04 ** 3, rel=1e-12)
    bnd = faces_shared_ok(p.conn, p.X)
    c = p.X[bnd].mean(1)
    on = np.isclose(c, 0.0) | np.isclose(c, 0.04)
    assert np.all(on.any(1))                      # unshared faces lie on the box surface
    assert len(bnd) == 6 * 2 * 100
    assert np.all(p.fix[np.isclose(p.X[:, 2], 0)] == 7) and p.fix.sum() == 7 * 121
    total = (p.q * V).sum()
    assert total == pytest.approx(5e7 * (2 * np.pi) ** 1.5 * 0.004 ** 3, rel=0.02)   # ~50.4 W


def test_cube_h8_orientation_and_fibres():
    p = W.cube_h8(n=6)
    s = oracle.OracleSim(8, p.X, p.conn, p.params, dt=1e-4)
    _, _, V0 = s.geometry()
    assert np.allclose(V0, (0.1 / 6) ** 3, rtol=1e-12)
    assert np.allclose(np.linalg.norm(p.a0, axis=1), 1.0)
    assert (p.q * V0).sum() == pytest.approx(10.0, rel=1e-12)
    assert p.t_off == 60.0


@pytest.mark.parametrize("target", [3000, 40000])
def test_ellipsoid_mesh_valid(target):
    p = W.ellipsoid_t4(target)
    V = tet_volumes(p.X, p.conn)
    assert V.min() > 0.05 * p.h ** 3 / 6
    assert abs(p.ne - target) < 0.1 * target
    bnd = faces_shared_ok(p.conn, p.X)
    assert (p.q * V).sum() == pytest.approx(10.0, rel=1e-9)
    assert np.allclose(np.linalg.norm(p.a0, axis=1), 1.0)
    assert p.fix.any() and not p.fix.all()
    # the order is randomised: consecutive elements are not neighbours
    d = np.linalg.norm(np.diff(p.X[p.conn[:, 0]], axis=0), axis=1)
    assert np.median(d) > 5 * p.h
