"""Training data made in separate runs (host logic, CPU): a shard written from snapshot fields
reads back as exactly the samples the same fields would give directly, at the stored nodes."""
import numpy as np

from paper_2009_10400_amd import surrogate as S, workloads as W


def _fake_snaps(sc, rng):
    snaps = []
    for s, (p, dur) in enumerate(sc):
        for j, frac in enumerate((0.5, 1.0)):
            T = p.params["T0"] + rng.uniform(0, 40, p.nn)
            u = rng.normal(0, 1e-5, (p.nn, 3))
            snaps.append((s, frac * dur, u, T))
    return snaps


def test_shard_roundtrip(tmp_path):
    sc = W.planning_scenarios(5, seed=31, lo=1500, hi=4000, duration_scale=1.0)
    rng = np.random.default_rng(0)
    t_ref = 300.0
    first = 2                                    # the shard holds scenarios 2..4 of the list
    snaps = _fake_snaps(sc[first:], rng)
    path = str(tmp_path / "shard_00_of_01.npz")
    S.write_shard(path, sc, first, snaps, per_field=300, seed=5)
    data = S.dataset_from_shards([path], sc, t_ref)
    assert data.field.max() + 1 == len(snaps)
    off = 0
    for f, (s, dur, u, T) in enumerate(snaps):
        p = sc[first + s][0]
        ordinal = sum(1 for (s2, _, _, _) in snaps[:f] if s2 == s)
        idx = S._shard_nodes(p.nn, first + s, ordinal, 300, 5)
        n = len(idx)
        assert n == min(p.nn, 300) and len(np.unique(idx)) == n
        x, pp = S.scenario_inputs(p, dur, t_ref)
        y = S.scaled_targets(p, dur, u[idx], T[idx])
        assert np.array_equal(data.x[off:off + n], x[idx]) and np.array_equal(data.p[off:off + n], pp[idx])
        assert np.array_equal(data.y[off:off + n, 0], y[:, 0].astype(np.float32))
        # displacement targets are stored in float16
        assert np.allclose(data.y[off:off + n, 1:], y[:, 1:], rtol=1e-3, atol=1e-4)
        assert np.all(data.field[off:off + n] == f)
        off += n
    assert off == len(data.x)


def test_shard_against_other_scenario_list_is_refused(tmp_path):
    sc = W.planning_scenarios(3, seed=31, lo=1500, hi=4000, duration_scale=1.0)
    other = W.planning_scenarios(3, seed=32, lo=20000, hi=40000, duration_scale=1.0)
    path = str(tmp_path / "shard_00_of_01.npz")
    S.write_shard(path, sc, 0, _fake_snaps(sc, np.random.default_rng(1)), per_field=4096, seed=5)
    try:
        S.dataset_from_shards([path], other, 300.0)
    except ValueError:
        return
    raise AssertionError("a shard read against a different scenario list was accepted")
