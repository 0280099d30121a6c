"""Pins of the FP64 reference of the surrogate network (oracle/mlp_ref.py).

The reference is pinned to closed forms and to central finite differences, so
that the GPU gradient checks compare against something checked by other means.
"""
import numpy as np

from oracle import mlp_ref as R

CFG = dict(n_param=3, n_freq=5, width=8, depth=2, n_out=2)


def _net(seed=0, cfg=CFG):
    rng = np.random.default_rng(seed)
    _, K0, P = R.layout(**cfg)
    theta = rng.standard_normal(P) * 0.5
    B = rng.standard_normal((cfg["n_freq"], 3))
    return theta, B, K0


def test_parameter_count_closed_form():
    for cfg in (CFG, dict(n_param=11, n_freq=64, width=256, depth=5, n_out=4)):
        lay, K0, P = R.layout(**cfg)
        W, D, no = cfg["width"], cfg["depth"], cfg["n_out"]
        assert K0 % 32 == 0 and K0 >= 2 * cfg["n_freq"] + cfg["n_param"] and K0 - 32 < 2 * cfg["n_freq"] + cfg["n_param"]
        assert P == W * K0 + W + (D - 1) * (W * W + W) + no * W + no
        assert len(lay) == D + 1
    # the network of the planning surrogate: 64 frequencies, 11 parameters -> 139 inputs padded to 160
    assert R.layout(n_param=11, n_freq=64, width=256, depth=5, n_out=4)[1] == 160


def test_features_unit_circle_and_padding():
    rng = np.random.default_rng(1)
    x, p = rng.standard_normal((20, 3)), rng.standard_normal((20, 3))
    B = rng.standard_normal((5, 3))
    f = R.features(x, p, B, 32)
    assert f.shape == (20, 32)
    np.testing.assert_allclose(f[:, :5] ** 2 + f[:, 5:10] ** 2, 1.0, atol=1e-14)
    np.testing.assert_array_equal(f[:, 10:13], p)
    assert not f[:, 13:].any()
    # x = 0: sin 0 = 0, cos 0 = 1
    f0 = R.features(np.zeros((1, 3)), p[:1], B, 32)
    np.testing.assert_array_equal(f0[0, :5], 0.0)
    np.testing.assert_array_equal(f0[0, 5:10], 1.0)


def test_silu_special_values():
    assert R.silu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(R.silu(np.array([40.0])), 40.0, rtol=1e-15)
    np.testing.assert_allclose(R.silu(np.array([-40.0])), 0.0, atol=1e-15)
    np.testing.assert_allclose(R.silu(np.array([1.0])), 1.0 / (1.0 + np.exp(-1.0)), rtol=1e-15)


def test_forward_hand_built_network():
    """A one-hidden-layer network whose weights pick one input: output = silu(p0) by hand."""
    cfg = dict(n_param=1, n_freq=1, width=4, depth=1, n_out=1)
    lay, K0, P = R.layout(**cfg)
    theta = np.zeros(P)
    (w0, s0, b0), (w1, s1, b1) = lay
    W0 = np.zeros(s0)
    W0[0, 2] = 1.0                     # input 2 = the parameter (after sin, cos)
    theta[w0] = W0.ravel()
    W1 = np.zeros(s1)
    W1[0, 0] = 2.0
    theta[w1] = W1.ravel()
    theta[b1] = 0.25
    p = np.array([[-1.0], [0.0], [3.0]])
    y, _, _ = R.forward(theta, np.zeros((3, 3)), p, np.ones((1, 3)), cfg)
    expect = 2.0 * p[:, 0] / (1.0 + np.exp(-p[:, 0])) + 0.25
    np.testing.assert_allclose(y[:, 0], expect, rtol=1e-15)


def test_zero_loss_at_exact_fit():
    theta, B, _ = _net(2)
    rng = np.random.default_rng(3)
    x, p = rng.standard_normal((7, 3)), rng.standard_normal((7, 3))
    y, _, _ = R.forward(theta, x, p, B, CFG)
    loss, g = R.loss_and_grad(theta, x, p, y, B, CFG)
    assert loss == 0.0 and not g.any()


def test_gradient_matches_central_differences():
    theta, B, _ = _net(4)
    rng = np.random.default_rng(5)
    x, p = rng.standard_normal((11, 3)), rng.standard_normal((11, 3))
    tgt = rng.standard_normal((11, 2))
    loss, g = R.loss_and_grad(theta, x, p, tgt, B, CFG)
    lay, K0, P = R.layout(**CFG)
    # padded first-layer inputs are zero: their weights have zero gradient
    ws, wsh, _ = lay[0]
    g0 = g[ws].reshape(wsh)
    assert not g0[:, 2 * CFG["n_freq"] + CFG["n_param"]:].any()
    h = 1e-6
    idx = rng.choice(P, 60, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (R.loss_and_grad(tp, x, p, tgt, B, CFG)[0] - R.loss_and_grad(tm, x, p, tgt, B, CFG)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])
