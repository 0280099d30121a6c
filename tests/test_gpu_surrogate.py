"""GPU tests of the surrogate network: MFMA GEMM, forward, gradient, training.

The GEMM is checked against an FP64 product of the same bfloat16 inputs; the
network's forward pass and gradient against the FP64 reference of
oracle/mlp_ref.py evaluated with the same (bfloat16-rounded) weights.
"""
import numpy as np
import pytest

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


def _bf16_bits(a):
    """float32 -> bfloat16 bits, round to nearest even (finite inputs)."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_round(a):
    return (_bf16_bits(a).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda", 0)


def _mlp(**kw):
    from paper_2009_10400_amd import surrogate
    return surrogate.MLP(0, **kw)


@pytest.mark.parametrize("m,n,k", [(64, 64, 32), (100, 70, 45), (1, 1, 1), (5, 256, 8192), (8192, 256, 256),
                                   (257, 129, 300), (4, 200, 4096), (100, 72, 48),
                                   (130, 136, 1000)])
def test_gemm_matches_fp64_product(torch_dev, m, n, k):
    import torch
    print(f"[gemm] m={m} n={n} k={k}", flush=True)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((m, k)).astype(np.float32)
    B = rng.standard_normal((k, n)).astype(np.float32)
    Ab, Bb = _bf16_bits(A), _bf16_bits(B)
    ref = _bf16_round(A) @ _bf16_round(B)
    mlp = _mlp(n_param=1, n_freq=4, width=64, depth=1, n_out=4)
    dA = torch.from_numpy(Ab.view(np.int16)).to(torch_dev)
    dB = torch.from_numpy(Bb.view(np.int16)).to(torch_dev)
    C = torch.full((m, n), float("nan"), dtype=torch.float32, device=torch_dev)
    mlp.gemm(dA, dB, C)
    got = C.cpu().numpy().astype(np.float64)
    # products of bfloat16 values are exact in FP32; only the FP32 summation rounds
    tol = 4e-7 * np.sqrt(k) * (np.abs(_bf16_round(A)) @ np.abs(_bf16_round(B))) + 1e-30
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


def _small_case(seed, n=300, cfg=None):
    cfg = cfg or dict(n_param=3, n_freq=16, width=64, depth=2, n_out=4)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    p = rng.uniform(-1, 1, (n, cfg["n_param"])).astype(np.float32)
    t = rng.standard_normal((n, cfg["n_out"])).astype(np.float32)
    return cfg, x, p, t


def _ref_theta(mlp):
    """FP64 reference parameters: weights rounded to bfloat16 as the kernels use them, FP32 biases."""
    theta = mlp.params().astype(np.float64)
    lay, _, _ = R.layout(**mlp.cfg)
    for ws, _, _ in lay:
        theta[ws] = _bf16_round(theta[ws].astype(np.float32))
    return theta


@pytest.mark.parametrize("n,layerwise", [(1, False), (300, False), (1000, False), (1000, True)])
def test_forward_matches_reference(torch_dev, n, layerwise):
    import torch
    print(f"[forward] n={n} layerwise={layerwise}", flush=True)
    cfg, x, p, t = _small_case(11, n)
    mlp = _mlp(**cfg, sigma=0.7, seed=3, layerwise=layerwise)
    B = mlp.frequencies().astype(np.float64)
    y = mlp.forward(torch.from_numpy(x).to(torch_dev), torch.from_numpy(p).to(torch_dev)).cpu().numpy()
    yr, _, _ = R.forward(_ref_theta(mlp), x.astype(np.float64), p.astype(np.float64), B, cfg)
    scale = np.abs(yr).max()
    assert np.abs(y - yr).max() <= 2e-2 * scale, (np.abs(y - yr).max(), scale)


# n = 40000 and 70001: 625 and 1094 workgroups, four wavefronts each (eight below two per CU)
@pytest.mark.parametrize("width,depth,n_out,n", [(64, 2, 4, 1000), (256, 5, 4, 4097), (128, 3, 20, 77),
                                                  (256, 1, 1, 1), (256, 5, 4, 40000), (128, 2, 4, 70001)])
def test_fused_inference_equals_layerwise(torch_dev, width, depth, n_out, n):
    """The fused whole-network kernel and the layer-by-layer GEMMs give the same bits."""
    import torch
    print(f"[fused] width={width} depth={depth} n_out={n_out} n={n}", flush=True)
    cfg = dict(n_param=11, n_freq=64, width=width, depth=depth, n_out=n_out)
    rng = np.random.default_rng(width + n)
    x = torch.from_numpy(rng.uniform(-2, 2, (n, 3)).astype(np.float32)).to(torch_dev)
    p = torch.from_numpy(rng.uniform(-1, 1, (n, 11)).astype(np.float32)).to(torch_dev)
    a = _mlp(**cfg, seed=4)
    b = _mlp(**cfg, seed=4, layerwise=True)
    ya, yb = a.forward(x, p).cpu().numpy(), b.forward(x, p).cpu().numpy()
    assert np.isfinite(ya).all()
    assert np.array_equal(ya, yb)


def test_frequencies_are_gaussian():
    """The Fourier frequencies are N(0, sigma^2): moments of 3 x 4096 draws."""
    mlp = _mlp(n_param=0, n_freq=4096, width=64, depth=1, n_out=1, sigma=2.0, seed=9)
    B = mlp.frequencies()
    assert abs(B.mean()) < 0.06 and abs(B.std() - 2.0) < 0.05


# n = 700: split-K weight gradients with the bias sums in their partials and a ragged
# last chunk; n = 100: one k chunk (the bias sums written directly); n_out = 12: the
# output layer through the GEMMs and column-sum kernels instead of its own kernels; width 320:
# the output-layer kernel's two column blocks and partial GEMM tiles (layer by layer)
@pytest.mark.parametrize("depth,width,n_out,n", [(2, 64, 4, 700), (5, 256, 4, 700), (3, 128, 12, 700),
                                                 (2, 64, 4, 100), (2, 320, 4, 300)])
def test_gradient_matches_fp64_reference(torch_dev, depth, width, n_out, n):
    import torch
    print(f"[gradient] depth={depth} width={width} n_out={n_out} n={n}", flush=True)
    cfg, x, p, t = _small_case(21, n, dict(n_param=8, n_freq=64, width=width, depth=depth, n_out=n_out))
    mlp = _mlp(**cfg, sigma=1.0, seed=5)
    B = mlp.frequencies().astype(np.float64)
    dx, dp, dt = (torch.from_numpy(a).to(torch_dev) for a in (x, p, t))
    loss, g = mlp.gradient(dx, dp, dt)
    lr, gr = R.loss_and_grad(_ref_theta(mlp), x.astype(np.float64), p.astype(np.float64), t.astype(np.float64),
                             B, cfg)
    assert abs(loss - lr) <= 1e-2 * lr
    mag = R.grad_magnitude(_ref_theta(mlp), x.astype(np.float64), p.astype(np.float64), t.astype(np.float64),
                           B, cfg)
    lay, _, _ = R.layout(**cfg)
    for l, (ws, _, bs) in enumerate(lay):
        for sl in (ws, bs):
            a, b, m = g[sl].astype(np.float64), gr[sl], mag[sl]
            err = np.abs(a - b)
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            elem = err.max() / np.abs(b).max()              # every element, against the layer's largest
            term = (err / np.maximum(m, 1e-300)).max()      # every element, against its terms' magnitude
            print(f"  layer {l} {'W' if sl is ws else 'b'}: norm rel {rel:.2e}, max elem err / max |g| "
                  f"{elem:.2e}, max elem err / sum|terms| {term:.2e}", flush=True)
            # element-wise: every gradient entry within 0.5 % of the layer's largest entry, and
            # within 3 % of the sum of the magnitudes of the terms that make it (bfloat16
            # activations and weights round at 2^-9 relative, a few times through the layers)
            assert elem <= 5e-3, (l, elem)
            assert term <= 3e-2, (l, term)


def test_training_reduces_loss_and_is_deterministic(torch_dev):
    import torch
    rng = np.random.default_rng(7)
    n = 4096
    x = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    p = rng.uniform(-1, 1, (n, 2)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * p[:, 0], np.exp(-(x ** 2).sum(1)), x[:, 1] * x[:, 2], p[:, 1] ** 2],
                 axis=1).astype(np.float32)
    dx, dp, dt = (torch.from_numpy(a).to(torch_dev) for a in (x, p, t))
    cfg = dict(n_param=2, n_freq=32, width=128, depth=3, n_out=4)
    a, b = _mlp(**cfg, seed=1, sigma=0.5), _mlp(**cfg, seed=1, sigma=0.5)
    l0 = a.train_step(dx, dp, dt, 2e-3, want_loss=True)
    for _ in range(300):
        a.train_step(dx, dp, dt, 2e-3)
    l1 = a.train_step(dx, dp, dt, 1e-3, want_loss=True)
    print(f"[train] loss {l0:.4g} -> {l1:.4g}", flush=True)
    assert l1 < 0.05 * l0
    b.train_step(dx, dp, dt, 2e-3)
    for _ in range(300):
        b.train_step(dx, dp, dt, 2e-3)
    b.train_step(dx, dp, dt, 1e-3)
    assert np.array_equal(a.params(), b.params())


@pytest.mark.parametrize("width,depth,n", [(64, 2, 1000), (256, 5, 4097), (128, 3, 77), (256, 2, 40000)])
def test_fused_training_forward_equals_layerwise(torch_dev, width, depth, n):
    """Training steps whose forward pass is the fused kernel (storing the features, every
    pre-activation and activation for the backward pass) leave the same parameters, bit for bit,
    as steps through the layer-by-layer GEMMs."""
    import torch
    print(f"[fused train] width={width} depth={depth} n={n}", flush=True)
    rng = np.random.default_rng(width + depth)
    x = torch.from_numpy(rng.uniform(-1, 1, (n, 3)).astype(np.float32)).to(torch_dev)
    p = torch.from_numpy(rng.uniform(-1, 1, (n, 5)).astype(np.float32)).to(torch_dev)
    t = torch.from_numpy(rng.normal(size=(n, 4)).astype(np.float32)).to(torch_dev)
    cfg = dict(n_param=5, n_freq=32, width=width, depth=depth, n_out=4)
    a, b = _mlp(**cfg, seed=2, sigma=0.5), _mlp(**cfg, seed=2, sigma=0.5, layerwise=True)
    for k in range(12):
        la = a.train_step(x, p, t, 2e-3, want_loss=k == 11)
        lb = b.train_step(x, p, t, 2e-3, want_loss=k == 11)
    assert la == lb
    assert np.array_equal(a.params(), b.params())


def test_argument_errors(torch_dev):
    import torch
    from paper_2009_10400_amd import surrogate
    from paper_2009_10400_amd.tled import TledError
    with pytest.raises(TledError):
        surrogate.MLP(0, width=100)
    with pytest.raises(TledError):
        surrogate.MLP(0, n_out=65)
    m = _mlp(n_param=2, n_freq=4, width=64, depth=1, n_out=2)
    x = torch.zeros((0, 3), device=torch_dev)
    assert m.forward(x, torch.zeros((0, 2), device=torch_dev)).shape == (0, 2)
    with pytest.raises(TledError):
        m.train_step(torch.zeros((4, 3), device=torch_dev), torch.zeros((4, 2), device=torch_dev),
                     torch.zeros((4, 2), device=torch_dev), -1.0)
    # tensors the kernels would misread are refused by the binding
    with pytest.raises(ValueError):
        m.forward(torch.zeros((4, 3), dtype=torch.float64, device=torch_dev), torch.zeros((4, 2), device=torch_dev))
    with pytest.raises(ValueError):
        m.forward(torch.zeros((3, 4), device=torch_dev).t(), torch.zeros((4, 2), device=torch_dev))
    with pytest.raises(ValueError):
        m.forward(torch.zeros((4, 3), device=torch_dev), torch.zeros((5, 2), device=torch_dev))
    with pytest.raises(ValueError):
        m.train_step(torch.zeros((4, 3), device=torch_dev), torch.zeros((4, 2), device=torch_dev),
                     torch.zeros((4, 3), device=torch_dev), 1e-3)
    with pytest.raises(ValueError):
        m.forward(torch.zeros((4, 3)), torch.zeros((4, 2)))


def test_ensemble_statistics_kernel(torch_dev):
    """Mean over members (scaled) and the member spread of output 0, against numpy."""
    import ctypes
    import torch
    from paper_2009_10400_amd import surrogate as S
    rng = np.random.default_rng(31)
    K, n, no = 4, 1003, 4
    outs = rng.standard_normal((K, n, no)).astype(np.float32)
    scale = np.array([2.5, 0.5, 1.0, 3.0], np.float32)
    d_outs = torch.from_numpy(outs).to(torch_dev)
    d_scale = torch.from_numpy(scale).to(torch_dev)
    mean = torch.empty((n, no), dtype=torch.float32, device=torch_dev)
    spread = torch.empty(n, dtype=torch.float32, device=torch_dev)
    st = S._lib.tled_mlp_ensemble_stats(n, K, no, S._dp(d_outs), S._dp(d_scale), S._dp(mean), S._dp(spread),
                                        ctypes.c_void_p(torch.cuda.current_stream(torch_dev).cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    np.testing.assert_allclose(mean.cpu().numpy(), scale * outs.astype(np.float64).mean(0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(spread.cpu().numpy(), scale[0] * (outs[..., 0].max(0) - outs[..., 0].min(0)),
                               rtol=1e-6)
    assert S._lib.tled_mlp_ensemble_stats(n, 0, no, S._dp(d_outs), S._dp(d_scale), S._dp(mean), S._dp(spread),
                                          None) != 0


def test_scenario_inputs_and_outputs_match_the_host_path(torch_dev):
    """predict_many assembles the inputs and unscales the outputs on the device; both are bitwise
    those of the host functions (fill_inputs, unscale), on scenarios of different sizes."""
    import torch
    from paper_2009_10400_amd import surrogate as S, workloads as W
    items = W.planning_scenarios(5, seed=41, lo=1500, hi=9000, duration_scale=1e-3)
    ens = S.Ensemble(2, t_ref=0.3)
    ens.y_std = np.array([0.7, 1.3, 0.9, 1.1], np.float32)
    got = ens.predict_many(items)
    for (p, d), (T, u, sp) in zip(items, got):
        x, prm = S.scenario_inputs(p, d, ens.t_ref)
        mean, spread = ens._forward_device(torch.from_numpy(x).to(torch_dev), torch.from_numpy(prm).to(torch_dev))
        mean, spread = mean.cpu().numpy(), spread.cpu().numpy()
        Tr, ur = S.unscale(p, d, mean)
        spr = S.temperature_scale(p, d) * spread
        assert T.dtype == Tr.dtype == np.float32 and T.shape == (p.nn,) and u.shape == (p.nn, 3)
        assert np.array_equal(T, Tr) and np.array_equal(u, ur) and np.array_equal(sp, spr)
    # the input kernel alone against fill_inputs, and its argument checks
    p, d = items[0]
    x, prm = S.scenario_inputs(p, d, ens.t_ref)
    probe, pm = S._scenario_params(p, d, ens.t_ref)
    offs = torch.tensor([0, p.nn], dtype=torch.int64, device=torch_dev)
    Xd = torch.from_numpy(np.asarray(p.X, np.float64)).to(torch_dev)
    pr = torch.from_numpy(probe.reshape(1, 3)).to(torch_dev)
    xi = torch.tensor([1.0 / (S.XI_SCALE * p.h)], dtype=torch.float64, device=torch_dev)
    pmd = torch.from_numpy(pm.astype(np.float32).reshape(1, -1)).to(torch_dev)
    xo = torch.empty((p.nn, 3), dtype=torch.float32, device=torch_dev)
    po = torch.empty((p.nn, S.N_PARAM), dtype=torch.float32, device=torch_dev)
    assert S._lib.tled_mlp_scenario_inputs(1, S.N_PARAM - 3, p.nn, S._dp(offs), S._dp(Xd), S._dp(pr), S._dp(xi),
                                           1.0 / 0.05, S._dp(pmd), S._dp(xo), S._dp(po), None) == 0
    torch.cuda.synchronize()
    assert np.array_equal(xo.cpu().numpy(), x) and np.array_equal(po.cpu().numpy(), prm)
    assert S._lib.tled_mlp_scenario_inputs(0, S.N_PARAM - 3, p.nn, S._dp(offs), S._dp(Xd), S._dp(pr), S._dp(xi),
                                           1.0 / 0.05, S._dp(pmd), S._dp(xo), S._dp(po), None) != 0
    assert S._lib.tled_mlp_scenario_outputs(1, p.nn, None, S._dp(xo), S._dp(xo), S._dp(pmd), S._dp(pmd),
                                            S._dp(pmd), S._dp(xo), S._dp(xo), S._dp(xo), None) != 0
