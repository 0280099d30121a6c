"""The allocation-free GEMM entry point (tled_mlp_gemm_static, split-K partials in the
library's static device array) against tled_mlp_gemm (partials in a buffer the handle
allocates), through the C-ABI: the same bits, on two calls in a row, the second with a
smaller product, and with shapes that do and do not split K."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bits(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r


@pytest.mark.parametrize("shapes", [[(64, 64, 4096), (48, 40, 1000)],       # split-K, then a smaller one
                                    [(200, 256, 2048), (100, 128, 512)],
                                    [(1024, 512, 256), (300, 70, 96)]])      # no split, then a smaller one
def test_static_scratch_gemm_matches_allocating_gemm(shapes):
    import torch
    from paper_2009_10400_amd import surrogate
    dev = torch.device("cuda:0")
    mlp = surrogate.MLP(0, n_param=1, n_freq=4, width=64, depth=1, n_out=4)
    for call, (m, n, k) in enumerate(shapes):
        print(f"[no-alloc] call {call}: m={m} n={n} k={k}", flush=True)
        rng = np.random.default_rng(1000 * call + m + n + k)
        A = torch.from_numpy(_bits(rng.standard_normal((m, k))).view(np.int16)).to(dev)
        B = torch.from_numpy(_bits(rng.standard_normal((k, n))).view(np.int16)).to(dev)
        ref = torch.full((m, n), float("nan"), dtype=torch.float32, device=dev)
        got = torch.full((m, n), float("nan"), dtype=torch.float32, device=dev)
        mlp.gemm(A, B, ref)
        mlp.gemm_static(A, B, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(r).all()
        assert np.array_equal(r.view(np.uint32), g.view(np.uint32)), f"call {call}: results differ"
