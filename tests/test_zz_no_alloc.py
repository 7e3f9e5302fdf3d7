"""The allocation-free backward pass (grprec_mlp_backward_noalloc, for callers
that cannot allocate device memory) against grprec_mlp_backward with caller
workspace, called through the C ABI: two calls in a row, the second with a
smaller batch, each equal bit for bit to the workspace form; sizes beyond the
fixed scratch array are rejected."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21911_amd import grprec
    grprec.lib()
    return grprec


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(scale=0.3, size=1325)
    P[1313:1319] = rng.normal(scale=0.1, size=6)
    P[1319:1325] = rng.uniform(0.5, 2.0, size=6)
    x = rng.normal(size=(n, 6))
    dy = rng.normal(size=n)
    return [torch.from_numpy(a.astype(np.float32)).cuda() for a in (P, x, dy)]


def test_noalloc_equals_workspace_form_on_two_calls(G):
    L = G.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, seed in ((G.GRPREC_MLP_NOALLOC_MAX, 1), (1000, 2)):
        print(f"noalloc backward n={n}", flush=True)
        P, x, dy = _inputs(n, seed)
        g_ref = torch.full((G.GRPREC_MLP_WEIGHTS,), float("nan"), dtype=torch.float32, device="cuda")
        work = torch.zeros(G.grprec_mlp_work_bytes(n), dtype=torch.uint8, device="cuda")
        assert L.grprec_mlp_backward(P.data_ptr(), x.data_ptr(), dy.data_ptr(), g_ref.data_ptr(), n,
                                     work.data_ptr(), stream) == 0
        g = torch.full_like(g_ref, float("nan"))
        assert L.grprec_mlp_backward_noalloc(P.data_ptr(), x.data_ptr(), dy.data_ptr(), g.data_ptr(), n,
                                             stream) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(g).all()
        assert torch.equal(g, g_ref), (g - g_ref).abs().max().item()


def test_noalloc_rejects_sizes_beyond_its_array(G):
    L = G.lib()
    P, x, dy = _inputs(4, 3)
    g = torch.zeros(G.GRPREC_MLP_WEIGHTS, dtype=torch.float32, device="cuda")
    for n in (0, -5, G.GRPREC_MLP_NOALLOC_MAX + 1):
        assert L.grprec_mlp_backward_noalloc(P.data_ptr(), x.data_ptr(), dy.data_ptr(), g.data_ptr(), n,
                                             None) == G.GRPREC_E_INVALID
