"""The gradient entry point that allocates nothing
(ilves_mlp_grad_f32_static, partial sums in the library's fixed device
array) against the workspace entry point (ilves_mlp_grad_f32) through the C
ABI: two calls in a row, the first at the maximum sample count, the second
smaller (the array keeps the first call's partials, which the second must
not read), each compared with the workspace call on the same inputs; a
request above the maximum is refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_2503_13075_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _inputs(torch, n, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, L.mlp_param_count()).astype(np.float32)
    x = rng.normal(0, 1.0, (n, 16)).astype(np.float32)
    y = rng.normal(0, 0.5, n).astype(np.float32)
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(p).to(dev), torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))


def test_static_gradient_matches_workspace_gradient(torch):
    lib = L.lib()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    n_max = L.MLP_GRAD_STATIC_MAX_SAMPLES
    for call, (n, seed) in enumerate(((n_max, 1), (1000, 2))):
        print(f"== static gradient call {call}: n = {n}, seed {seed}", flush=True)
        p, x, y = _inputs(torch, n, seed)
        g_ref = torch.zeros(L.mlp_param_count(), dtype=torch.float32, device=p.device)
        l_ref = torch.zeros(1, dtype=torch.float32, device=p.device)
        work = torch.zeros(L.mlp_grad_workspace(n), dtype=torch.float32, device=p.device)
        L.check(lib.ilves_mlp_grad_f32(p.data_ptr(), x.data_ptr(), y.data_ptr(), n, g_ref.data_ptr(),
                                       l_ref.data_ptr(), work.data_ptr(), work.numel(), sp))
        g = torch.full_like(g_ref, float("nan"))
        loss = torch.full_like(l_ref, float("nan"))
        L.check(lib.ilves_mlp_grad_f32_static(p.data_ptr(), x.data_ptr(), y.data_ptr(), n, g.data_ptr(),
                                              loss.data_ptr(), sp))
        torch.cuda.synchronize()
        gn, gr = g.cpu().numpy(), g_ref.cpu().numpy()
        print(f"   loss {float(loss.item()):.6e} vs {float(l_ref.item()):.6e}, "
              f"max |dgrad| {np.max(np.abs(gn - gr)):.1e}", flush=True)
        # same kernels, same partial sums, same fixed summation order: identical bits
        assert np.array_equal(gn, gr) and float(loss.item()) == float(l_ref.item())
        assert np.all(np.isfinite(gn))
    p, x, y = _inputs(torch, 4, 3)
    g = torch.zeros(L.mlp_param_count(), dtype=torch.float32, device=p.device)
    loss = torch.zeros(1, dtype=torch.float32, device=p.device)
    code = lib.ilves_mlp_grad_f32_static(p.data_ptr(), x.data_ptr(), y.data_ptr(), n_max + 1, g.data_ptr(),
                                         loss.data_ptr(), sp)
    assert code == L.ERR_ARG and b"exceeds" in lib.ilves_last_error()
