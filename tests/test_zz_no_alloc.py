"""GPU test of the allocation-free gradient entry point (hx_mlp_grad_noalloc, through the C ABI):
two calls in a row, the second on a smaller batch, each equal bit for bit to hx_mlp_grad with a
caller-provided scratch on the same inputs (both run the same deterministic kernels), and both
checked against the FP64 oracle's gradient at the FP32 bar of the gradient test."""
import numpy as np
import pytest

from oracle import oracle as O

from parity import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_04428_amd import hydro
    hydro.load_library()
    return hydro, torch


def _case(seed, n):
    rng = np.random.default_rng(seed)
    w = rng.normal(scale=0.3, size=O.MLP_NPARAM).astype(np.float32)
    x = rng.uniform(-1, 1, size=(n, 4))
    a = rng.uniform(-1, 1, size=n)
    t = rng.uniform(-1, 1, size=n)
    wt = (rng.uniform(size=n) > 0.2).astype(np.float64)
    return w, x, a, t, wt


def test_noalloc_gradient_equals_workspace_gradient(env):
    H, torch = env
    dev = lambda v: torch.tensor(v, dtype=torch.float32, device="cuda").contiguous()
    # 300 000 samples fill the capped grid (1024 blocks, grid-stride); 5 000 use 20 blocks, so
    # the second call leaves most of the first call's partial rows in the scratch untouched
    for seed, n in ((11, 300_000), (12, 5_000)):
        announce(f"noalloc grad n={n}")
        w, x, a, t, wt = _case(seed, n)
        xs, as_, ts, wts = dev(x), dev(a), dev(t), dev(wt)
        ref = H.MlpTrainer(w, n)
        g_ref, l_ref = ref.gradient(xs, as_, ts, wts)
        g_ref, l_ref = g_ref.cpu().numpy().copy(), float(l_ref.item())
        tr = H.MlpTrainer(w, 1)  # its own workspace is far too small: only the static scratch is used
        g, loss = tr.gradient_noalloc(xs, as_, ts, wts)
        torch.cuda.synchronize()
        g, loss = g.cpu().numpy(), float(loss.item())
        assert np.array_equal(g, g_ref), np.max(np.abs(g - g_ref))
        assert loss == l_ref
        if n <= 5_000:
            lo, go = O.mlp_loss_grad(w.astype(np.float64), x.astype(np.float32).astype(np.float64),
                                     a.astype(np.float32).astype(np.float64),
                                     t.astype(np.float32).astype(np.float64), wt)
            assert abs(loss - lo) < 1e-5 * abs(lo)
            scale = np.abs(go).max()
            assert np.all(np.abs(g - go) <= 1e-4 * np.abs(go) + 2e-5 * scale)


def test_noalloc_gradient_rejects_bad_arguments(env):
    H, torch = env
    import ctypes as C
    L = H.load_library()
    st = L.hx_mlp_grad_noalloc(None, None, None, None, None, C.c_longlong(0), None, None, None)
    assert st == -1
    assert b"invalid" in L.hx_last_error()
