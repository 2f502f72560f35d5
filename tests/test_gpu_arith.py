"""GPU test of the FP64 division and square root the sweeps use (through the C ABI,
hx_arith_check): for operands with exponents in [-300, 300] (quotients) and [-700, 700] (roots),
mixed signs, equal operands and tiny/huge ratios, every quotient equals the CPU's IEEE
round-to-nearest a / b and every root equals the CPU's sqrt, bit for bit; zero numerators give
zeros (of either sign: the value is what the method uses)."""
import numpy as np
import pytest

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


def _operands(rng, n, emax):
    m = 1.0 + rng.random(n)
    e = rng.integers(-emax, emax + 1, n)
    s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return s * np.ldexp(m, e)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_division_and_root_are_ieee(env, seed):
    H, torch = env
    announce(f"arith check seed {seed}")
    rng = np.random.default_rng(seed)
    n = 1 << 20
    a = _operands(rng, n, 300)
    b = _operands(rng, n, 300)
    b[::97] = a[::97]                                   # exact quotients 1
    a[5::101] = b[5::101] * 3.0                         # exact quotients 3
    b[7::89] = np.ldexp(1.0, rng.integers(-40, 40, b[7::89].size))   # powers of two
    a[11::113] = 0.0                                    # zero numerators
    r = _operands(rng, n, 700)
    dev = lambda v: torch.tensor(v, dtype=torch.float64, device="cuda")
    q, _ = H.arith_check(dev(a), dev(b))
    _, s = H.arith_check(dev(r), dev(np.ones(n)))
    q = q.cpu().numpy()
    s = s.cpu().numpy()
    qe = a / b
    se = np.sqrt(np.abs(r))
    assert np.array_equal(q, qe), int(np.sum(q != qe))
    nz = qe != 0
    assert np.array_equal(q[nz].view(np.int64), qe[nz].view(np.int64))
    assert np.array_equal(s.view(np.int64), se.view(np.int64)), int(np.sum(s != se))
    print(f"seed {seed}: {n} quotients and {n} roots equal to IEEE (bitwise for non-zero quotients)")


def test_arith_check_rejects_bad_arguments(env):
    H, torch = env
    import ctypes as C
    L = H.load_library()
    assert L.hx_arith_check(None, None, 4, None, None, None) == H.EINVAL
    assert L.hx_arith_check(None, None, 0, None, None, None) == H.EINVAL
