"""GPU tests of the learned-limiter path (through the C ABI): BF16 matrix-core inference, training
samples, gradients and Adam against the FP64 oracle (and torch's Adam), the batched 1D solver, and
the learned form of the fused sweep."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_04428_amd import problems as P

from parity import announce, assert_parity, parity_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_04428_amd import hydro
    hydro.load_library()
    return hydro, torch


def _weights(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return (rng.normal(scale=scale, size=O.MLP_NPARAM)).astype(np.float32)


def _emulate_gpu_phi(w, x):
    """The device's rounding steps written out in numpy: BF16 parameters and inputs, FP32 layer-1
    sums, BF16 hidden layer 1, FP32 layer-2 sums, FP32 output layer."""
    wb = O.bf16_round(w).astype(np.float32)
    xb = O.bf16_round(x).astype(np.float32)
    W1, b1 = wb[:128].reshape(32, 4), wb[128:160]
    W2, b2 = wb[160:1184].reshape(32, 32), wb[1184:1216]
    w3, b3 = wb[1216:1248], wb[1248]
    gelu = lambda z: 0.5 * z * (1 + np.tanh(np.float32(0.7978845608028654) * (z + np.float32(0.044715) * z ** 3)))
    h1 = gelu(xb @ W1.T + b1).astype(np.float32)
    h1 = O.bf16_round(h1).astype(np.float32)
    h2 = gelu(h1 @ W2.T + b2).astype(np.float32)
    z = h2 @ w3 + b3
    return 2.0 / (1.0 + np.exp(-z.astype(np.float64)))


def test_mlp_eval_matches_emulation_and_oracle(env):
    H, torch = env
    announce("mlp eval")
    w = _weights(1)
    rng = np.random.default_rng(2)
    n = 1000  # 62.5 tiles: a ragged last tile
    x = rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    phi = H.mlp_eval(torch.tensor(w, device="cuda"), torch.tensor(x, device="cuda")).cpu().numpy()
    emu = _emulate_gpu_phi(w, x)
    assert np.max(np.abs(phi - emu)) < 2e-3, np.max(np.abs(phi - emu))
    wb = O.bf16_round(w)
    ref = np.array([O.mlp_phi(wb, x[i].astype(np.float64)) for i in range(n)])
    err = np.abs(phi - ref)
    print(f"mlp eval: max |phi - oracle| {err.max():.3e}, mean {err.mean():.3e}")
    assert err.max() < 0.05 and err.mean() < 0.01


def test_mlp_grad_matches_oracle(env):
    """GPU FP32 loss gradient vs the FP64 oracle's hand-written backward on the same weights."""
    H, torch = env
    announce("mlp grad")
    w = _weights(3, scale=0.3)
    rng = np.random.default_rng(4)
    n = 5000
    x = rng.uniform(-1, 1, size=(n, 4))
    a = rng.uniform(-1, 1, size=n)
    t = rng.uniform(-1, 1, size=n)
    wt = (rng.uniform(size=n) > 0.2).astype(np.float64)
    tr = H.MlpTrainer(w, n)
    dev = lambda v: torch.tensor(v, dtype=torch.float32, device="cuda").contiguous()
    g, loss = tr.gradient(dev(x), dev(a), dev(t), dev(wt))
    g = g.cpu().numpy().astype(np.float64)
    lo, go = O.mlp_loss_grad(w.astype(np.float64), x.astype(np.float32).astype(np.float64),
                             a.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64), wt)
    assert abs(float(loss.item()) - lo) < 1e-5 * abs(lo)
    scale = np.abs(go).max()
    assert np.all(np.abs(g - go) <= 1e-4 * np.abs(go) + 2e-5 * scale), np.max(np.abs(g - go) / scale)


def test_mlp_adam_matches_torch(env):
    H, torch = env
    announce("mlp adam")
    w = _weights(5)
    tr = H.MlpTrainer(w, 16)
    ref = torch.nn.Parameter(torch.tensor(w, dtype=torch.float32))
    opt = torch.optim.Adam([ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(6)
    for k in range(4):
        g = rng.normal(size=O.MLP_NPARAM).astype(np.float32)
        tr.grad.copy_(torch.tensor(g, device="cuda"))
        tr.adam(lr=1e-2)
        ref.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(tr.w.cpu().numpy(), ref.detach().numpy(), rtol=1e-5, atol=1e-7)


def test_mlp_features_match_oracle(env):
    H, torch = env
    announce("mlp features")
    rng = np.random.default_rng(7)
    rows, nf, R = 6, 96, 4
    xf = (np.arange(nf) + 0.5) / nf
    U = np.zeros((5, rows, nf))
    for r in range(rows):
        k = rng.uniform(1, 6, size=3)
        ph = rng.uniform(0, 6, size=3)
        rho = 1.0 + 0.5 * np.sin(k[0] * 2 * np.pi * xf + ph[0])
        u = 0.7 * np.sin(k[1] * 2 * np.pi * xf + ph[1])
        p = 1.0 + 0.4 * np.cos(k[2] * 2 * np.pi * xf + ph[2])
        U[0, r], U[1, r], U[4, r] = rho, rho * u, p / 0.4 + 0.5 * rho * u * u
        U[2, r] = rho * 0.1
    x, a, t, wt = H.mlp_features(torch.tensor(U, device="cuda"), R, 1.4)
    xo, ao, to, wto = O.mlp_features(U, R, 1.4)
    assert np.array_equal(wt.cpu().numpy(), wto.astype(np.float32))
    assert wto.sum() > 50
    assert np.allclose(x.cpu().numpy(), xo, rtol=1e-6, atol=1e-7)
    assert np.allclose(a.cpu().numpy(), ao, rtol=1e-6, atol=1e-7)
    assert np.allclose(t.cpu().numpy(), to, rtol=1e-5, atol=1e-6)


def test_batched_1d_rows_match_oracle(env):
    """A batch of 1D Riemann problems solved as independent rows equals the oracle on each row."""
    H, torch = env
    announce("batched 1D parity")
    b = P.riemann_batch(8, 200, seed=77)
    rows = [P.riemann_row(b, r) for r in range(8)]
    orc = [O.Oracle(r) for r in rows]
    Us = [r.U0.copy() for r in rows]
    s = H.Solver(b)
    s.set_state(b.U0)
    for n in range(40):
        dts = [o.compute_dt(U)[0] for o, U in zip(orc, Us)]
        dt = min(dts)
        if n in (0, 39):
            assert s.compute_dt() == pytest.approx(dt, rel=1e-14)
        Us = [o.step(U, dt)[0] for o, U in zip(orc, Us)]
        s.step(dt)
    G = s.state_numpy()
    for r in range(8):
        assert_parity(G[:, :, r:r + 1, :], Us[r], what=f"row {r}")


def _mlp_const(b3):
    w = np.zeros(O.MLP_NPARAM, dtype=np.float32)
    w[1248] = b3
    return w


def test_learned_form_special_cases(env):
    """phi = 0 weights give the first-order scheme; phi = 2 weights give the closed-form TVD rule
    of the oracle (FP32 form vs FP64 oracle)."""
    H, torch = env
    pr = P.random_periodic(n=(19, 17, 15), ndim=3, nscalar=0, seed=8, ng=3, precision="fp32")
    announce("learned form special cases")
    first = H.Solver(pr.with_(limiter="none"))
    first.set_state(pr.U0)
    zero = H.Solver(pr.with_(limiter="mlp"))
    zero.set_mlp(_mlp_const(-1000.0))
    zero.set_state(pr.U0)
    two = H.Solver(pr.with_(limiter="mlp"))
    two.set_mlp(_mlp_const(1000.0))
    two.set_state(pr.U0)
    o2 = O.Oracle(pr.with_(limiter="mlp"), mlp_weights=_mlp_const(1000.0).astype(np.float64))
    U = pr.U0.copy()
    for _ in range(5):
        dt, _ = o2.compute_dt(U)
        U, st = o2.step(U, dt)
        for s in (first, zero, two):
            s.step(dt)
    a, b, c = first.state_numpy(), zero.state_numpy(), two.state_numpy()
    assert np.allclose(a, b, rtol=1e-6, atol=1e-7)
    assert np.allclose(c, U, rtol=2e-5, atol=1e-6), np.max(np.abs(c - U))


def test_learned_form_close_to_oracle(env):
    """Random network: the BF16/FP32 fused sweep vs the FP64 oracle with BF16-rounded parameters,
    after 3 steps of a 3D random problem (tolerance of BF16 inference)."""
    H, torch = env
    announce("learned form vs oracle")
    w = _weights(9, scale=0.4)
    pr = P.random_periodic(n=(21, 18, 16), ndim=3, nscalar=1, seed=10, ng=3, precision="fp32", limiter="mlp",
                           bc=[["transmissive"] * 2, ["reflective"] * 2, ["periodic"] * 2])
    o = O.Oracle(pr, mlp_weights=O.bf16_round(w))
    s = H.Solver(pr)
    s.set_mlp(w)
    s.set_state(pr.U0)
    U = pr.U0.copy()
    for _ in range(3):
        dt, _ = o.compute_dt(U)
        U, _ = o.step(U, dt)
        s.step(dt)
    G = s.state_numpy()
    rel = np.abs(G - U).reshape(pr.nvar, -1).mean(axis=1) / np.abs(U).reshape(pr.nvar, -1).mean(axis=1)
    print("learned form L1 relative difference per field:", rel)
    assert np.all(rel < 2e-3)
    assert np.all(np.isfinite(G))


LEARNED_CASES = {
    "1d_periodic_s1": lambda: P.random_periodic(n=(157,), ndim=1, nscalar=1, seed=41, ng=3, precision="fp32",
                                                limiter="mlp"),
    "2d_mixed_s2": lambda: P.random_periodic(
        n=(37, 29), ndim=2, nscalar=2, seed=42, ng=3, precision="fp32", limiter="mlp",
        bc=[["transmissive", "reflective"], ["periodic"] * 2, ["periodic"] * 2]),
    "3d_periodic_s2": lambda: P.random_periodic(n=(19, 17, 13), ndim=3, nscalar=2, seed=43, ng=3,
                                                precision="fp32", limiter="mlp"),
    "wedge2d_point": lambda: P.random_wedge(nr=20, nth=18, ndim=2, nscalar=1, seed=44, ng=3, gravity="point",
                                            precision="fp32", limiter="mlp",
                                            bc=[["reflective", "transmissive"], ["reflective"] * 2,
                                                ["periodic"] * 2]),
    "wedge3d_monopole_s1": lambda: P.random_wedge(nr=17, nth=15, nph=13, nscalar=1, seed=45, ng=3,
                                                  gravity="point_monopole", precision="fp32", limiter="mlp",
                                                  bc=[["reflective", "transmissive"], ["reflective"] * 2,
                                                      ["periodic"] * 2]),
}


@pytest.mark.parametrize("name", list(LEARNED_CASES))
def test_learned_form_cases_close_to_oracle(env, name):
    """The learned form in every dimension, both geometries and 5 to 7 fields (each a learned-form
    instantiation of its own), with the trained network if present (else a random one): 3 steps
    with the oracle's time steps against the FP64 oracle with BF16-rounded parameters, per field in
    L1 at the tolerance of BF16 inference (phi within ~2^-8 of the oracle's), and per cell at 1e-2 of
    the value plus 1e-3 of the field's scale in all but 0.1 % of the values: the van Leer fallback
    (phi > min(2, 2r)) is a jump in phi, so where the BF16 and the FP64 networks fall on either side
    of it a slope, and the cells it feeds, differ by a part of themselves."""
    from paper_2503_04428_amd import learned
    H, torch = env
    try:
        w = learned.load_weights()
    except OSError:
        w = _weights(12, scale=0.4)
    pr = LEARNED_CASES[name]()
    announce(f"learned form {name} n={pr.n} nvar={pr.nvar}")
    o = O.Oracle(pr, mlp_weights=O.bf16_round(w))
    s = H.Solver(pr)
    s.set_mlp(w)
    s.set_state(pr.U0)
    U = pr.U0.copy()
    for _ in range(3):
        dt, st = o.compute_dt(U)
        assert st == 0
        U, st = o.step(U, dt)
        assert st == 0
        s.step(dt)
    G = s.state_numpy()
    s.check()
    s.close()
    assert np.all(np.isfinite(G))
    mean = np.abs(U).reshape(pr.nvar, -1).mean(axis=1)
    still = mean == 0.0  # momenta of inactive axes: exactly 0 on both sides
    assert np.all(G[still] == 0.0)
    rel = np.abs(G - U).reshape(pr.nvar, -1).mean(axis=1)[~still] / mean[~still]
    print(f"{name}: learned form L1 relative difference per field {rel}")
    assert np.all(rel < 2e-3)
    tol = parity_tolerance(U, 1e-2, 1e-3, flow_scale=True)
    frac = float(np.mean(np.abs(G - U) > tol))
    print(f"{name}: share of values beyond the per-cell bar {frac:.2e}")
    assert frac <= 1e-3


def test_training_reduces_loss(env):
    """Samples from fine FP64 runs of the library itself; Adam on the GPU lowers the loss."""
    H, torch = env
    from paper_2503_04428_amd import learned
    announce("training pipeline (small)")
    samples, info = learned.generate_samples(nprob=64, ncoarse=64, ratio=4, times=(0.01, 0.02), seed=123)
    assert info["samples"] > 200
    w, log = learned.train(samples, steps=300, batch=4096, lr=3e-3, log_every=50)
    first, last = log["loss_log"][0][1], log["loss_log"][-1][1]
    assert last < 0.8 * first, log["loss_log"]


def test_deployed_rounding_keeps_the_training_loss(env):
    """Training runs in FP32; the sweep evaluates the network with BF16 parameters, inputs and first
    hidden layer.  On samples drawn with the training recipe from held-out problems, the loss of the
    deployed evaluation stays within 1 % of the FP32 training forward's, and both stay below the
    loss of van Leer's slope on the same samples."""
    H, torch = env
    from paper_2503_04428_amd import learned
    try:
        w = learned.load_weights()
    except OSError:
        pytest.skip("no trained weights")
    announce("deployed BF16 loss vs FP32 training loss")
    samples, info = learned.generate_samples(nprob=128, ncoarse=256, ratio=4, times=(0.02, 0.04, 0.06), seed=4321)
    assert info["samples"] > 10000
    l32 = learned.training_loss(w, samples)
    ldep = learned.deployed_loss(w, samples)
    lvl = learned.baseline_loss(samples, "vanleer")
    print(f"loss on {info['samples']} held-out samples: FP32 training forward {l32:.5f}, deployed BF16 "
          f"{ldep:.5f} ({(ldep - l32) / l32:+.2%}), van Leer {lvl:.5f}")
    assert abs(ldep - l32) <= 0.01 * l32
    assert ldep < lvl and l32 < lvl


@pytest.mark.parametrize("t_end", [0.05, 0.1])
def test_trained_network_gains_over_vanleer(env, t_end):
    """What the trained network gains: on held-out 1D Riemann problems (a seed that neither the
    training set nor its validation set used), the learned FP32 form's L1 error against the 4x-fine
    FP64 solution restricted to the coarse grid is below that of van Leer, in FP32 and in FP64, for
    rho, the momentum and E (relative L1 over 128 problems of 256 cells)."""
    H, torch = env
    from paper_2503_04428_amd import learned
    try:
        w = learned.load_weights()
    except OSError:
        pytest.skip("no trained weights")
    announce(f"learned gain, held-out problems, t_end={t_end}")
    res = learned.coarse_error(w, nprob=128, ncoarse=256, ratio=4, t_end=t_end, seed=7000)
    names = {0: "rho", 1: "m", 4: "E"}
    for v, nm in names.items():
        lr, vf, vd = res["learned_fp32"][v], res["vanleer_fp32"][v], res["vanleer_fp64"][v]
        print(f"t={t_end} {nm}: L1 learned {lr:.4e}, van Leer FP32 {vf:.4e}, FP64 {vd:.4e}, "
              f"ratio {lr / vf:.3f}")
        assert lr < vf and lr < vd, (nm, lr, vf, vd)
