"""Learned warm start on the GPU against the FP64 oracle.

Descriptors (FP32 on the GPU) are compared to the FP64 oracle at 1e-5
relative.  The network runs on BF16 MFMA; the oracle rounds the matrix-product
operands to bf16 at the same points, so the two sides differ by FP32 vs FP64
accumulation, plus the rare bf16 rounding decision that FP32 and FP64 values
straddle (a handful of activations per thousand atoms): most outputs agree to
1e-5, all to 1e-2 of the output scale; gradients (sums over atoms) to 1e-3
relative.
"""
import numpy as np
import pytest

from inputs import gen
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CENTERS = np.linspace(1.0, 9.0, 16)
WIDTH, RCUT_DESC = 0.5, 9.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def T(a, dev, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def oracle_params(nets):
    p = np.zeros(len(nets) * omlp.STRIDE)
    for e, n in enumerate(nets):
        o = e * omlp.STRIDE
        p[o + omlp.OFF_W1:o + omlp.OFF_W1 + 512] = np.asarray(n["W1"]).ravel()
        p[o + omlp.OFF_B1:o + omlp.OFF_B1 + 32] = n["b1"]
        p[o + omlp.OFF_W2:o + omlp.OFF_W2 + 1024] = np.asarray(n["W2"]).ravel()
        p[o + omlp.OFF_B2:o + omlp.OFF_B2 + 32] = n["b2"]
        p[o + omlp.OFF_W3:o + omlp.OFF_W3 + 32] = n["W3"]
        p[o + omlp.OFF_B3] = n["b3"]
    return p


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("which", ["n512", "batch11", "n512_weighted", "batch11_weighted"])
def test_descriptors_match_oracle(dev, which):
    """Plain and neighbour-weighted radial descriptors (weights = chi, signed)."""
    from paper_2607_17978_amd import qeq
    s = gen.system_512() if which.startswith("n512") else gen.batch_structure(11)
    w = s.chi if which.endswith("weighted") else None
    plan = qeq.Plan(s.n, eta=2.0, r_cut=11.0, grid=s.grid)
    G = plan.descriptors(T(s.pos, dev), s.cell, T(s.sigma, dev), CENTERS, WIDTH, RCUT_DESC,
                         weights=None if w is None else T(w, dev)).cpu().numpy()
    ref = omlp.radial_descriptors(s.pos, s.cell, CENTERS, WIDTH, RCUT_DESC, weights=w)
    err = np.abs(G - ref).max() / np.abs(ref).max()
    print(which, "desc rel err", err)
    assert err <= 1e-5
    plan.close()


def _setup(dev, n=2048, seed=3):
    rng = np.random.default_rng(seed)
    G = rng.gamma(2.0, 0.6, size=(n, 16))
    species = (rng.uniform(size=n) < 0.5).astype(np.int32)
    target = rng.normal(0, 0.2, n)
    nets = gen.warmstart_init(1005, 2)
    return G, species, target, nets


def test_feature_stats_and_forward(dev):
    from paper_2607_17978_amd import qeq
    G, species, target, nets = _setup(dev)
    net = qeq.WarmStartNet(nets, device=dev)
    Gd = T(G, dev, torch.float32)
    sd = T(species, dev, torch.int32)
    net.fit_scaling(Gd, sd)
    stats = net.stats.cpu().numpy().reshape(2, 3, 16)
    ref_stats = omlp.feature_stats(f32(G), species, 2)
    assert np.abs(stats - ref_stats).max() <= 1e-5 * np.abs(ref_stats).max()
    y = net.predict(Gd, sd).cpu().numpy()
    X = omlp.scale(f32(G), species, f32(ref_stats))
    ref_y, _ = omlp.forward(oracle_params(nets), X, species, use_bf16=True)
    d = np.abs(y - ref_y)
    print("forward: frac > 1e-5:", np.mean(d > 1e-5), "max", d.max())
    assert np.mean(d > 1e-5) < 0.01
    assert d.max() <= 1e-2 * np.abs(ref_y).max()


def test_gradients_and_adam(dev):
    from paper_2607_17978_amd import qeq
    G, species, target, nets = _setup(dev, seed=4)
    net = qeq.WarmStartNet(nets, device=dev)
    Gd, sd, td = T(G, dev, torch.float32), T(species, dev, torch.int32), T(target, dev)
    net.fit_scaling(Gd, sd)
    stats = omlp.feature_stats(f32(G), species, 2)
    X = omlp.scale(f32(G), species, f32(stats))
    p0 = oracle_params(nets)
    grad = torch.zeros_like(net.params)
    loss = float(net.train_step(Gd, sd, td, update=False, grad_out=grad).cpu())
    y, cache = omlp.forward(p0, X, species, use_bf16=True)
    ref_loss, dy = omlp.mse_loss(y, target)
    ref_g = omlp.backward(p0, cache, dy, use_bf16=True)
    g = grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    print("loss", loss, ref_loss, "grad rel", rel)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    assert rel <= 1e-3
    # three Adam steps against the oracle's Adam on its own gradients
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in (1, 2, 3):
        net.train_step(Gd, sd, td, lr=1e-3)
        y, cache = omlp.forward(p, X, species, use_bf16=True)
        _, dy = omlp.mse_loss(y, target)
        p, m, v = omlp.adam(p, omlp.backward(p, cache, dy, use_bf16=True), m, v, step)
    dp = np.abs(net.params.cpu().numpy() - p)
    print("adam: frac > 1e-6:", np.mean(dp > 1e-6), "max", dp.max())
    assert np.mean(dp > 1e-6) < 0.02
    assert dp.max() <= 6e-3   # a sign flip of a near-zero gradient moves a weight by ~2 lr


def test_training_reduces_loss(dev):
    from paper_2607_17978_amd import qeq
    G, species, target, nets = _setup(dev, n=4096, seed=5)
    # a learnable target: a smooth function of the features
    target = np.tanh(G[:, 0] - G[:, 5]) * 0.2 + 0.05 * species
    net = qeq.WarmStartNet(nets, device=dev)
    Gd, sd, td = T(G, dev, torch.float32), T(species, dev, torch.int32), T(target, dev)
    net.fit_scaling(Gd, sd)
    first = float(net.train_step(Gd, sd, td, lr=3e-3).cpu())
    for _ in range(300):
        last = net.train_step(Gd, sd, td, lr=3e-3)
    last = float(last.cpu())
    print("loss", first, "->", last)
    assert last < 0.2 * first


def test_learned_warm_start_on_small_trajectory(dev):
    """4,096-atom version of the trajectory workload: the trained networks'
    starts need fewer CG iterations than the cold start, the
    electronegativity-aware one fewer than the previous frame's charges, and
    every start converges to the cold-start charges."""
    from paper_2607_17978_amd import warmstart
    out = warmstart.run_trajectory(n=4096, side=17, frames=24, epochs=40, tol=1e-6, device=dev)
    print(out)
    for k in ("cold", "prev", "learned", "learned_chi"):
        assert out[k]["all_converged"]
    assert out["max_dq_vs_cold"] <= 1e-5
    assert out["learned"]["iters"] < out["cold"]["iters"]
    assert out["prev"]["iters"] < out["cold"]["iters"]
    assert out["learned_chi"]["iters"] < out["prev"]["iters"]


def test_descriptors_reuse_geometry(dev):
    """pos=None reuses the geometry of the last solve / descriptor call: same
    values as a fresh set-up, and the solve's tape stays valid."""
    from paper_2607_17978_amd import qeq
    s = gen.system_512()
    plan = qeq.Plan(s.n, eta=2.0, r_cut=11.0, grid=s.grid, tol=1e-8)
    pos, sig, chi = T(s.pos, dev), T(s.sigma, dev), T(s.chi, dev)
    with pytest.raises(qeq.QEqError):
        plan.descriptors(None, s.cell, sig, CENTERS, WIDTH, RCUT_DESC)   # nothing to reuse yet
    G0 = plan.descriptors(pos, s.cell, sig, CENTERS, WIDTH, RCUT_DESC, weights=chi)
    G1 = plan.descriptors(None, s.cell, sig, CENTERS, WIDTH, RCUT_DESC, weights=chi)
    assert torch.equal(G0, G1)
    plan.solve(pos, s.cell, sig, T(s.J, dev), chi, s.q_tot)
    g = T(np.random.default_rng(2).normal(size=s.n), dev)
    d0 = plan.backward(g, 0.0, 0.0)[0].cpu().numpy()
    G2 = plan.descriptors(None, s.cell, sig, CENTERS, WIDTH, RCUT_DESC)
    d1 = plan.backward(g, 0.0, 0.0)[0].cpu().numpy()   # tape kept
    assert np.abs(d0 - d1).max() <= 1e-12 * np.abs(d0).max()
    G3 = plan.descriptors(pos, s.cell, sig, CENTERS, WIDTH, RCUT_DESC)
    assert torch.equal(G2, G3)
    plan.close()
