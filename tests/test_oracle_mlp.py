"""Pins of the warm-start network oracle (oracle/mlp.py) on the CPU.

Each function is checked against something other than itself: bfloat16
rounding against hand-chosen values whose correct rounding follows from the
format (8 significant bits, ties to even); Adam against its closed form after
one step and a three-step sequence summed out by hand; the loss, the scaling
and the statistics against hand values; the network against per-atom scalar
loops and its gradient against central differences; the bf16 network against
the error bound that bf16's unit roundoff propagates through the layers.
Planted mistakes (a missing bias correction, truncation instead of rounding,
a transposed weight) are shown to fail the corresponding pin.
"""
import math

import numpy as np
import pytest

from inputs import gen
from oracle import mlp

U = 2.0 ** -8


# ----------------------------------------------------------------- bfloat16
@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                       # tie, even neighbour below
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),       # tie, even neighbour above
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),   # just above the tie: up
    (1.0 + 2.0 ** -8 - 2.0 ** -20, 1.0),          # just below the tie: down
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),  # sign-symmetric
    (0.1, 0.10009765625),                         # 0.1 = 1.6 * 2^-4 -> 205/2048
    (3.0e38, 226 * 2.0 ** 120),                   # 3e38 = 225.7 * 2^120: up to 226
    ((2.0 - 2.0 ** -8) * 2.0 ** 127, math.inf),   # tie at the top: to even = overflow
    (3.4028234e38, math.inf),                     # float32 max overflows
    (-3.4028234e38, -math.inf),
    (2.0 ** -133, 2.0 ** -133),                   # smallest subnormal kept
    (2.0 ** -134, 0.0),                           # tie with zero: even (zero)
    (3 * 2.0 ** -134, 2.0 ** -132),               # subnormal tie, even neighbour above
    (math.inf, math.inf),
])
def test_bf16_rounds_to_nearest_even(x, want):
    got = float(mlp.bf16(np.array([x]))[0])
    if want == 0.0 or math.isinf(want):
        assert got == want
    else:
        assert got == want


def test_bf16_special_values_and_a_planted_truncation():
    r = mlp.bf16(np.array([np.nan, -0.0, 0.0]))
    assert np.isnan(r[0]) and r[1] == 0.0 and math.copysign(1.0, r[1]) < 0 and r[2] == 0.0
    # NaN payloads in the low bits stay NaN (a plain add-and-mask turns them into inf)
    nan_low = np.array([0x7F800001], dtype=np.uint32).view(np.float32)
    assert np.isnan(mlp.bf16(nan_low))[0]
    # every result has at most 8 significant bits and is the nearest such number
    rng = np.random.default_rng(0)
    x = (rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32).astype(np.float64)
    r = mlp.bf16(x)
    m, e = np.frexp(r)
    assert np.all(m * 256 == np.rint(m * 256))
    assert np.all(np.abs(r - x) <= U * np.abs(x))
    # truncation (round toward zero) would fail the tie/round-up pins
    trunc = np.trunc(x / np.ldexp(1.0, np.frexp(x)[1] - 8)) * np.ldexp(1.0, np.frexp(x)[1] - 8)
    assert np.any(trunc != r)


# ---------------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    """Step 1: m_hat = g, v_hat = g^2, so the update is -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-9, 0.0, 5e3])
    p0 = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    lr = 1e-3
    p, m, v = mlp.adam(p0, g, np.zeros(5), np.zeros(5), 1, lr=lr)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_three_steps_summed_by_hand():
    """Three steps with gradients g1, g2, g3, the moments written out:
    m3 = 0.1 (0.81 g1 + 0.9 g2 + g3), v3 = 0.001 (0.998001 g1^2 + 0.999 g2^2 + g3^2),
    bias corrections 1 - 0.9^t and 1 - 0.999^t."""
    g1, g2, g3 = 0.5, -1.0, 2.0
    lr = 0.01
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t, g in enumerate((g1, g2, g3), start=1):
        p, m, v = mlp.adam(p, np.array([g]), m, v, t, lr=lr)
    m1, v1 = 0.1 * g1, 0.001 * g1 ** 2
    m2, v2 = 0.1 * (0.9 * g1 + g2), 0.001 * (0.999 * g1 ** 2 + g2 ** 2)
    m3, v3 = 0.1 * (0.81 * g1 + 0.9 * g2 + g3), 0.001 * (0.998001 * g1 ** 2 + 0.999 * g2 ** 2 + g3 ** 2)
    steps = [m1 / 0.1 / (math.sqrt(v1 / 0.001) + 1e-8),
             m2 / 0.19 / (math.sqrt(v2 / 0.001999) + 1e-8),
             m3 / 0.271 / (math.sqrt(v3 / 0.002997001) + 1e-8)]
    want = -lr * sum(steps)
    assert abs(p[0] - want) <= 1e-14
    assert abs(m[0] - m3) <= 1e-15 and abs(v[0] - v3) <= 1e-15

    # a planted mistake: Adam without the bias correction moves far less
    def adam_no_bc(p, g, m, v, step, lr):
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        return p - lr * m / (np.sqrt(v) + 1e-8), m, v
    q, mm, vv = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t, g in enumerate((g1, g2, g3), start=1):
        q, mm, vv = adam_no_bc(q, np.array([g]), mm, vv, t, lr)
    assert abs(q[0] - want) > 1e-3


def test_adam_is_invariant_to_the_gradient_scale():
    """With eps = 0 the update depends on the gradients only through their
    ratios (m_hat / sqrt(v_hat) is homogeneous of degree 0)."""
    rng = np.random.default_rng(1)
    gs = [rng.normal(size=50) for _ in range(4)]
    runs = []
    for c in (1.0, 1e3, 1e-3):
        p, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
        for t, g in enumerate(gs, start=1):
            p, m, v = mlp.adam(p, c * g, m, v, t, lr=1e-2, eps=0.0)
        runs.append(p)
    assert np.abs(runs[0] - runs[1]).max() <= 1e-15
    assert np.abs(runs[0] - runs[2]).max() <= 1e-15


# ------------------------------------------------- loss, scaling, statistics
def test_mse_loss_hand_values_and_gradient():
    y, t = np.array([1.0, 2.0, 3.0]), np.array([0.0, 2.0, 5.0])
    L, g = mlp.mse_loss(y, t)
    assert L == pytest.approx(5.0 / 6.0, abs=1e-15)
    assert np.allclose(g, [1.0 / 3.0, 0.0, -2.0 / 3.0], atol=1e-15)
    h = 1e-6
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (mlp.mse_loss(y + e, t)[0] - mlp.mse_loss(y - e, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-9


def test_feature_stats_and_scale_hand_values():
    G = np.array([[0.0, 5.0], [1.0, 5.0], [3.0, 5.0], [10.0, -2.0], [20.0, 4.0]])
    species = np.array([0, 0, 0, 1, 1], dtype=np.int32)
    st = mlp.feature_stats(G, species, 2)
    assert np.allclose(st[0], [[4.0 / 3.0, 5.0], [0.0, 5.0], [3.0, 5.0]])
    assert np.allclose(st[1], [[15.0, 1.0], [10.0, -2.0], [20.0, 4.0]])
    X = mlp.scale(G, species, st)
    # species 0: (G - 4/3) / 3 and a zero-range feature -> (G - mean) / 1 = 0
    assert np.allclose(X[:3, 0], [-4.0 / 9.0, -1.0 / 9.0, 5.0 / 9.0])
    assert np.all(X[:3, 1] == 0.0)
    assert np.allclose(X[3:], [[-0.5, -0.5], [0.5, 0.5]])
    # outside the training range: clipped to +-1.5
    Xo = mlp.scale(np.array([[100.0, 0.0], [-100.0, 0.0]]), np.array([0, 1], dtype=np.int32), st)
    assert Xo[0, 0] == 1.5 and Xo[1, 0] == -1.5


# --------------------------------------------------------- network and gradient
def _net(seed=2, n=40):
    rng = np.random.default_rng(seed)
    nets = gen.warmstart_init(1005, 2)
    p = np.zeros(2 * mlp.STRIDE)
    for e, nt in enumerate(nets):
        o = e * mlp.STRIDE
        p[o + mlp.OFF_W1:o + mlp.OFF_W1 + 512] = np.asarray(nt["W1"]).ravel()
        p[o + mlp.OFF_B1:o + mlp.OFF_B1 + 32] = rng.normal(0, 0.3, 32)
        p[o + mlp.OFF_W2:o + mlp.OFF_W2 + 1024] = np.asarray(nt["W2"]).ravel()
        p[o + mlp.OFF_B2:o + mlp.OFF_B2 + 32] = rng.normal(0, 0.3, 32)
        p[o + mlp.OFF_W3:o + mlp.OFF_W3 + 32] = np.asarray(nt["W3"]).ravel()
        p[o + mlp.OFF_B3] = 0.05 * (e + 1)
    X = rng.uniform(-1.2, 1.2, size=(n, 16))
    species = rng.integers(0, 2, n).astype(np.int32)
    return p, X, species


def test_forward_matches_scalar_loops():
    p, X, species = _net()
    y, _ = mlp.forward(p, X, species)
    for a in range(X.shape[0]):
        o = species[a] * mlp.STRIDE
        h1 = []
        for j in range(32):
            z = p[o + mlp.OFF_B1 + j]
            for k in range(16):
                z += p[o + mlp.OFF_W1 + 16 * j + k] * X[a, k]
            h1.append(math.tanh(z))
        out = p[o + mlp.OFF_B3]
        for j in range(32):
            z = p[o + mlp.OFF_B2 + j]
            for k in range(32):
                z += p[o + mlp.OFF_W2 + 32 * j + k] * h1[k]
            out += p[o + mlp.OFF_W3 + j] * math.tanh(z)
        assert abs(y[a] - out) <= 1e-12


def test_backward_matches_central_differences():
    p, X, species = _net(seed=3, n=24)
    dy = np.random.default_rng(4).normal(size=X.shape[0])
    _, cache = mlp.forward(p, X, species)
    g = mlp.backward(p, cache, dy)
    f = lambda pp: float(dy @ mlp.forward(pp, X, species)[0])
    rng = np.random.default_rng(5)
    idx = []
    for e in range(2):
        o = e * mlp.STRIDE
        for off, size in ((mlp.OFF_W1, 512), (mlp.OFF_B1, 32), (mlp.OFF_W2, 1024), (mlp.OFF_B2, 32),
                          (mlp.OFF_W3, 32), (mlp.OFF_B3, 1)):
            idx += list(o + off + rng.choice(size, min(size, 4), replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (f(p + e) - f(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * (1 + abs(fd)), (i, fd, g[i])
    # padding entries of the packed layout carry no gradient
    for e in range(2):
        assert np.all(g[e * mlp.STRIDE + mlp.N_PARAM:(e + 1) * mlp.STRIDE] == 0.0)


def test_bf16_network_stays_within_the_propagated_bounds():
    """Outputs of the bf16 network differ from the FP64 network by no more than
    the first-order worst-case bound and the (tighter) probabilistic bound;
    the probabilistic one is not vacuous (below 3% of the output scale) and a
    planted rounding to 5 significant bits (8x coarser than bf16) breaks it.
    Gradients of the loss stay within their worst-case first-order bound."""
    p, X, species = _net(seed=6, n=2000)
    t = np.random.default_rng(7).normal(0, 0.2, X.shape[0])
    y64, c64 = mlp.forward(p, X, species)
    y16, c16 = mlp.forward(p, X, species, use_bf16=True)
    _, dy64 = mlp.mse_loss(y64, t)
    _, dy16 = mlp.mse_loss(y16, t)
    ey, gb = mlp.bf16_error_bounds(p, X, species, dy64, dy_err=None)
    pb = mlp.bf16_output_prob_bound(p, X, species)
    assert np.all(np.abs(y16 - y64) <= ey)
    assert np.all(np.abs(y16 - y64) <= pb)
    assert pb.max() <= 0.03 * np.abs(y64).max()
    _, gb = mlp.bf16_error_bounds(p, X, species, dy64, dy_err=ey / X.shape[0])
    g64 = mlp.backward(p, c64, dy64)
    g16 = mlp.backward(p, c16, dy16, use_bf16=True)
    assert np.all(np.abs(g16 - g64) <= gb + 1e-15)

    def coarse(a):
        f = np.asarray(a, dtype=np.float64)
        q = np.ldexp(1.0, np.frexp(f)[1] - 5)
        return np.rint(f / q) * q
    orig = mlp.bf16
    try:
        mlp.bf16 = coarse
        yc, _ = mlp.forward(p, X, species, use_bf16=True)
    finally:
        mlp.bf16 = orig
    assert np.any(np.abs(yc - y64) > pb)
