"""FP64 oracle for the learned warm start (test infrastructure only).

* ``radial_descriptors`` -- radial symmetry functions of the paper's type-2
  ACSF (eq. g2; SI "Radial ACSF"): G_i,mu = sum_j exp(-eta_mu (r_ij - R_mu)^2)
  f_c(r_ij) with the cosine cutoff f_c(r) = (cos(pi r / r_c) + 1) / 2 (SI
  cutoff functions, inner radius 0), over all periodic images, all neighbours
  (not element-resolved); optionally each neighbour term carries a scalar
  weight w_j (the paper's weighted ACSFs with a per-neighbour prefactor).
* ``feature_stats`` / ``scale`` -- per-element feature scaling
  (G - mean) / (max - min) (SI "Feature scaling").
* ``forward`` / ``backward`` -- the element network: tanh hidden layers and a
  linear output (SI "Feed-forward neural networks"; activations), with an
  optional bf16 rounding of the matrix-product operands at the points where
  the GPU kernel rounds them, so that both sides take the same rounding
  decisions and differ only by FP32 vs FP64 accumulation.
* ``mse_loss`` -- 1/2 mean squared error (SI loss functions, 1/2 prefactor).
* ``adam`` -- Adam update (SI "Adam": beta1 0.9, beta2 0.999, eps 1e-8).

Pins (tests/test_oracle_mlp.py): bf16 on hand-chosen values (ties to even
both ways, round-up, overflow to infinity, NaN, subnormals); Adam against its
step-1 closed form -lr g / (|g| + eps), a three-step sequence with the bias
corrections summed out by hand and its invariance to the gradient scale;
mse_loss, scale and feature_stats on hand values; forward against per-atom
scalar loops; backward against central differences; the bf16 forward within
the error bound that bf16's unit roundoff 2^-8 propagates through the layers.
"""
from __future__ import annotations

import math

import numpy as np

from . import matfree

# parameter layout of one element network 16-32-32-1 (row-major weights)
N_IN, N_H = 16, 32
OFF_W1, OFF_B1 = 0, 512
OFF_W2, OFF_B2 = 544, 1568
OFF_W3, OFF_B3 = 1600, 1632
N_PARAM = 1633
STRIDE = 1664          # per-element stride in the packed parameter vector


def radial_descriptors(pos, cell, centers, width, r_cut, weights=None):
    """G (N x n_mu) with eta_mu = 1 / (2 width^2) and the cosine cutoff; with
    weights, every neighbour term is multiplied by its neighbour's weight w_j
    (weighted ACSF)."""
    pos = np.asarray(pos, dtype=np.float64)
    ii, jj, d = matfree.real_space_pairs(pos, cell, r_cut)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    fc = 0.5 * (np.cos(math.pi * r / r_cut) + 1.0)
    if weights is not None:
        fc = fc * np.asarray(weights, dtype=np.float64)[jj]
    eta = 1.0 / (2.0 * width * width)
    G = np.zeros((pos.shape[0], len(centers)))
    for m, c in enumerate(centers):
        G[:, m] = np.bincount(ii, weights=np.exp(-eta * (r - c) ** 2) * fc, minlength=pos.shape[0])
    return G


def feature_stats(G, species, n_species):
    """(n_species, 3, n_feat): mean, min, max per element."""
    out = np.zeros((n_species, 3, G.shape[1]))
    for s in range(n_species):
        g = G[species == s]
        out[s, 0], out[s, 1], out[s, 2] = g.mean(0), g.min(0), g.max(0)
    return out


CLIP = 1.5


def scale(G, species, stats):
    """(G - mean) / (max - min), clipped to [-1.5, 1.5].

    Training data scale into [-1, 1]; the clip only bounds features of atoms
    that leave the training range (the extrapolation the paper monitors during
    MD), which would otherwise saturate the network.
    """
    mean, mn, mx = stats[species, 0], stats[species, 1], stats[species, 2]
    rng = np.where(mx - mn > 0, mx - mn, 1.0)
    return np.clip((G - mean) / rng, -CLIP, CLIP)


BF16_SIG = 8                 # significant bits of bfloat16 (7 stored + the implicit one)
BF16_EMIN = -126             # smallest normal exponent (the float32 exponent range)
BF16_MAX_EXP = 128           # values of magnitude >= 2^128 overflow


def bf16(x):
    """bfloat16 rounding of float32 values, returned as float64.

    The value is first rounded to float32 (the type the kernels hold their
    activations in), then to the nearest number with 8 significant bits whose
    exponent lies in the float32 range, ties to the even neighbour: the quantum
    is 2^(e - 8) for x = m 2^e, 1/2 <= |m| < 1, but never below the subnormal
    quantum 2^(-126 - 7).  Results of magnitude 2^128 or more overflow to
    infinity; NaN stays NaN, infinities and signed zeros are kept.
    """
    with np.errstate(invalid="ignore", over="ignore"):
        f = np.asarray(x, dtype=np.float32).astype(np.float64)
    out = f.copy()
    fin = np.isfinite(f) & (f != 0.0)
    _, e = np.frexp(f[fin])
    quantum = np.ldexp(1.0, np.maximum(e - BF16_SIG, BF16_EMIN - (BF16_SIG - 1)))
    r = np.rint(f[fin] / quantum) * quantum            # rint: ties to even
    r[np.abs(r) >= 2.0 ** BF16_MAX_EXP] = np.inf * np.sign(r[np.abs(r) >= 2.0 ** BF16_MAX_EXP])
    out[fin] = r
    return out


def unpack(params, s):
    p = np.asarray(params, dtype=np.float64)[s * STRIDE:(s + 1) * STRIDE]
    W1 = p[OFF_W1:OFF_W1 + 512].reshape(32, 16)
    b1 = p[OFF_B1:OFF_B1 + 32]
    W2 = p[OFF_W2:OFF_W2 + 1024].reshape(32, 32)
    b2 = p[OFF_B2:OFF_B2 + 32]
    W3 = p[OFF_W3:OFF_W3 + 32]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def forward(params, X, species, use_bf16=False):
    """Per-atom output of its element's network and the cache for backward."""
    rb = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    n = X.shape[0]
    y = np.zeros(n)
    cache = {}
    for s in np.unique(species):
        m = species == s
        W1, b1, W2, b2, W3, b3 = unpack(params, s)
        x = rb(X[m])
        z1 = x @ rb(W1).T + b1
        h1 = np.tanh(z1)
        h1r = rb(h1)
        z2 = h1r @ rb(W2).T + b2
        h2 = np.tanh(z2)
        y[m] = h2 @ W3 + b3
        cache[s] = (m, x, h1, h1r, h2)
    return y, cache


def backward(params, cache, dy, use_bf16=False):
    """Gradient of sum(dy * y) with respect to the packed parameters."""
    rb = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    g = np.zeros_like(np.asarray(params, dtype=np.float64))
    for s, (m, x, h1, h1r, h2) in cache.items():
        W1, b1, W2, b2, W3, b3 = unpack(params, s)
        d = dy[m]
        gs = g[s * STRIDE:(s + 1) * STRIDE]
        gs[OFF_W3:OFF_W3 + 32] = h2.T @ d
        gs[OFF_B3] = d.sum()
        dz2 = (d[:, None] * W3[None, :]) * (1.0 - h2 * h2)
        dz2r = rb(dz2)
        gs[OFF_W2:OFF_W2 + 1024] = (dz2r.T @ h1r).ravel()
        gs[OFF_B2:OFF_B2 + 32] = dz2.sum(0)
        dh1 = dz2r @ rb(W2)
        dz1 = dh1 * (1.0 - h1 * h1)
        dz1r = rb(dz1)
        gs[OFF_W1:OFF_W1 + 512] = (dz1r.T @ x).ravel()
        gs[OFF_B1:OFF_B1 + 32] = dz1.sum(0)
    return g


BF16_U = 2.0 ** -BF16_SIG    # unit roundoff of bfloat16 (round to nearest)


def bf16_error_bounds(params, X, species, dy, dy_err=None, u=BF16_U):
    """First-order bounds on how far the bf16 network (``use_bf16=True``) can be
    from the FP64 one, per output and per gradient component.

    Every bf16 rounding multiplies a value by (1 + d) with |d| <= u.  With the
    FP64 activations x, h1 = tanh(z1), h2 = tanh(z2) and |tanh'| <= 1:
      z1 error  e1 = 2u |x| |W1|^T             (x and W1 rounded)
      h1 error  e1;  rounded h1: e1 + u |h1|
      z2 error  e2 = (e1 + 2u |h1|) |W2|^T      (h1 rounded, W2 rounded)
      h2 error  e2;  y error  ey = e2 |W3|      (output layer in FP32)
    and through the backward pass of sum(dy * y), whose output gradient dy
    may itself be off by dy_err (from ey):
      dz2 = dy W3 (1 - h2^2):   e_dz2 = (|dy| 2|h2| e2 + dy_err) |W3|
      dW2 = dz2r^T h1r:         sum (e_dz2 + u|dz2|) |h1| + |dz2| (e1 + u|h1|)
      dh1 = dz2r W2r:           (e_dz2 + 2u |dz2|) |W2|
      dz1 = dh1 (1 - h1^2):     e_dh1 + |dh1| 2|h1| e1
      dW1 = dz1r^T x:           sum (e_dz1 + 2u |dz1|) |x|
    bias and W3 gradients likewise without their own rounding.  Products of
    two u terms are dropped (first order); the bound is worst case over signs.
    Returns (ey per atom, gradient bound like ``params``).
    """
    dy = np.asarray(dy, dtype=np.float64)
    dy_err = np.zeros_like(dy) if dy_err is None else np.asarray(dy_err, dtype=np.float64)
    n = X.shape[0]
    ey = np.zeros(n)
    gb = np.zeros_like(np.asarray(params, dtype=np.float64))
    for s in np.unique(species):
        m = species == s
        W1, b1, W2, b2, W3, b3 = unpack(params, s)
        aW1, aW2, aW3 = np.abs(W1), np.abs(W2), np.abs(W3)
        x = np.asarray(X[m], dtype=np.float64)
        h1 = np.tanh(x @ W1.T + b1)
        h2 = np.tanh(h1 @ W2.T + b2)
        ax, ah1, ah2 = np.abs(x), np.abs(h1), np.abs(h2)
        e1 = 2.0 * u * (ax @ aW1.T)
        e2 = (e1 + 2.0 * u * ah1) @ aW2.T
        ey[m] = e2 @ aW3
        d, de = np.abs(dy[m]), dy_err[m]
        g = gb[s * STRIDE:(s + 1) * STRIDE]
        g[OFF_W3:OFF_W3 + 32] = d @ e2 + de @ ah2
        g[OFF_B3] = de.sum()
        dz2 = (d[:, None] * aW3[None, :]) * (1.0 - h2 * h2)
        e_dz2 = (d[:, None] * 2.0 * ah2 * e2 + de[:, None] * (1.0 - h2 * h2)) * aW3[None, :]
        g[OFF_W2:OFF_W2 + 1024] = ((e_dz2 + u * dz2).T @ ah1 + dz2.T @ (e1 + u * ah1)).ravel()
        g[OFF_B2:OFF_B2 + 32] = e_dz2.sum(0)
        dh1 = dz2 @ aW2
        e_dh1 = (e_dz2 + 2.0 * u * dz2) @ aW2
        dz1 = dh1 * (1.0 - h1 * h1)
        e_dz1 = e_dh1 * (1.0 - h1 * h1) + dh1 * 2.0 * ah1 * e1
        g[OFF_W1:OFF_W1 + 512] = ((e_dz1 + 2.0 * u * dz1).T @ ax).ravel()
        g[OFF_B1:OFF_B1 + 32] = e_dz1.sum(0)
    return ey, gb


def bf16_output_prob_bound(params, X, species, lam=6.0, u=BF16_U):
    """Probabilistic bound on |y_bf16 - y_fp64| per atom (the probabilistic
    rounding-error analysis of Higham and Mary, SIAM J. Sci. Comput. 41 (2019)
    A2815: rounding errors modelled as independent, mean-zero and bounded by u).

    To first order y_bf16 - y = sum_r c_r d_r over the rounding sites r (the
    inputs x, W1, the hidden activations h1, W2), with c_r = (dy/dv_r) v_r and
    |d_r| <= u; Hoeffding's inequality bounds the sum by lam u sqrt(sum c_r^2)
    except with probability 2 exp(-lam^2 / 2) (3e-8 for lam = 6).  The
    sensitivities are the FP64 network's: s3 = W3 (1 - h2^2) = dy/dz2,
    dy/dh1 = s3 W2, s1 = dy/dh1 (1 - h1^2) = dy/dz1, dy/dx = s1 W1.
    """
    n = X.shape[0]
    out = np.zeros(n)
    for s in np.unique(species):
        m = species == s
        W1, b1, W2, b2, W3, b3 = unpack(params, s)
        x = np.asarray(X[m], dtype=np.float64)
        h1 = np.tanh(x @ W1.T + b1)
        h2 = np.tanh(h1 @ W2.T + b2)
        s3 = W3[None, :] * (1.0 - h2 * h2)
        gh1 = s3 @ W2
        s1 = gh1 * (1.0 - h1 * h1)
        gx = s1 @ W1
        c2 = (np.sum((gh1 * h1) ** 2, 1)                         # h1 rounded
              + np.sum(s3 ** 2 * ((h1 ** 2) @ (W2 ** 2).T), 1)   # W2 rounded
              + np.sum((gx * x) ** 2, 1)                          # x rounded
              + np.sum(s1 ** 2 * ((x ** 2) @ (W1 ** 2).T), 1))   # W1 rounded
        out[m] = lam * u * np.sqrt(c2)
    return out


def mse_loss(y, target):
    """L = 1/2 mean (y - t)^2 and dL/dy."""
    r = y - target
    return 0.5 * np.mean(r * r), r / r.shape[0]


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def charge_loss_through_qeq(params, X, species, pos, cell, sigma, J, q_tot, q_ref, use_bf16=False):
    """4G charge training: electronegativities from the element networks, charges
    from the QEq solve, loss L = mean_i (q_i - q_ref,i)^2 and its parameter
    gradient by the chain rule dL/dtheta = sum_i dL/dchi_i dchi_i/dtheta, with
    dL/dchi from the adjoint of the solve (SI 4G section: the charges depend on
    chi through the linear system; eq. 4g_force_trick's Lagrange route).
    Returns (L, dL/dtheta, q, dL/dchi).
    """
    from . import ewald
    chi, cache = forward(params, X, species, use_bf16=use_bf16)
    E = ewald.coulomb_matrix(pos, cell, sigma)
    q, _ = ewald.solve_qeq(E, J, chi, q_tot)
    r = q - np.asarray(q_ref, dtype=np.float64)
    L = float(np.mean(r * r))
    _, dchi, _, _ = ewald.qeq_adjoint(pos, cell, sigma, J, chi, q_tot, 2.0 * r / r.shape[0])
    return L, backward(params, cache, dchi, use_bf16=use_bf16), q, dchi


def charge_loss_through_qeq_chi_j(params_chi, params_j, X, species, pos, cell, sigma, j_elem, j_scale, q_tot,
                                  q_ref, use_bf16=False):
    """As ``charge_loss_through_qeq`` with a second set of element networks for
    the hardness, J_i = j_elem_i exp(j_scale y_i) (positive, as J > 0 requires),
    y the J network's output.  dL/dJ from the same adjoint solve
    (dL/dJ_i = -a_i q_i), chained through the exponential.
    Returns (L, dL/dtheta_chi, dL/dtheta_J, q)."""
    from . import ewald
    chi, cache_c = forward(params_chi, X, species, use_bf16=use_bf16)
    y, cache_j = forward(params_j, X, species, use_bf16=use_bf16)
    J = np.asarray(j_elem, dtype=np.float64) * np.exp(j_scale * y)
    E = ewald.coulomb_matrix(pos, cell, sigma)
    q, _ = ewald.solve_qeq(E, J, chi, q_tot)
    r = q - np.asarray(q_ref, dtype=np.float64)
    L = float(np.mean(r * r))
    _, dchi, _, dJ = ewald.qeq_adjoint(pos, cell, sigma, J, chi, q_tot, 2.0 * r / r.shape[0])
    g_chi = backward(params_chi, cache_c, dchi, use_bf16=use_bf16)
    g_j = backward(params_j, cache_j, dJ * J * j_scale, use_bf16=use_bf16)
    return L, g_chi, g_j, q
