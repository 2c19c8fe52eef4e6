"""4G charge training through the QEq solve (workflow over the C ABI).

In a 4G-HDNNP the element networks predict electronegativities chi_i from the
atomic environment; the charges follow from the QEq solve, and the networks
are fitted so that those charges match reference charges (the paper's 4G
charge training; the SI's Lagrange route differentiates through the linear
system).  Here one training step on a structure is

    chi = net(G)                     element networks (mlp_forward, BF16 MFMA)
    q   = QEq(chi)                   qeq_solve
    L   = mean_i (q_i - q_ref,i)^2
    dL/dchi                          qeq_backward (one adjoint solve)
    Adam step with dL/dtheta = sum_i dL/dchi_i dchi_i/dtheta

The last line reuses the network's own training kernel, whose loss is
1/2 mean (y - t)^2: with the target t = chi - n dL/dchi its output gradient
(y - t)/n is exactly dL/dchi, so mlp_train_step back-propagates the QEq
gradient through the network and applies Adam.

Hardness networks (the 4G J_i) are trained the same way: J_i = J_e exp(s y_i)
with y the J network's output (positive for any output), and
dL/dy_i = dL/dJ_i J_i s with dL/dJ from the same adjoint solve.

The workload: a 4,096-atom subset of a simple-cubic lattice (density 0.01
bohr^-3) moving as in the trajectory workload; reference charges are QEq
charges of a hidden "teacher" electronegativity model (the fixed random
network on radial descriptors of the trajectory workload); the student sees
the same 16 radial descriptors.  The element-mean electronegativity (the
method without a chi network) is the baseline the trained network must beat.
"""
from __future__ import annotations

import time

import numpy as np

from . import qeq
from .warmstart import CENTERS, RCUT_DESC, WIDTH

J_SCALE = 0.2   # J_i = J_e exp(J_SCALE y_i): positive for any network output


def charge_step(plan, net, G, species, pos, cell, sigma, J, q_ref, q_tot=0.0, lr=2e-3, update=True,
                grad_out=None, jnet=None, j_scale=J_SCALE, jgrad_out=None):
    """One training step (or only the gradients with update=False, into
    grad_out / jgrad_out).  J: the element hardnesses; with ``jnet`` the
    hardness of atom i is J_i exp(j_scale y_i), y the J network's output, and
    that network is trained through dL/dJ of the same adjoint solve.
    Returns (loss, q, dL/dchi, solve stats, adjoint stats)."""
    n = int(G.shape[0])
    chi = net.predict(G, species)
    if jnet is not None:
        yj = jnet.predict(G, species)
        Jv = J * (j_scale * yj).exp()
    else:
        Jv = J
    q, _, _, st = plan.solve(pos, cell, sigma, Jv, chi, q_tot, forces=False)
    r = q - q_ref
    loss = float((r * r).mean())
    dchi, dJ, _, st_b = plan.backward(2.0 * r / n)
    net.train_step(G, species, chi - n * dchi, lr=lr, update=update, grad_out=grad_out)
    if jnet is not None:
        jnet.train_step(G, species, yj - n * (dJ * Jv * j_scale), lr=lr, update=update, grad_out=jgrad_out)
    return loss, q, dchi, st, st_b


def init_networks(n_species=2, seed=1011, chi_means=(0.1, -0.1)):
    """Xavier weights, output weights scaled by 0.1 and output biases at the
    element means: an untrained network starts near the element-mean model
    (chi_means = (0, 0) for the J networks: J starts at the element value)."""
    from inputs import gen
    nets = gen.warmstart_init(seed, n_species)
    for e, net in enumerate(nets):
        net["W3"] = 0.1 * np.asarray(net["W3"])
        net["b3"] = chi_means[e]
    return nets


def run_chi_training(n=4096, side=17, train_frames=8, test_frames=4, epochs=40, lr=2e-3, tol=1e-8,
                     device=None, log=None, train_j=False, vary_j=None):
    """Train the chi networks (and with train_j the J networks) on reference
    charges of a teacher model.  With vary_j (default: train_j) the teacher's
    hardness also varies with the environment, J_i = J_e exp(0.1 z_i), z a
    second fixed random network on the descriptors (unit std on the first
    frame)."""
    import torch

    from inputs import gen

    if vary_j is None:
        vary_j = train_j
    spacing = gen.MD_SPACING
    dev = device or torch.device("cuda", torch.cuda.current_device())
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    pos, cell, species, sigma, J = gen.md_initial(n, side, spacing, seed=1010)
    k = gen.grid_dim(side * spacing, 0.8)
    plan = qeq.Plan(n, eta=2.0, r_cut=11.0, grid=(k, k, k), tol=tol, max_iter=3000)
    chi_w = gen.chi_network_weights(1004)
    sig_d, J_d, sp_d = T(sigma), T(J), T(species, torch.int32)
    frames = []
    scaling = y_std = None
    j_w = gen.chi_network_weights(1014)
    scaling_j = zj_std = None
    for t in range(train_frames + test_frames):
        if t > 0:
            pos = pos + gen.md_displacement(t - 1, n, seed=1010)
        posd = T(gen.wrap_positions(pos, cell))
        G = plan.descriptors(posd, cell, sig_d, CENTERS, WIDTH, RCUT_DESC)
        chi, scaling, y_std = gen.chi_from_descriptors(G.cpu().numpy(), species, chi_w, scaling, y_std)
        Jt = J_d
        if vary_j:
            # chi_from_descriptors returns m_e + 0.05 z / z_std: recover z
            zj, scaling_j, zj_std = gen.chi_from_descriptors(G.cpu().numpy(), species, j_w, scaling_j, zj_std)
            z = (zj - np.asarray(gen.CHI_MEAN_2EL)[species]) / gen.CHI_SD
            Jt = J_d * T(np.exp(0.1 * z))
        q_ref, _, _, st = plan.solve(posd, cell, sig_d, Jt, T(chi), 0.0, forces=False)
        frames.append((posd, G, q_ref))
    train, test = frames[:train_frames], frames[train_frames:]

    # the method without a chi network: one electronegativity per element
    chi_base = T(np.asarray(gen.CHI_MEAN_2EL)[species])

    def rms(qa, qb):
        return float((qa - qb).pow(2).mean().sqrt())

    base = float(np.mean([rms(plan.solve(p, cell, sig_d, J_d, chi_base, 0.0, forces=False)[0], qr)
                          for p, _, qr in test]))
    net = qeq.WarmStartNet(init_networks(), device=dev)
    Gall, spall = torch.cat([g for _, g, _ in train]), sp_d.repeat(train_frames)
    net.fit_scaling(Gall, spall)
    jnet = None
    if train_j:
        jnet = qeq.WarmStartNet(init_networks(seed=1015, chi_means=(0.0, 0.0)), device=dev)
        jnet.fit_scaling(Gall, spall)
    del Gall, spall

    def test_rms():
        errs = []
        for p, g, qr in test:
            Jv = J_d if jnet is None else J_d * (J_SCALE * jnet.predict(g, sp_d)).exp()
            q, _, _, _ = plan.solve(p, cell, sig_d, Jv, net.predict(g, sp_d), 0.0, forces=False)
            errs.append(rms(q, qr))
        return float(np.mean(errs))

    init = test_rms()
    order = np.random.default_rng(1012).permutation
    hist, step_ms = [], []
    for ep in range(epochs):
        losses = []
        for f in order(train_frames):
            p, g, qr = train[f]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            loss, _, _, st, st_b = charge_step(plan, net, g, sp_d, p, cell, sig_d, J_d, qr, lr=lr, jnet=jnet)
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t0) * 1e3)
            losses.append(loss)
        hist.append(float(np.mean(losses)))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: train loss {hist[-1]:.3e}")
    final = test_rms()
    plan.close()
    return {"n": n, "grid": [k, k, k], "train_frames": train_frames, "test_frames": test_frames,
            "train_j": bool(train_j), "vary_j": bool(vary_j),
            "epochs": epochs, "rms_element_means": base, "rms_untrained": init, "rms_trained": final,
            "train_loss_first": hist[0], "train_loss_last": hist[-1],
            "ms_per_step": float(np.median(step_ms))}
