"""Learned warm start on an MD-like trajectory (workflow over the C ABI).

Frames x_{t+1} = x_t + N(0, 0.05 bohr) of the 131,072-atom lattice subset;
chi per frame from a fixed random network on the frame's radial descriptors
(input synthesis, inputs.gen.chi_from_descriptors).  The first half of the
frames is solved cold; their descriptors and solver charges train the
per-element warm-start networks (mlp_train_step, Adam).  On the second half
every frame is solved three times to the same tolerance: cold (q0 = Q/N),
previous-frame start (q0 = charges of frame t-1) and learned start
(q0 = network output; the solve projects it onto sum(q) = Q).  Cold-start CG
stays the reference: all three must agree.
"""
from __future__ import annotations

import time

import numpy as np

from . import qeq

CENTERS = np.linspace(1.0, 9.0, 16)
WIDTH, RCUT_DESC = 0.5, 9.0


def run_trajectory(n=None, side=None, spacing=None, frames=200, epochs=30, lr=2e-3, tol=1e-6,
                   grid=None, log=None, device=None):
    import torch

    from inputs import gen

    n = n or gen.MD_N
    side = side or gen.MD_SIDE
    spacing = spacing or gen.MD_SPACING
    dev = device or torch.device("cuda", torch.cuda.current_device())
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    pos, cell, species, sigma, J = gen.md_initial(n, side, spacing)
    L = side * spacing
    if grid is None:
        # the 131,072-atom workload is specified on a 320^3 grid (spacing 0.74)
        k = 320 if n == gen.MD_N else gen.grid_dim(L, 0.8)
        grid = (k, k, k)
    plan = qeq.Plan(n, eta=2.0, r_cut=11.0, grid=grid, tol=tol, max_iter=3000)
    net = qeq.WarmStartNet(gen.warmstart_init(1005, 2), device=dev)
    chi_w = gen.chi_network_weights(1004)
    sig_d, J_d, sp_d = T(sigma), T(J), T(species, torch.int32)
    n_train = frames // 2
    scaling = y_std = None
    train_G, train_q = [], []
    rec = {"cold": [], "prev": [], "learned": []}
    q_prev = None

    def solve(posd, chid, q0=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q, en, _, st = plan.solve(posd, cell, sig_d, J_d, chid, 0.0, q0=q0, forces=False)
        torch.cuda.synchronize()
        return q, st, (time.perf_counter() - t0) * 1e3

    t_desc, t_pred, max_dq = [], [], 0.0
    for t in range(frames):
        if t > 0:
            pos = pos + gen.md_displacement(t - 1, n)
        posd = T(gen.wrap_positions(pos, cell))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = plan.descriptors(posd, cell, sig_d, CENTERS, WIDTH, RCUT_DESC)
        torch.cuda.synchronize()
        t_desc.append((time.perf_counter() - t0) * 1e3)
        chi, scaling, y_std = gen.chi_from_descriptors(G.cpu().numpy(), species, chi_w, scaling, y_std)
        chid = T(chi)
        if t < n_train:
            q, st, ms = solve(posd, chid)
            train_G.append(G)
            train_q.append(q)
            q_prev = q
            if log:
                log(f"frame {t} (train): cold {st['iters']} it {ms:.1f} ms")
            if t == n_train - 1:
                Gall = torch.cat(train_G)
                spall = sp_d.repeat(n_train)
                net.fit_scaling(Gall, spall)
                t0 = time.perf_counter()
                order = np.random.default_rng(1006).permutation
                for ep in range(epochs):
                    for f in order(n_train):
                        loss = net.train_step(train_G[f], sp_d, train_q[f], lr=lr)
                    if log and (ep % 5 == 0 or ep == epochs - 1):
                        log(f"epoch {ep}: loss {float(loss.cpu()):.3e}")
                torch.cuda.synchronize()
                rec["train_s"] = time.perf_counter() - t0
                rec["train_loss"] = float(loss.cpu())
                rec["train_steps"] = epochs * n_train
                del Gall, spall
                if log:
                    log(f"trained {epochs} epochs in {rec['train_s']:.1f} s, loss {rec['train_loss']:.3e}")
            continue
        q_c, st_c, ms_c = solve(posd, chid)
        q_p, st_p, ms_p = solve(posd, chid, q0=q_prev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q0 = net.predict(G, sp_d)
        torch.cuda.synchronize()
        t_pred.append((time.perf_counter() - t0) * 1e3)
        q_l, st_l, ms_l = solve(posd, chid, q0=q0)
        dq_p, dq_l = float((q_p - q_c).abs().max()), float((q_l - q_c).abs().max())
        max_dq = max(max_dq, dq_p, dq_l)
        for k, st, ms in (("cold", st_c, ms_c), ("prev", st_p, ms_p), ("learned", st_l, ms_l)):
            rec[k].append((st["iters"], ms, st["rc"], st["q0_rejected"]))
        q_prev = q_c
        if log:
            log(f"frame {t}: iters cold {st_c['iters']} prev {st_p['iters']} learned {st_l['iters']}; "
                f"ms {ms_c:.1f} / {ms_p:.1f} / {ms_l:.1f}; max|dq| prev {dq_p:.1e} learned {dq_l:.1e}; "
                f"|q0 - q| learned max {float((q0 - q_c).abs().max()):.2e} "
                f"rms {float((q0 - q_c).pow(2).mean().sqrt()):.2e}")
    plan.close()
    out = {"n": n, "grid": list(grid), "frames": frames, "train_frames": n_train,
           "max_dq_vs_cold": max_dq, "descriptor_ms": float(np.mean(t_desc)),
           "predict_ms": float(np.mean(t_pred)) if t_pred else None,
           "train_s": rec.get("train_s"), "train_loss": rec.get("train_loss"),
           "train_steps": rec.get("train_steps")}
    for k in ("cold", "prev", "learned"):
        a = np.array(rec[k], dtype=float)
        out[k] = {"iters": float(a[:, 0].mean()), "ms": float(a[:, 1].mean()),
                  "all_converged": bool((a[:, 2] == 0).all()), "q0_rejected": int(a[:, 3].sum())}
    return out
