"""Learned warm start on an MD-like trajectory (workflow over the C ABI).

Frames x_{t+1} = x_t + N(0, 0.05 bohr) of the 131,072-atom lattice subset;
chi per frame from a fixed random network on the frame's radial descriptors
(input synthesis, inputs.gen.chi_from_descriptors).  The first half of the
frames is solved cold; their descriptors and solver charges train the
per-element warm-start networks (mlp_train_step, Adam).  On the second half
every frame is solved three times to the same tolerance: cold (q0 = Q/N),
previous-frame start (q0 = charges of frame t-1) and learned start
(q0 = network output; the solve projects it onto sum(q) = Q).  Cold-start CG
stays the reference: all must agree.

Two learned starts are trained and compared: the network on the 16 radial
descriptors of the workload (``learned``), and the same network on 16
electronegativity-aware features (``learned_chi``): chi_i, 8 radial sums of
the neighbours' chi_j (weighted radial descriptors, width 1 bohr, centres
1..9) and 7 plain radial terms (width 1 bohr).  The charges follow the local
electronegativity differences, which the geometry alone does not determine.
"""
from __future__ import annotations

import time

import numpy as np

from . import qeq

CENTERS = np.linspace(1.0, 9.0, 16)
WIDTH, RCUT_DESC = 0.5, 9.0
CHI_CENTERS = np.linspace(1.0, 9.0, 8)
GEO_CENTERS = np.linspace(1.0, 9.0, 7)
AUX_WIDTH = 1.0


def chi_features(plan, posd, cell, sigma, chi):
    """n x 16 float32 features: chi_i | sum_j chi_j g_mu(r_ij) (8) | sum_j g_nu(r_ij) (7).

    posd=None reuses the plan's current geometry (the radial descriptors of
    the same frame have just built it)."""
    import torch
    Gc = plan.descriptors(posd, cell, sigma, CHI_CENTERS, AUX_WIDTH, RCUT_DESC, weights=chi)
    Gg = plan.descriptors(None, cell, sigma, GEO_CENTERS, AUX_WIDTH, RCUT_DESC)
    return torch.cat([chi.float()[:, None], Gc, Gg], 1).contiguous()


PROFILE_KINDS_MESH = 9   # kinds 0..8 of qeq_profile: the mesh passes, interpolation, CG, final pass


def run_trajectory(n=None, side=None, spacing=None, frames=200, epochs=30, lr=2e-3, tol=1e-6,
                   grid=None, log=None, device=None, spectral_kc=0.0, train_frames=None,
                   chi_override=None, keep_frame=None, profile_matvec=False):
    """Run the trajectory workflow and return its record.

    train_frames: frames solved cold for training (default frames // 2).
    chi_override: {frame: chi (numpy, n)} replaces the workload's
    electronegativities of those frames (e.g. values computed elsewhere for a
    parity check); the network inputs still come from the frame's geometry.
    keep_frame: an evaluation frame whose charges, energies and forces of
    every start are returned (numpy) under "kept".
    profile_matvec: after the last frame, one more cold solve of it with every
    launch kind bracketed by HIP events (kernels launched one by one); the
    per-launch microseconds are returned under "stage_us".
    """
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
    # a second plan with the spectral preconditioner (its own captured CG graph)
    plan_s = None
    if spectral_kc > 0.0:
        plan_s = qeq.Plan(n, eta=2.0, r_cut=11.0, grid=grid, tol=tol, max_iter=3000)
        plan_s.use_spectral_preconditioner(spectral_kc)
    net = qeq.WarmStartNet(gen.warmstart_init(1005, 2), device=dev)
    net_x = qeq.WarmStartNet(gen.warmstart_init(1005, 2), device=dev)
    chi_w = gen.chi_network_weights(1004)
    sig_d, J_d, sp_d = T(sigma), T(J), T(species, torch.int32)
    n_train = frames // 2 if train_frames is None else int(train_frames)
    scaling = y_std = None
    train_G, train_X, train_q = [], [], []
    variants = ["cold", "prev", "learned", "learned_chi"]
    if plan_s is not None:
        variants += ["cold_spectral", "prev_spectral", "learned_chi_spectral"]
    rec = {k: [] for k in variants}
    q_prev = None

    kept = {}

    def solve(posd, chid, q0=None, pl=None, keep=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q, en, f, st = (pl or plan).solve(posd, cell, sig_d, J_d, chid, 0.0, q0=q0, forces=keep is not None)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if keep is not None:
            kept[keep] = {"q": q.cpu().numpy(), "energies": en.cpu().numpy(), "forces": f.cpu().numpy(),
                          "iters": st["iters"], "rc": st["rc"], "q0_rejected": st["q0_rejected"]}
        return q, st, ms

    t_desc, t_feat, t_pred, t_pred_x, max_dq = [], [], [], [], 0.0
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
        if chi_override is not None and t in chi_override:
            chi = np.asarray(chi_override[t], dtype=np.float64)
        chid = T(chi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = chi_features(plan, None, cell, sig_d, chid)   # geometry of the descriptor call above
        torch.cuda.synchronize()
        t_feat.append((time.perf_counter() - t0) * 1e3)
        if t < n_train:
            q, st, ms = solve(posd, chid)
            train_G.append(G)
            train_X.append(X)
            train_q.append(q)
            q_prev = q
            if log:
                log(f"frame {t} (train): cold {st['iters']} it {ms:.1f} ms")
            if t == n_train - 1:
                spall = sp_d.repeat(n_train)
                for key, nt_, feats in (("", net, train_G), ("_chi", net_x, train_X)):
                    Gall = torch.cat(feats)
                    nt_.fit_scaling(Gall, spall)
                    del Gall
                    t0 = time.perf_counter()
                    order = np.random.default_rng(1006).permutation
                    for ep in range(epochs):
                        for f in order(n_train):
                            loss = nt_.train_step(feats[f], sp_d, train_q[f], lr=lr)
                        if log and (ep % 5 == 0 or ep == epochs - 1):
                            log(f"net{key} epoch {ep}: loss {float(loss.cpu()):.3e}")
                    torch.cuda.synchronize()
                    rec["train_s" + key] = time.perf_counter() - t0
                    rec["train_loss" + key] = float(loss.cpu())
                rec["train_steps"] = epochs * n_train
                del spall
                if log:
                    log(f"trained {epochs} epochs in {rec['train_s']:.1f} s, loss {rec['train_loss']:.3e}")
            continue
        kf = (lambda name: name) if t == keep_frame else (lambda name: None)
        q_c, st_c, ms_c = solve(posd, chid, keep=kf("cold"))
        q_p, st_p, ms_p = solve(posd, chid, q0=q_prev, keep=kf("prev"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q0 = net.predict(G, sp_d)
        torch.cuda.synchronize()
        t_pred.append((time.perf_counter() - t0) * 1e3)
        q_l, st_l, ms_l = solve(posd, chid, q0=q0, keep=kf("learned"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q0x = net_x.predict(X, sp_d)
        torch.cuda.synchronize()
        t_pred_x.append((time.perf_counter() - t0) * 1e3)
        q_x, st_x, ms_x = solve(posd, chid, q0=q0x, keep=kf("learned_chi"))
        dq_p, dq_l = float((q_p - q_c).abs().max()), float((q_l - q_c).abs().max())
        dq_x = float((q_x - q_c).abs().max())
        max_dq = max(max_dq, dq_p, dq_l, dq_x)
        runs = [("cold", st_c, ms_c), ("prev", st_p, ms_p), ("learned", st_l, ms_l),
                ("learned_chi", st_x, ms_x)]
        if plan_s is not None:
            for k, q0s in (("cold_spectral", None), ("prev_spectral", q_prev), ("learned_chi_spectral", q0x)):
                q_s, st_s, ms_s = solve(posd, chid, q0=q0s, pl=plan_s, keep=kf(k))
                max_dq = max(max_dq, float((q_s - q_c).abs().max()))
                runs.append((k, st_s, ms_s))
        for k, st, ms in runs:
            rec[k].append((st["iters"], ms, st["rc"], st["q0_rejected"]))
        q_prev = q_c
        if log:
            log(f"frame {t}: iters " + " ".join(f"{k} {st['iters']}" for k, st, _ in runs) +
                "; ms " + " / ".join(f"{ms:.1f}" for _, _, ms in runs) + "; "
                f"max|dq| {max_dq:.1e}; rms |q0 - q| learned "
                f"{float((q0 - q_c).pow(2).mean().sqrt()):.2e} learned_chi "
                f"{float((q0x - q_c).pow(2).mean().sqrt()):.2e}")
    stage = None
    if profile_matvec:
        plan.profile((1 << PROFILE_KINDS_MESH) - 1)
        plan.profile_read(reset=True)
        for _ in range(2):
            plan.solve(posd, cell, sig_d, J_d, chid, 0.0, forces=False)
        d = plan.profile_read(reset=True)
        plan.profile(0)
        stage = {k: (ms * 1e3 / c if c else 0.0, int(c)) for k, (ms, c) in d.items()}
    plan.close()
    if plan_s is not None:
        plan_s.close()
    out = {"n": n, "grid": list(grid), "frames": frames, "train_frames": n_train,
           "max_dq_vs_cold": max_dq, "descriptor_ms": float(np.mean(t_desc)),
           "chi_feature_ms": float(np.mean(t_feat)),
           "predict_ms": float(np.mean(t_pred)) if t_pred else None,
           "predict_chi_ms": float(np.mean(t_pred_x)) if t_pred_x else None,
           "train_s": rec.get("train_s"), "train_loss": rec.get("train_loss"),
           "train_s_chi": rec.get("train_s_chi"), "train_loss_chi": rec.get("train_loss_chi"),
           "train_steps": rec.get("train_steps")}
    if plan_s is not None:
        out["spectral_kc"] = spectral_kc
    if stage is not None:
        out["stage_us"] = stage
    if kept:
        out["kept"] = kept
        out["kept_frame"] = keep_frame
    for k in variants:
        a = np.array(rec[k], dtype=float)
        out[k] = {"iters": float(a[:, 0].mean()), "ms": float(a[:, 1].mean()),
                  "all_converged": bool((a[:, 2] == 0).all()), "q0_rejected": int(a[:, 3].sum())}
    # inference charged to the learned starts: the network, plus for the
    # chi-aware start the two feature calls that the workload's own
    # descriptors (needed for chi anyway) do not provide
    out["learned"]["ms_with_inference"] = out["learned"]["ms"] + (out["predict_ms"] or 0.0)
    for k in ("learned_chi", "learned_chi_spectral"):
        if k in out:
            out[k]["ms_with_inference"] = out[k]["ms"] + out["chi_feature_ms"] + (out["predict_chi_ms"] or 0.0)
    return out
