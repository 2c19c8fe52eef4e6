"""Autotuner of the batched solve: spline order, grid spacing and launch shape.

The batched workload (many small structures, each on its own grid, one
persistent launch) trades mesh work against accuracy: a higher spline order
reaches the same accuracy on a coarser grid (fewer FFT points, more spline
points per atom).  The tuner measures instead of modelling:

1. A reference solve of the whole batch at the most accurate setting every
   structure admits (order 8 at the configs' 0.8-bohr spacing, tight CG
   tolerance; its agreement with the FP64 oracle is covered by the tests).
2. For every candidate (order p, maximum spacing h): one solve at the
   working tolerance, compared with the reference per structure: charges
   (max |dq|), energies (relative E_QEq and E_elec) and forces (relative RMS).
   Candidates over the parity bars (1e-5 e, 1e-6, 1e-4), or with structures
   the grid limits refuse, are discarded.
3. Every surviving candidate is timed with each launch shape (workgroups per
   compute unit); the fastest (p, h, shape) wins.

Everything runs through the C ABI (qeq_solve_batched, qeq_batched_config);
the tuner itself is host-side bookkeeping.
"""
from __future__ import annotations

import time

import numpy as np

from . import qeq

# (spline order, maximum grid spacing in bohr)
CANDIDATES = ((6, 0.8), (6, 0.9), (6, 1.0), (8, 0.9), (8, 1.0), (8, 1.1), (8, 1.2), (4, 0.6), (4, 0.7))
WG_PER_CU = (1, 2)
REFERENCE = (8, 0.8)


def _errors(q, en, f, ref, offs):
    """Worst per-structure errors against the reference solve."""
    q_ref, en_ref, f_ref = ref
    dq = float(np.abs(q - q_ref).max())
    scale = np.maximum(np.abs(en_ref), 1e-3 * np.median(np.abs(en_ref)))
    de = float((np.abs(en - en_ref) / scale).max())
    df = 0.0
    for k in range(len(offs) - 1):
        sl = slice(offs[k], offs[k + 1])
        r = np.sqrt(np.mean(f_ref[sl] ** 2))
        if r > 0:
            df = max(df, float(np.sqrt(np.mean((f[sl] - f_ref[sl]) ** 2)) / r))
    return dq, de, df


def tune_batched(args, n_max=512, eta=2.0, r_cut=12.0, tol=1e-6, tol_q=1e-5, tol_e=1e-6, tol_f=1e-4,
                 candidates=CANDIDATES, wg_per_cu=WG_PER_CU, reps=3, log=None):
    """Choose (spline order, spacing, workgroups per CU) for a batch.

    args: the keyword arguments of Plan.solve_batched (device arrays, host
    offsets / cells / q_tot).  Returns a dict with the chosen setting
    ("best"), the reference's status and one row per candidate.
    """
    import torch

    offs = np.asarray(args["offsets"])
    p_ref, h_ref = REFERENCE
    plan = qeq.Plan(n_max, eta=eta, r_cut=r_cut, max_spacing=h_ref, spline_order=p_ref, tol=min(tol, 1e-9),
                    max_iter=4000)
    q, en, f, st, rc = plan.solve_batched(**args)
    plan.close()
    if rc != 0:
        raise qeq.QEqError(rc, "reference solve of the batch failed")
    ref = (q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy())
    rows = []
    for p, h in candidates:
        row = {"spline_order": p, "max_spacing": h}
        plan = qeq.Plan(n_max, eta=eta, r_cut=r_cut, max_spacing=h, spline_order=p, tol=tol, max_iter=4000)
        q, en, f, st, rc = plan.solve_batched(check=False, **args)
        row["rc"] = int(rc)
        if rc == 0:
            dq, de, df = _errors(q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), ref, offs)
            row.update(max_dq=dq, max_rel_dE=de, max_rel_dF=df)
            row["accurate"] = dq <= tol_q and de <= tol_e and df <= tol_f
            if row["accurate"]:
                for wg in wg_per_cu:
                    plan.batched_config(1024, wg)
                    plan.solve_batched(**args)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        plan.solve_batched(**args)
                    torch.cuda.synchronize()
                    row[f"ms_wg{wg}"] = (time.perf_counter() - t0) * 1e3 / reps
        else:
            row["accurate"] = False
        plan.close()
        rows.append(row)
        if log:
            log(f"autotune p={p} h={h}: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}"
                                                     for k, v in row.items() if k not in ("spline_order",
                                                                                          "max_spacing")))
    best = None
    for row in rows:
        for wg in wg_per_cu:
            ms = row.get(f"ms_wg{wg}")
            if ms is not None and (best is None or ms < best["ms"]):
                best = {"spline_order": row["spline_order"], "max_spacing": row["max_spacing"], "wg_per_cu": wg,
                        "ms": ms, "max_dq": row["max_dq"], "max_rel_dE": row["max_rel_dE"],
                        "max_rel_dF": row["max_rel_dF"]}
    return {"best": best, "reference": {"spline_order": p_ref, "max_spacing": h_ref}, "candidates": rows,
            "tolerances": {"q": tol_q, "E": tol_e, "F": tol_f}}
