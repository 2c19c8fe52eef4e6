"""Autotuners: the batched solve's spline order, grid spacing and launch
shape, and the single-structure solve's mesh tile widths.

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
   With ``references`` (solutions of sampled structures computed elsewhere,
   e.g. the FP64 oracle's stored solutions), a candidate must also meet the
   bars against every one of them: the absolute check on samples, beside the
   consistency check on the whole batch.
3. Every surviving candidate is timed with each launch shape (workgroups per
   compute unit); the fastest (p, h, shape) wins.

Single structure (``tune_tiles``): the axis-2 row tiles of the spread, the
axis-1 / complex-to-real passes and the axis-2 pass (qeq_set_tiles) change
only the blocking, so every candidate must reproduce the charges of the
built-in rule to FP32 rounding (and, with a reference solution, meet the
parity bars against it); the fastest measured one wins.  Choices are cached
per (grid, spline order, atom-count bucket) in a JSON file
(``cache_path()``), so later plans of the same shape skip the search.

Everything runs through the C ABI (qeq_solve_batched, qeq_batched_config,
qeq_solve, qeq_set_tiles); the tuners are host-side bookkeeping.
"""
from __future__ import annotations

import json
import math
import os
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


def _sample_errors(q, en, f, references, offs):
    """Worst errors on the sampled structures against their reference solutions."""
    dq = de = df = 0.0
    for k, r in references.items():
        sl = slice(offs[k], offs[k + 1])
        dq = max(dq, float(np.abs(q[sl] - r["q"]).max()))
        e = np.array([r["e_qeq"], r["e_elec"]])
        de = max(de, float((np.abs(en[k] - e) / np.abs(e)).max()))
        F = np.asarray(r["forces"])
        df = max(df, float(np.sqrt(np.mean((f[sl] - F) ** 2)) / np.sqrt(np.mean(F ** 2))))
    return dq, de, df


def tune_batched(args, n_max=512, eta=2.0, r_cut=12.0, tol=1e-6, tol_q=1e-5, tol_e=1e-6, tol_f=1e-4,
                 candidates=CANDIDATES, wg_per_cu=WG_PER_CU, reps=3, log=None, references=None):
    """Choose (spline order, spacing, workgroups per CU) for a batch.

    args: the keyword arguments of Plan.solve_batched (device arrays, host
    offsets / cells / q_tot).  references: optional {structure index:
    {"q", "e_qeq", "e_elec", "forces"}} solutions to gate every candidate on.
    Returns a dict with the chosen setting ("best"), the reference's status
    and one row per candidate.
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
            qh, enh, fh = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
            dq, de, df = _errors(qh, enh, fh, ref, offs)
            row.update(max_dq=dq, max_rel_dE=de, max_rel_dF=df)
            row["accurate"] = dq <= tol_q and de <= tol_e and df <= tol_f
            if references:
                sq, se, sf = _sample_errors(qh, enh, fh, references, offs)
                row.update(sample_max_dq=sq, sample_max_rel_dE=se, sample_max_rel_dF=sf)
                row["accurate"] = row["accurate"] and sq <= tol_q and se <= tol_e and sf <= tol_f
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
            "tolerances": {"q": tol_q, "E": tol_e, "F": tol_f},
            "sampled_references": sorted(int(k) for k in references) if references else []}


# ------------------------------------------------------------------ single-structure tiles
# (spread rows, axis-1 / complex-to-real tile rows, axis-2 rows); 0 = the built-in rule
TILE_ROWS = (8, 16, 32)
SPREAD_ROWS = (8, 12, 16, 24, 32)
FFT_ROWS = (4, 8, 16)


def cache_path():
    """JSON file of tuned choices: $QEQ_AUTOTUNE_CACHE, else under the user's cache directory."""
    p = os.environ.get("QEQ_AUTOTUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2607_17978_amd", "autotune.json")


def tile_key(grid, spline_order, n):
    """Cache key: grid, spline order and the atom count rounded to a power of two."""
    return f"tiles/{grid[0]}x{grid[1]}x{grid[2]}/p{spline_order}/n2^{int(round(math.log2(max(n, 1))))}"


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path, key, value):
    d = _load_cache(path)
    d[key] = value
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_tiles(grid, spline_order, n, path=None):
    """The cached tile choice (spread, tile, fft rows) for this shape, or None."""
    v = _load_cache(path or cache_path()).get(tile_key(grid, spline_order, n))
    return tuple(v["tiles"]) if v else None


def tune_tiles(system, dev, eta=2.0, r_cut=11.0, spline_order=6, tol=1e-6, reps=3, reference=None,
               tol_q=1e-5, tol_e=1e-6, tol_f=1e-4, use_cache=True, path=None, log=None):
    """Measure the mesh tile widths for one structure's solve and pick the fastest.

    system: an object with pos, cell, sigma, J, chi, q_tot, grid (numpy).
    reference: optional {"q", "e_qeq", "e_elec", "forces"} solution (e.g. the
    oracle's stored one) that every candidate must match to the parity bars.
    Every candidate must also reproduce the built-in rule's charges to 1e-7 e
    (the tiles change the blocking only).  Returns {"tiles", "ms", "rows", ...};
    the choice is stored in the cache (and read from it when use_cache).
    """
    import torch
    path = path or cache_path()
    key = tile_key(system.grid, spline_order, len(system.pos))
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            return dict(hit, cached=True)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    args = (T(system.pos), system.cell, T(system.sigma), T(system.J), T(system.chi), system.q_tot)
    n = len(system.pos)
    cands = [(0, 0, 0)] + [(a, b, c) for a in SPREAD_ROWS for b in TILE_ROWS for c in FFT_ROWS]
    rows, base_q = [], None
    for tiles in cands:
        row = {"tiles": list(tiles)}
        plan = qeq.Plan(n, eta=eta, r_cut=r_cut, grid=system.grid, spline_order=spline_order, tol=tol,
                        max_iter=4000)
        try:
            plan.set_tiles(*tiles)
            q, en, f, st = plan.solve(*args, check=False)
            row["rc"] = int(st["rc"])
            if st["rc"] != 0:
                rows.append(row)
                continue
            qh = q.cpu().numpy()
            if base_q is None:
                base_q = qh
            row["dq_vs_rule"] = float(np.abs(qh - base_q).max())
            ok = row["dq_vs_rule"] <= 1e-7
            if reference is not None:
                enh, fh = en.cpu().numpy(), f.cpu().numpy()
                F = np.asarray(reference["forces"], dtype=np.float64)
                row["ref_dq"] = float(np.abs(qh - reference["q"]).max())
                row["ref_dE"] = max(abs(enh[0] - float(reference["e_qeq"])) / abs(float(reference["e_qeq"])),
                                    abs(enh[1] - float(reference["e_elec"])) / abs(float(reference["e_elec"])))
                row["ref_dF"] = float(np.sqrt(np.mean((fh - F) ** 2)) / np.sqrt(np.mean(F ** 2)))
                ok = ok and row["ref_dq"] <= tol_q and row["ref_dE"] <= tol_e and row["ref_dF"] <= tol_f
            row["accurate"] = bool(ok)
            if ok:
                plan.solve(*args, forces=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    plan.solve(*args, forces=True)
                torch.cuda.synchronize()
                row["ms"] = (time.perf_counter() - t0) * 1e3 / reps
        finally:
            plan.close()
        rows.append(row)
        if log:
            log(f"tiles {tiles}: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}"
                                               for k, v in row.items() if k != "tiles"))
    timed = [r for r in rows if "ms" in r]
    if not timed:
        raise qeq.QEqError(qeq.QEQ_EPLAN, "no tile candidate solved this structure")
    best = min(timed, key=lambda r: r["ms"])
    rule = rows[0].get("ms")
    out = {"key": key, "tiles": best["tiles"], "ms": best["ms"], "rule_ms": rule, "candidates": len(rows),
           "timed": len(timed)}
    _store_cache(path, key, out)
    return dict(out, rows=rows, cached=False)
