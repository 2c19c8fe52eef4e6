"""Autotuner of the batched solve: its choice meets the parity bars against
the tuner's reference and, re-verified, against the FP64 oracle on sampled
structures; candidates that miss the bars or that the grid limits refuse are
never chosen."""
import numpy as np
import pytest

from inputs import gen
from oracle import ewald

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def pack(structs, dev):
    offs = np.concatenate([[0], np.cumsum([s.n for s in structs])]).astype(np.int32)
    cat = lambda f: np.concatenate([getattr(s, f) for s in structs])
    return dict(pos=T(cat("pos"), dev), offsets=offs, cells=np.stack([s.cell for s in structs]),
                sigma=T(cat("sigma"), dev), J=T(cat("J"), dev), chi=T(cat("chi"), dev),
                q_tot=np.array([s.q_tot for s in structs]))


def test_autotune_choice_meets_oracle(dev):
    from paper_2607_17978_amd import autotune, qeq
    structs = [gen.batch_structure(s) for s in range(48)]
    args = pack(structs, dev)
    refs = {}
    for k in (5, 23, 31):
        s = structs[k]
        r = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
        refs[k] = {"q": r.q, "e_qeq": r.e_qeq, "e_elec": r.e_elec, "forces": r.forces}
    out = autotune.tune_batched(args, reps=2, log=print, references=refs)
    best = out["best"]
    print("best", best)
    assert best is not None
    assert out["sampled_references"] == [5, 23, 31]
    for row in out["candidates"]:
        if row["accurate"]:
            assert row["max_dq"] <= 1e-5 and row["max_rel_dE"] <= 1e-6 and row["max_rel_dF"] <= 1e-4
            assert row["sample_max_dq"] <= 1e-5 and row["sample_max_rel_dE"] <= 1e-6
            assert row["sample_max_rel_dF"] <= 1e-4
    # the configs' own setting (order 6, spacing 0.8) is accurate enough to be a candidate
    assert any(r["accurate"] for r in out["candidates"] if (r["spline_order"], r["max_spacing"]) == (6, 0.8))
    # re-verify the choice against the oracle on sampled members
    plan = qeq.Plan(512, eta=2.0, r_cut=12.0, max_spacing=best["max_spacing"], spline_order=best["spline_order"],
                    tol=1e-8)
    plan.batched_config(1024, best["wg_per_cu"])
    q, en, f, st, rc = plan.solve_batched(**args)
    assert rc == 0
    q, en, f = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
    offs = args["offsets"]
    for k in (0, 17, 40):
        s = structs[k]
        ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
        sl = slice(offs[k], offs[k + 1])
        dq = np.abs(q[sl] - ref.q).max()
        de = np.abs(en[k] - np.array([ref.e_qeq, ref.e_elec])).max() / abs(ref.e_qeq)
        df = np.sqrt(np.mean((f[sl] - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
        print("member", k, "n", s.n, "dq", dq, "dE", de, "dF", df)
        assert dq <= 1e-5 and de <= 1e-6 and df <= 1e-4
    plan.close()


def test_tile_tuner_meets_oracle_and_caches(dev, tmp_path):
    """Single-structure mesh tiles: every timed candidate reproduces the
    built-in rule's charges and meets the bars against the FP64 oracle; the
    choice is the fastest timed one, lands in the JSON cache and is served
    from it on the next call; an impossible tile choice is refused."""
    from oracle import matfree
    from paper_2607_17978_amd import autotune, qeq
    s = gen.system_4096()
    r = matfree.qeq_matfree(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot, tol=1e-10, forces=True)
    ref = {"q": r.q, "e_qeq": r.e_qeq, "e_elec": r.e_elec, "forces": r.forces}
    path = str(tmp_path / "autotune.json")
    out = autotune.tune_tiles(s, dev, reference=ref, path=path, reps=2, log=print, tol=1e-7)
    assert not out["cached"] and out["timed"] >= 2
    timed = [row for row in out["rows"] if "ms" in row]
    for row in timed:
        assert row["accurate"] and row["dq_vs_rule"] <= 1e-7 and row["ref_dq"] <= 1e-5
        assert row["ref_dE"] <= 1e-6 and row["ref_dF"] <= 1e-4
    assert out["ms"] == min(row["ms"] for row in timed)
    again = autotune.tune_tiles(s, dev, reference=ref, path=path)
    assert again["cached"] and again["tiles"] == out["tiles"]
    assert autotune.cached_tiles(s.grid, 6, s.n, path=path) == tuple(out["tiles"])
    plan = qeq.Plan(s.n, eta=2.0, r_cut=11.0, grid=s.grid)
    plan.set_tiles(32, 0, 0)                          # 32 spread rows: fits 96 rows, allowed
    with pytest.raises(qeq.QEqError):
        plan.set_tiles(10, 0, 0)                          # neither a power of two nor 12 / 24
    solve_args = (T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    plan.set_tiles(12, 0, 0)                          # accepted, but 96 has no compiled 12-row spread
    q, _, _, st = plan.solve(*solve_args, check=False)
    assert st["rc"] == qeq.QEQ_EPLAN
    plan.set_tiles(0, 0, 32)
    q, _, _, st = plan.solve(*solve_args, check=False)
    assert st["rc"] == 0
    plan.close()
