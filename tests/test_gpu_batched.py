"""Batched persistent solve (many structures, one launch) on the GPU.

* parity of several triclinic, charged structures with the FP64 oracle;
* equality with the single-structure GPU solve of each structure, and with
  the same batch split over two calls;
* launch shapes (threads per workgroup, LDS staging size) agree;
* per-structure failures are reported per structure;
* the full 1,024-structure workload in the launch shape the benchmark uses,
  with sampled structures against stored oracle solutions
  (tests/golden/make_batch_reference.py).
"""
import os

import numpy as np
import pytest

from inputs import gen
from oracle import ewald

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ETA, RC = 2.0, 12.0    # sigma up to 1.7 bohr: a 12-bohr cutoff keeps the real-space tail below 1e-7


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def T(a, dev, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def pack(structs, dev):
    offs = np.concatenate([[0], np.cumsum([s.n for s in structs])]).astype(np.int32)
    cat = lambda f: np.concatenate([getattr(s, f) for s in structs])
    return dict(pos=T(cat("pos"), dev), offsets=offs, cells=np.stack([s.cell for s in structs]),
                sigma=T(cat("sigma"), dev), J=T(cat("J"), dev), chi=T(cat("chi"), dev),
                q_tot=np.array([s.q_tot for s in structs]))


def test_batched_matches_oracle(dev):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(s) for s in (3, 17, 40, 5)]
    a = pack(structs, dev)
    plan = qeq.Plan(64, eta=ETA, r_cut=RC, tol=1e-8)
    q, en, f, st, rc = plan.solve_batched(**a)
    assert rc == 0, st
    q, en, f = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
    for k, s in enumerate(structs):
        lo, hi = a["offsets"][k], a["offsets"][k + 1]
        ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
        dq = np.abs(q[lo:hi] - ref.q).max()
        de_q = abs(en[k, 0] - ref.e_qeq) / abs(ref.e_qeq)
        de_e = abs(en[k, 1] - ref.e_elec) / abs(ref.e_elec)
        df = np.sqrt(np.mean((f[lo:hi] - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
        print(s.name, s.n, s.grid, s.q_tot, st[k], "dq", dq, "dEqeq", de_q, "dEelec", de_e, "dF", df)
        assert st[k]["status"] == 0
        assert abs(q[lo:hi].sum() - s.q_tot) < 1e-10
        assert dq <= 1e-5
        assert de_q <= 1e-6 and de_e <= 1e-6
        assert df <= 1e-4
        assert abs(st[k]["mu"] - ref.mu) <= 1e-5
    plan.close()


def test_batched_equals_single_and_split(dev):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(s) for s in range(24)]
    a = pack(structs, dev)
    plan = qeq.Plan(512, eta=ETA, r_cut=RC, tol=1e-8)
    q, en, f, st, rc = plan.solve_batched(**a)
    assert rc == 0
    q, en, f = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
    for k, s in enumerate(structs):
        lo, hi = a["offsets"][k], a["offsets"][k + 1]
        single = qeq.Plan(s.n, eta=ETA, r_cut=RC, grid=s.grid, tol=1e-8)
        q1, e1, f1, s1 = single.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        single.close()
        dq = np.abs(q[lo:hi] - q1.cpu().numpy()).max()
        de = np.abs(en[k] - e1.cpu().numpy()).max() / abs(e1[0].item())
        df = np.abs(f[lo:hi] - f1.cpu().numpy()).max() / np.abs(f1.cpu().numpy()).max()
        assert st[k]["status"] == 0 and s1["rc"] == 0
        assert dq < 1e-6 and de < 1e-7 and df < 1e-5, (k, dq, de, df)
    # the same structures over two calls
    h = 11
    b1 = pack(structs[:h], dev)
    b2 = pack(structs[h:], dev)
    qa = plan.solve_batched(**b1)[0].cpu().numpy()
    qb = plan.solve_batched(**b2)[0].cpu().numpy()
    assert np.abs(np.concatenate([qa, qb]) - q).max() < 1e-6
    plan.close()


@pytest.mark.parametrize("shape", [
    pytest.param((256, 2), marks=pytest.mark.skip(
        reason="256-thread workgroups are disabled: a run of this shape ended in a GPU fault whose cause "
               "has not been found (the host replay of every thread-count-dependent index, "
               "tests/test_batched_index_replay.py, and a reading of the barriers after early exits found "
               "none); qeq_batched_config rejects 256")),
    pytest.param((512, 1), marks=pytest.mark.skip(
        reason="512-thread workgroups are disabled: with the fixed-point spread they returned "
               "NOT_CONVERGED on structures the 1024-thread shape solves; cause not found (index replay "
               "and barrier reading clean); qeq_batched_config rejects 512")),
    (1024, 1), (1024, 2)])
def test_batched_launch_shapes_agree(dev, shape):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(s) for s in range(8)]
    a = pack(structs, dev)
    plan = qeq.Plan(512, eta=ETA, r_cut=RC, tol=1e-8)
    q0 = plan.solve_batched(**a)[0].cpu().numpy()
    plan.batched_config(*shape)
    q1, _, _, st, rc = plan.solve_batched(**a)
    assert rc == 0
    assert np.abs(q1.cpu().numpy() - q0).max() < 1e-6
    plan.close()


def test_batched_config_rejects_disabled_shapes(dev):
    """Host-side check only: the disabled 256-thread shape is refused before any launch."""
    from paper_2607_17978_amd import qeq
    plan = qeq.Plan(64, eta=ETA, r_cut=RC)
    for shape in ((256, 1), (256, 2), (128, 1), (512, 1), (1024, 0), (1024, 9)):
        with pytest.raises(qeq.QEqError):
            plan.batched_config(*shape)
    plan.batched_config(1024, 2)
    plan.close()


def test_batched_per_structure_errors(dev):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(s) for s in range(4)]
    bad = structs[1]
    bad.J = bad.J.copy()
    bad.J[3] = -1.0
    a = pack(structs, dev)
    cells = a["cells"].copy()
    cells[2] = 0.0                       # singular cell
    a["cells"] = cells
    plan = qeq.Plan(512, eta=ETA, r_cut=RC, tol=1e-8)
    q, en, f, st, rc = plan.solve_batched(**a)
    assert rc == qeq.QEQ_EINVAL
    assert [x["status"] for x in st] == [0, qeq.QEQ_EINVAL, qeq.QEQ_EINVAL, 0]
    # the good structures match a batch without the bad ones
    a2 = pack([structs[0], structs[3]], dev)
    q2 = plan.solve_batched(**a2)[0].cpu().numpy()
    o = a["offsets"]
    qn = q.cpu().numpy()
    assert np.abs(np.concatenate([qn[o[0]:o[1]], qn[o[3]:o[4]]]) - q2).max() < 1e-6
    # max_iter reached: status NOT_CONVERGED with valid stats
    p1 = qeq.Plan(512, eta=ETA, r_cut=RC, tol=1e-8, max_iter=2)
    _, _, _, st1, rc1 = p1.solve_batched(**a2)
    assert rc1 == qeq.QEQ_NOT_CONVERGED
    assert all(x["status"] == qeq.QEQ_NOT_CONVERGED and x["iters"] == 2 for x in st1)
    p1.close()
    plan.close()


def test_full_batch_1024_matches_oracle_samples(dev):
    """The 1,024-structure workload in the benchmark's launch shape: every
    structure converges, charges sum to Q_tot, and sampled structures match the
    stored FP64 oracle solutions."""
    from paper_2607_17978_amd import qeq
    path = os.path.join(os.path.dirname(__file__), "golden", "batch1024_samples.npz")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    ref = np.load(path)
    structs = gen.batch(1024)
    a = pack(structs, dev)
    plan = qeq.Plan(512, eta=ETA, r_cut=RC, tol=1e-6)
    q, en, f, st, rc = plan.solve_batched(**a)
    assert rc == 0
    q, en, f = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
    o = a["offsets"]
    for k, s in enumerate(structs):
        assert abs(q[o[k]:o[k + 1]].sum() - s.q_tot) < 1e-9
    assert max(x["true_rel_resid"] for x in st) <= 2e-6
    for k in ref["index"]:
        k = int(k)
        lo, hi = o[k], o[k + 1]
        rq, re, rf = ref[f"q{k}"], ref[f"e{k}"], ref[f"f{k}"]
        dq = np.abs(q[lo:hi] - rq).max()
        de = np.abs(en[k] - re).max() / abs(re[0])
        df = np.sqrt(np.mean((f[lo:hi] - rf) ** 2)) / np.sqrt(np.mean(rf ** 2))
        print("batch", k, structs[k].n, "dq", dq, "dE", de, "dF", df)
        assert dq <= 1e-5 and de <= 1e-6 and df <= 1e-4
    plan.close()
