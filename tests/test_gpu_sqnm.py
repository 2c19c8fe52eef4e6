"""SQNM solver (qeq_use_sqnm) on the GPU against the FP64 oracle.

The QEq energy has a unique minimiser on the constraint plane, so SQNM and
CG must return the oracle's charges within the parity bars; the iteration
counts are reported beside CG's (SQNM is the paper's alternative solver, not
a faster one for this quadratic problem).  The oracle's own SQNM
(oracle.sqnm, pinned in test_oracle_sqnm.py) gives the expected iteration
count on the small cells.
"""
import os

import numpy as np
import pytest

from inputs import gen
from oracle import ewald, sqnm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ETA = 2.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def errs(q, en, f, ref):
    dq = np.abs(q - ref.q).max()
    de_q = abs(en[0] - ref.e_qeq) / abs(ref.e_qeq)
    de_e = abs(en[1] - ref.e_elec) / abs(ref.e_elec)
    df = np.sqrt(np.mean((f - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
    return dq, de_q, de_e, df


def solve(dev, s, solver, rc=11.0, tol=1e-9, op="mesh", history=10):
    from paper_2607_17978_amd import qeq
    plan = qeq.Plan(s.n, eta=ETA, r_cut=rc, grid=s.grid, tol=tol, max_iter=3000)
    plan.use_sqnm(solver == "sqnm", history)
    if op == "ewald":
        plan.use_ewald(True)
    elif op == "planewave":
        plan.use_planewave(True)
    q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    plan.close()
    assert st["rc"] == 0, st
    return q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), st


@pytest.mark.parametrize("which", ["n64", "batch17", "batch40", "n512"])
def test_sqnm_matches_oracle(dev, which):
    if which == "n64":
        s, rc = gen.system_64(), 11.0
    elif which == "n512":
        s, rc = gen.system_512(), 11.0
    else:
        s, rc = gen.batch_structure(int(which[5:])), 12.0
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    q, en, f, st = solve(dev, s, "sqnm", rc)
    qc, enc, fc, stc = solve(dev, s, "cg", rc)
    e = errs(q, en, f, ref)
    print(which, s.n, "q_tot", s.q_tot, "sqnm iters", st["iters"], "cg iters", stc["iters"], "errs", e,
          "true resid", st["true_rel_resid"])
    assert e[0] <= 1e-5 and e[1] <= 1e-6 and e[2] <= 1e-6 and e[3] <= 1e-4
    assert np.abs(q - qc).max() <= 1e-6
    assert abs(st["mu"] - ref.mu) <= 1e-5
    assert st["true_rel_resid"] <= 2e-7   # the FP32 gradient floor (SQNM stops at max(tol, 1e-7))
    if s.n <= 256:
        E = ewald.coulomb_matrix(s.pos, s.cell, s.sigma)
        _, it_o, _ = sqnm.qeq_sqnm(E, s.J, s.chi, s.q_tot, s.sigma, tol=1e-9)
        print("oracle sqnm iters", it_o)
        assert st["iters"] <= 2 * it_o + 10


def test_sqnm_full_size_32768(dev):
    path = os.path.join(os.path.dirname(__file__), "golden", "n32768_reference.npz")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    ref = np.load(path)
    s = gen.system_32k()
    q, en, f, st = solve(dev, s, "sqnm", tol=1e-6)
    dq = np.abs(q - ref["q"]).max()
    de_q = abs(en[0] - float(ref["e_qeq"])) / abs(float(ref["e_qeq"]))
    de_e = abs(en[1] - float(ref["e_elec"])) / abs(float(ref["e_elec"]))
    df = np.sqrt(np.mean((f - ref["forces"]) ** 2)) / np.sqrt(np.mean(ref["forces"] ** 2))
    print("n32768 sqnm", st, "dq", dq, "dEqeq", de_q, "dEelec", de_e, "dF", df)
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4


@pytest.mark.parametrize("op", ["ewald", "planewave"])
def test_sqnm_with_other_operators(dev, op):
    s = gen.batch_structure(40)
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    q, en, f, st = solve(dev, s, "sqnm", 12.0, op=op)
    e = errs(q, en, f, ref)
    print(op, "sqnm iters", st["iters"], e)
    assert e[0] <= 1e-5 and e[1] <= 1e-6 and e[2] <= 1e-6 and e[3] <= 1e-4


def test_sqnm_history_backward_and_errors(dev):
    from paper_2607_17978_amd import qeq
    s = gen.system_512()
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    for m in (1, 4, 16):
        q, en, f, st = solve(dev, s, "sqnm", history=m)
        print("history", m, "iters", st["iters"])
        assert np.abs(q - ref.q).max() <= 1e-5
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=s.grid, tol=1e-9)
    for bad in (-1, 17):
        with pytest.raises(qeq.QEqError):
            plan.use_sqnm(True, bad)
    args = (T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    w = T(np.random.default_rng(4).uniform(size=s.n), dev)
    plan.use_sqnm(True)
    q1, _, _, _ = plan.solve(*args)
    g1 = plan.backward(w * q1, dL_dEelec=1.0)
    plan.use_sqnm(False)
    q2, _, _, _ = plan.solve(*args)
    g2 = plan.backward(w * q2, dL_dEelec=1.0)
    for a, b in zip(g1[:3], g2[:3]):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max())
    plan.close()
