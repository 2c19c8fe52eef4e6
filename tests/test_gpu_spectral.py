"""Spectral (small-k Woodbury) preconditioner of the projected CG on the GPU.

The preconditioner changes the path to the solution, not the solution: the
charges, energies and forces must meet the same bars against the FP64 oracle
as the Jacobi solve (max |dq| <= 1e-5 e, relative energies <= 1e-6, relative
force RMS <= 1e-4), in fewer iterations.
"""
import os

import numpy as np
import pytest

from inputs import gen
from oracle import ewald, matfree

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


def solve(dev, s, rc, kc, tol=1e-7, plan=None):
    from paper_2607_17978_amd import qeq
    own = plan is None
    if own:
        plan = qeq.Plan(s.n, eta=ETA, r_cut=rc, grid=s.grid, tol=tol)
    plan.use_spectral_preconditioner(kc)
    q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    out = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), st
    if own:
        plan.close()
    return out


def check(q, en, f, ref):
    dq = np.abs(q - ref.q).max()
    de_q = abs(en[0] - ref.e_qeq) / abs(ref.e_qeq)
    de_e = abs(en[1] - ref.e_elec) / abs(ref.e_elec)
    df = np.sqrt(np.mean((f - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4, (dq, de_q, de_e, df)
    return dq, de_q, de_e, df


@pytest.mark.parametrize("which,kc", [("batch17", 0.5), ("batch40", 0.5), ("n4096", 0.25)])
def test_spectral_solve_matches_oracle(dev, which, kc):
    if which == "n4096":
        s, rc = gen.system_4096(), 11.0
        ref = matfree.qeq_matfree(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot, tol=1e-10, forces=True)
    else:
        s, rc = gen.batch_structure(int(which[5:])), 12.0
        ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    q0, e0, f0, st0 = solve(dev, s, rc, 0.0)
    q1, e1, f1, st1 = solve(dev, s, rc, kc)
    print(which, "Jacobi iters", st0["iters"], "spectral iters", st1["iters"], check(q1, e1, f1, ref))
    assert st1["rc"] == 0
    assert st1["iters"] < st0["iters"]


def test_spectral_full_size_32768(dev):
    """The benchmark configuration with the spectral preconditioner against the
    stored oracle solution, in at most 20 CG iterations (Jacobi takes 57)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "n32768_reference.npz")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    ref = np.load(path)
    s = gen.system_32k()
    q, en, f, st = solve(dev, s, 11.0, 0.2, tol=1e-6)
    dq = np.abs(q - ref["q"]).max()
    de_q = abs(en[0] - float(ref["e_qeq"])) / abs(float(ref["e_qeq"]))
    de_e = abs(en[1] - float(ref["e_elec"])) / abs(float(ref["e_elec"]))
    df = np.sqrt(np.mean((f - ref["forces"]) ** 2)) / np.sqrt(np.mean(ref["forces"] ** 2))
    print("n32768 spectral", st, "dq", dq, "dEqeq", de_q, "dEelec", de_e, "dF", df)
    assert st["rc"] == 0 and st["iters"] <= 20
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4


def test_spectral_repeat_and_switch(dev):
    """Graph replays give the same charges on repeated solves; switching back to
    Jacobi restores the Jacobi iteration count; cutoffs below the smallest
    reciprocal vector fall back to Jacobi."""
    from paper_2607_17978_amd import qeq
    s = gen.system_4096()
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=s.grid, tol=1e-7)
    qa, _, _, sa = solve(dev, s, 11.0, 0.25, plan=plan)
    qb, _, _, sb = solve(dev, s, 11.0, 0.25, plan=plan)
    assert sa["iters"] == sb["iters"] and np.abs(qa - qb).max() <= 1e-12
    _, _, _, sj = solve(dev, s, 11.0, 0.0, plan=plan)
    _, _, _, sj2 = solve(dev, s, 11.0, 0.01, plan=plan)   # 2 pi / L = 0.085 > 0.01: no modes
    assert sj["iters"] == sj2["iters"] > sa["iters"]
    with pytest.raises(qeq.QEqError):
        plan.use_spectral_preconditioner(float("nan"))
    plan.close()


def test_spectral_adjoint_matches_jacobi(dev):
    """qeq_backward with the spectral preconditioner gives the Jacobi gradients."""
    from paper_2607_17978_amd import qeq
    s = gen.batch_structure(40)
    rng = np.random.default_rng(3)
    g = T(rng.normal(size=s.n), dev)
    out = []
    for kc in (0.0, 0.5):
        plan = qeq.Plan(s.n, eta=ETA, r_cut=12.0, grid=s.grid, tol=1e-9)
        plan.use_spectral_preconditioner(kc)
        plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        dchi, dJ, dpos, st = plan.backward(g, dL_dEelec=0.7, dL_dEqeq=0.3)
        out.append((dchi.cpu().numpy(), dpos.cpu().numpy(), st["iters"]))
        plan.close()
    (c0, p0, i0), (c1, p1, i1) = out
    print("adjoint iters Jacobi", i0, "spectral", i1)
    assert np.abs(c1 - c0).max() <= 1e-6 * np.abs(c0).max()
    assert np.abs(p1 - p0).max() <= 1e-5 * np.abs(p0).max()


def test_precond_field_of_the_plan_parameters(dev):
    """qeq_params.precond = 1 with spectral_kcut selects the same preconditioner
    as qeq_use_spectral_preconditioner: identical iteration count and charges
    (same kernels, same modes), and the oracle's bars."""
    from paper_2607_17978_amd import qeq
    s = gen.system_4096()
    ref = matfree.qeq_matfree(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot, tol=1e-10)
    q1, en1, f1, st1 = solve(dev, s, 11.0, 0.25)
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=s.grid, tol=1e-7, spectral_kcut=0.25)
    assert plan.params.precond == 1
    q2, en2, f2, st2 = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    q2 = q2.cpu().numpy()
    plan.close()
    assert st2["iters"] == st1["iters"] and st1["iters"] < 40, (st1["iters"], st2["iters"])
    assert np.abs(q2 - q1).max() <= 1e-9
    check(q2, en2.cpu().numpy(), f2.cpu().numpy(), ref)
