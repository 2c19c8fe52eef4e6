"""Direct Ewald reciprocal sums (qeq_use_ewald) against the FP64 oracle.

The explicit k-space sums replace the particle mesh on the same CG path, so
the only approximation left is the real-space truncation at r_cut: the bars
are the parity bars, and the errors come out well below the mesh path's.
"""
import numpy as np
import pytest

from inputs import gen
from oracle import ewald

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


def errs(q, en, f, st, ref):
    dq = np.abs(q - ref.q).max()
    de_q = abs(en[0] - ref.e_qeq) / abs(ref.e_qeq)
    de_e = abs(en[1] - ref.e_elec) / abs(ref.e_elec)
    df = np.sqrt(np.mean((f - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
    return dq, de_q, de_e, df, abs(st["mu"] - ref.mu)


@pytest.mark.parametrize("which", ["n64", "batch17", "batch40", "n512"])
def test_ewald_matches_oracle(dev, which):
    from paper_2607_17978_amd import qeq
    if which == "n64":
        s, rc = gen.system_64(), 11.0
    elif which == "n512":
        s, rc = gen.system_512(), 11.0
    else:
        s, rc = gen.batch_structure(int(which[5:])), 12.0
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    out = {}
    for mode in ("mesh", "ewald"):
        plan = qeq.Plan(s.n, eta=ETA, r_cut=rc, grid=s.grid, tol=1e-9, max_iter=3000)
        plan.use_ewald(mode == "ewald")
        q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        assert st["rc"] == 0, st
        out[mode] = errs(q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), st, ref)
        plan.close()
    print(which, "mesh", out["mesh"], "ewald", out["ewald"])
    dq, de_q, de_e, df, dmu = out["ewald"]
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4 and dmu <= 1e-5
    # exact reciprocal sums: at least as close to the oracle as the mesh
    assert de_e <= out["mesh"][2] + 1e-8


def test_ewald_with_spectral_and_refusals(dev):
    from paper_2607_17978_amd import qeq
    s = gen.system_512()
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=s.grid, tol=1e-8)
    args = (T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    plan.use_ewald(True)
    qa, _, _, sa = plan.solve(*args)
    plan.use_spectral_preconditioner(0.4)
    qb, _, _, sb = plan.solve(*args)
    print("ewald iters jacobi", sa["iters"], "spectral", sb["iters"])
    assert sb["iters"] < sa["iters"]
    assert np.abs(qa.cpu().numpy() - qb.cpu().numpy()).max() <= 1e-6
    with pytest.raises(qeq.QEqError):
        plan.backward(T(np.ones(s.n), dev))
    with pytest.raises(qeq.QEqError):
        plan.element_potentials(T(s.species, dev).to(torch.int32), 2)
    # back to the mesh: the tape is there again
    plan.use_ewald(False)
    plan.use_spectral_preconditioner(0.0)
    qm, _, _, sm = plan.solve(*args)
    plan.backward(T(np.ones(s.n), dev))
    assert np.abs(qm.cpu().numpy() - qa.cpu().numpy()).max() <= 1e-5
    plan.close()
