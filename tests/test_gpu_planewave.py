"""Gaussian-on-grid ("plane-wave") operator (qeq_use_planewave) against the
FP64 oracle.

The GPU operator samples each atom's Gaussian density on the plan's grid and
solves Poisson's equation there with the unscreened kernel 4 pi / k^2: with
the k = 0 term dropped it is a discretisation of the same plane-wave energy
the oracle's dense Ewald matrix equals (an oracle pin), so the bars are the
parity bars.  At the configs' spacing (<= 0.8 bohr, sigma >= 1 bohr) and a
6-sigma support the discretisation changes the operator by ~1e-8 relative;
the FP32 grid arithmetic is the larger error.
"""
import os

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


def solve(dev, s, mode, rc=11.0, tol=1e-9, support=6.0):
    from paper_2607_17978_amd import qeq
    plan = qeq.Plan(s.n, eta=ETA, r_cut=rc, grid=s.grid, tol=tol, max_iter=3000)
    if mode == "planewave":
        plan.use_planewave(True, support)
    q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    plan.close()
    assert st["rc"] == 0, st
    return q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), st


# neutral cubic cells, charged and neutral triclinic cells (sigma up to 1.7)
@pytest.mark.parametrize("which", ["n64", "batch3", "batch17", "batch40", "n512"])
def test_planewave_matches_oracle(dev, which):
    if which == "n64":
        s, rc = gen.system_64(), 11.0
    elif which == "n512":
        s, rc = gen.system_512(), 11.0
    else:
        s, rc = gen.batch_structure(int(which[5:])), 12.0
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    out = {mode: errs(*solve(dev, s, mode, rc), ref) for mode in ("mesh", "planewave")}
    print(which, s.n, s.grid, "q_tot", s.q_tot, "mesh", out["mesh"], "planewave", out["planewave"])
    dq, de_q, de_e, df, dmu = out["planewave"]
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4 and dmu <= 1e-5


def test_planewave_full_size_32768(dev):
    """The benchmark system (32,768 atoms, 192^3) against the stored FP64
    matrix-free oracle solution (tests/golden/make_n32768_reference.py)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "n32768_reference.npz")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    ref = np.load(path)
    s = gen.system_32k()
    q, en, f, st = solve(dev, s, "planewave", tol=1e-6)
    dq = np.abs(q - ref["q"]).max()
    de_q = abs(en[0] - float(ref["e_qeq"])) / abs(float(ref["e_qeq"]))
    de_e = abs(en[1] - float(ref["e_elec"])) / abs(float(ref["e_elec"]))
    df = np.sqrt(np.mean((f - ref["forces"]) ** 2)) / np.sqrt(np.mean(ref["forces"] ** 2))
    print("n32768 planewave", st, "dq", dq, "dEqeq", de_q, "dEelec", de_e, "dF", df)
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4


def test_planewave_support_and_refusals(dev):
    from paper_2607_17978_amd import qeq
    s = gen.system_512()
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    # a shorter support cuts more of each Gaussian: larger but bounded error
    e5 = errs(*solve(dev, s, "planewave", support=5.0), ref)
    e8 = errs(*solve(dev, s, "planewave", support=8.0), ref)
    print("support 5", e5, "support 8", e8)
    assert e8[0] <= 1e-5 and e8[2] <= 1e-6
    assert e5[2] >= e8[2]
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=s.grid, tol=1e-8)
    for bad in (2.0, 13.0, float("nan")):
        with pytest.raises(qeq.QEqError):
            plan.use_planewave(True, bad)
    args = (T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    plan.use_planewave(True)
    qa, _, _, sa = plan.solve(*args)
    # the spectral preconditioner approximates any operator with the same
    # long-wavelength part: same charges, fewer iterations
    plan.use_spectral_preconditioner(0.4)
    qb, _, _, sb = plan.solve(*args)
    print("planewave iters jacobi", sa["iters"], "spectral", sb["iters"])
    assert sb["iters"] < sa["iters"]
    assert np.abs(qa.cpu().numpy() - qb.cpu().numpy()).max() <= 1e-6
    with pytest.raises(qeq.QEqError):
        plan.backward(T(np.ones(s.n), dev))
    with pytest.raises(qeq.QEqError):
        plan.virial()
    with pytest.raises(qeq.QEqError):
        plan.element_potentials(T(s.species, dev).to(torch.int32), 2)
    # Ewald and plane-wave exclude each other; the last call wins
    plan.use_ewald(True)
    plan.use_spectral_preconditioner(0.0)
    qe, _, _, se = plan.solve(*args)
    assert np.abs(qe.cpu().numpy() - ref.q).max() <= 1e-5
    plan.use_planewave(True)
    plan.use_planewave(False)
    plan.use_ewald(False)
    qm, _, _, sm = plan.solve(*args)
    plan.backward(T(np.ones(s.n), dev))
    assert np.abs(qm.cpu().numpy() - qa.cpu().numpy()).max() <= 1e-5
    plan.close()



def test_planewave_grid320_matches_oracle(dev):
    """The 320^3 grid (8-row tiles in the axis-3 pass of the plane-wave path
    too): 64 atoms in the 235.7-bohr cube against dense Ewald
    (tests/golden/make_grid320_reference.py)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "grid320_reference.npz")
    if not os.path.exists(path):
        pytest.skip("reference not generated")
    ref = np.load(path)
    s = gen.lattice_system(4, 235.7, 1009, grid=(320, 320, 320), name="n64_L235.7")
    q, en, f, st = solve(dev, s, "planewave")
    dq = np.abs(q - ref["q"]).max()
    de_q = abs(en[0] - float(ref["e_qeq"])) / abs(float(ref["e_qeq"]))
    de_e = abs(en[1] - float(ref["e_elec"])) / abs(float(ref["e_elec"]))
    df = np.sqrt(np.mean((f - ref["forces"]) ** 2)) / np.sqrt(np.mean(ref["forces"] ** 2))
    print("grid320 planewave", st["iters"], "dq", dq, "dEqeq", de_q, "dEelec", de_e, "dF", df)
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4
