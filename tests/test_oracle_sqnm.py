"""Pins of the SQNM oracle (oracle.sqnm) against what the mathematics fixes.

* The QEq energy is strictly convex on the constraint plane (J > 0), so its
  minimiser is unique: SQNM must reach the Gaussian-elimination solution of
  the bordered system (dense oracle) on neutral and charged, cubic and
  triclinic cells.
* On a quadratic the gradient differences are exactly A times the
  displacements, so the subspace Hessian SQNM builds from them must have the
  Rayleigh-Ritz values of A on the span of the history (computed here
  directly from A), and its basis must be orthonormal in the D metric.
* With three atoms the plane is two-dimensional: once the history spans it
  the quasi-Newton step is the exact Newton step.
"""
import numpy as np
import pytest

from inputs import gen
from oracle import ewald, sqnm

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def dense(s):
    E = ewald.coulomb_matrix(s.pos, s.cell, s.sigma)
    return E, ewald.solve_qeq(E, s.J, s.chi, s.q_tot)[0]


@pytest.mark.parametrize("which", ["n64", "batch17", "batch40"])
def test_sqnm_reaches_the_unique_minimiser(which):
    s = gen.system_64() if which == "n64" else gen.batch_structure(int(which[5:]))
    E, q_ref = dense(s)
    q, it, res = sqnm.qeq_sqnm(E, s.J, s.chi, s.q_tot, s.sigma, tol=1e-11)
    print(which, s.n, "q_tot", s.q_tot, "iterations", it, "res", res)
    assert res <= 1e-11
    assert abs(q.sum() - s.q_tot) <= 1e-10
    assert np.abs(q - q_ref).max() <= 1e-9


def test_subspace_hessian_is_rayleigh_ritz_of_A():
    s = gen.system_64()
    E, _ = dense(s)
    A = E + np.diag(s.J)
    D = s.J + 1.0 / (s.sigma * np.sqrt(np.pi))
    rec = []
    sqnm.sqnm_minimise(lambda v: A @ v, D, s.chi, s.q_tot, tol=1e-9, record=rec)
    assert len(rec) >= 5
    for kap, dvec in rec[1:6]:
        gram = dvec.T @ (D[:, None] * dvec)
        assert np.abs(gram - np.eye(gram.shape[0])).max() <= 1e-8
        assert np.abs(dvec.sum(axis=0)).max() <= 1e-10       # displacements stay on the plane
        ritz = np.linalg.eigvalsh(dvec.T @ A @ dvec)
        assert np.allclose(np.sort(kap), ritz, rtol=1e-7, atol=1e-10)


def test_three_atoms_newton_step():
    rng = np.random.default_rng(5)
    M = rng.normal(size=(3, 3))
    A = M @ M.T + 3 * np.eye(3)
    chi = rng.normal(size=3)
    D = np.diag(A).copy()
    q, it, res = sqnm.sqnm_minimise(lambda v: A @ v, D, chi, 0.7, tol=1e-13)
    B = np.block([[A, np.ones((3, 1))], [np.ones((1, 3)), np.zeros((1, 1))]])
    x = np.linalg.solve(B, np.concatenate([-chi, [0.7]]))
    print("iterations", it)
    assert np.abs(q - x[:3]).max() <= 1e-12
    assert it <= 6


def test_sqnm_pin_catches_a_wrong_gradient_difference(monkeypatch):
    """Planting a mistake in the oracle (gradient differences off by 10%)
    breaks the Rayleigh-Ritz pin."""
    s = gen.system_64()
    E, _ = dense(s)
    A = E + np.diag(s.J)
    D = s.J + 1.0 / (s.sigma * np.sqrt(np.pi))
    calls = {"n": 0}

    def apply_bad(v):
        calls["n"] += 1
        return (A @ v) * (1.1 if calls["n"] % 2 else 1.0)
    rec = []
    sqnm.sqnm_minimise(apply_bad, D, s.chi, s.q_tot, tol=1e-9, max_iter=30, record=rec)
    bad = False
    for kap, dvec in rec[1:6]:
        ritz = np.linalg.eigvalsh(dvec.T @ A @ dvec)
        bad |= not np.allclose(np.sort(kap), ritz, rtol=1e-7, atol=1e-10)
    assert bad
