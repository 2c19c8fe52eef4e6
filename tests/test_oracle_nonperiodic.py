"""Pins of the non-periodic (isolated-system) QEq oracle.

The oracle writes out the paper's Coulomb kernel between normalised Gaussians
(E_ii = 1/(sigma_i sqrt(pi)), E_ij = erf(r_ij/(sqrt2 gamma_ij))/r_ij; the
Electrostatics and Charge Equilibration section) and solves the bordered
system of eq. 4G_qeq_prime.  Each test checks it against something other
than itself: closed forms and limits of the kernel, a scalar evaluation of
the two-atom solution, brute-force minimisation, finite differences of the
re-solved energy, the symmetries of an isolated system, the independent
periodic Ewald oracle in growing boxes, and planted mistakes.
"""
import math

import numpy as np
import pytest

from inputs import gen
from oracle import direct, ewald

SQRTPI = math.sqrt(math.pi)


def test_kernel_limits_and_derivative():
    # i = j limit with equal widths is the paper's Gaussian self energy
    for sig in (0.7, 1.0, 1.5):
        gam = math.sqrt(2.0) * sig
        assert abs(direct.nonperiodic_kernel(0.0, gam) - 1.0 / (sig * SQRTPI)) < 1e-15
        # the small-r series agrees with the closed form (scalar erf) below the switch
        for r in (1e-6, 0.99e-4):
            closed = math.erf(r / (math.sqrt(2.0) * gam)) / r
            assert abs(direct.nonperiodic_kernel(r, gam) - closed) < 1e-14
    # far field: a point-charge Coulomb law
    assert abs(direct.nonperiodic_kernel(40.0, 1.0) * 40.0 - 1.0) < 1e-15
    # derivative against central differences of the kernel
    r = np.linspace(1e-3, 20.0, 400)
    for gam in (1.2, 2.1):
        h = 1e-6
        fd = (direct.nonperiodic_kernel(r + h, gam) - direct.nonperiodic_kernel(r - h, gam)) / (2 * h)
        assert np.abs(fd - direct.nonperiodic_kernel_deriv(r, gam)).max() < 1e-8


def test_two_atom_closed_form_scalar():
    s = gen.cluster_system(2, q_tot=0.0, seed=11)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 0.0)
    r = float(np.linalg.norm(s.pos[0] - s.pos[1]))
    gam = math.sqrt(s.sigma[0] ** 2 + s.sigma[1] ** 2)
    e12 = math.erf(r / (math.sqrt(2.0) * gam)) / r
    e11, e22 = 1.0 / (s.sigma[0] * SQRTPI), 1.0 / (s.sigma[1] * SQRTPI)
    q1 = (s.chi[1] - s.chi[0]) / (s.J[0] + s.J[1] + e11 + e22 - 2.0 * e12)
    assert abs(res.q[0] - q1) < 1e-14 and abs(res.q[1] + q1) < 1e-14


def test_single_atom():
    s = gen.cluster_system(1, q_tot=-1.0)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, -1.0)
    e_self = 0.5 / (s.sigma[0] * SQRTPI)
    assert res.q[0] == -1.0
    assert abs(res.e_elec - e_self) < 1e-15
    assert abs(res.e_qeq - (e_self - s.chi[0] + 0.5 * s.J[0])) < 1e-15
    assert np.abs(res.forces).max() == 0.0


@pytest.mark.parametrize("n,q_tot", [(5, 0.0), (6, 1.0), (8, -1.0)])
def test_brute_force(n, q_tot):
    s = gen.cluster_system(n, q_tot=q_tot, seed=20 + n)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, q_tot)
    qb = direct.brute_force_qeq(res.E + np.diag(s.J), s.chi, q_tot)
    assert np.abs(qb - res.q).max() < 1e-9


@pytest.mark.parametrize("q_tot", [0.0, 1.0])
def test_stationarity_and_constraint(q_tot):
    s = gen.cluster_system(64, q_tot=q_tot)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, q_tot)
    g = res.E @ res.q + s.J * res.q + s.chi
    assert np.ptp(g) < 1e-12 and abs(g.mean() - res.mu) < 1e-12
    assert abs(res.q.sum() - q_tot) < 1e-12
    # E_QEq = 1/2 chi.q + 1/2 mu Q at the solution
    assert abs(res.e_qeq - (0.5 * s.chi @ res.q + 0.5 * res.mu * q_tot)) < 1e-13


def test_forces_by_finite_differences():
    """F = -dE_QEq/dr with the charges re-solved at every displaced geometry."""
    s = gen.cluster_system(9, q_tot=1.0, seed=31)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 1.0)
    h = 1e-5
    for i in (0, 4, 8):
        for c in range(3):
            e = []
            for sgn in (1, -1):
                p = s.pos.copy()
                p[i, c] += sgn * h
                e.append(direct.qeq_nonperiodic(p, s.sigma, s.J, s.chi, 1.0, forces=False).e_qeq)
            fd = -(e[0] - e[1]) / (2 * h)
            assert abs(fd - res.forces[i, c]) < 1e-9


def test_isolated_system_symmetries():
    s = gen.cluster_system(40, q_tot=1.0, seed=41)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 1.0)
    # no net force and no net torque on an isolated system
    assert np.abs(res.forces.sum(0)).max() < 1e-14
    assert np.abs(np.cross(s.pos, res.forces).sum(0)).max() < 1e-13
    # rotation + translation: same charges and energy, rotated forces
    rng = np.random.default_rng(5)
    Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    p2 = s.pos @ Qm.T + np.array([3.0, -7.0, 11.0])
    r2 = direct.qeq_nonperiodic(p2, s.sigma, s.J, s.chi, 1.0)
    assert np.abs(r2.q - res.q).max() < 1e-12 and abs(r2.e_qeq - res.e_qeq) < 1e-12
    assert np.abs(r2.forces - res.forces @ Qm.T).max() < 1e-12
    # permutation equivariance
    perm = rng.permutation(s.n)
    r3 = direct.qeq_nonperiodic(s.pos[perm], s.sigma[perm], s.J[perm], s.chi[perm], 1.0)
    assert np.abs(r3.q - res.q[perm]).max() < 1e-12


def test_cg_matches_dense():
    s = gen.cluster_system(517, q_tot=-1.0)
    a = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, -1.0)
    b = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, -1.0, method="cg", tol=1e-13)
    assert np.abs(a.q - b.q).max() < 1e-11
    assert abs(a.e_qeq - b.e_qeq) < 1e-11 * abs(a.e_qeq)


def test_periodic_oracle_large_box_limit():
    """The independent periodic Ewald oracle of a neutral cluster in a cubic box
    of edge L converges to the isolated result as L^-3 (the tin-foil dipole
    term); Richardson extrapolation in L^-3 lands on it."""
    s = gen.cluster_system(16, q_tot=0.0, seed=5)
    ref = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 0.0)
    out = {}
    for L in (40.0, 80.0):
        r = ewald.qeq_dense(s.pos + 0.5 * L, np.eye(3) * L, s.sigma, s.J, s.chi, 0.0)
        out[L] = r
    e40 = np.abs(out[40.0].q - ref.q).max()
    e80 = np.abs(out[80.0].q - ref.q).max()
    assert 6.0 < e40 / e80 < 10.0
    q_inf = (8.0 * out[80.0].q - out[40.0].q) / 7.0
    assert np.abs(q_inf - ref.q).max() < 0.1 * e80
    f_inf = (8.0 * out[80.0].forces - out[40.0].forces) / 7.0
    assert np.abs(f_inf - ref.forces).max() < 0.25 * np.abs(out[80.0].forces - ref.forces).max()


# ---------------------------------------------------------------------------
# Planted mistakes: copies of the oracle with a plausible error fail the pins
# ---------------------------------------------------------------------------

def test_planted_wrong_width_is_caught(monkeypatch):
    good = direct.nonperiodic_kernel

    def wrong(r, gamma):   # erf(r / gamma) / r: the sqrt(2) dropped
        return good(r, np.asarray(gamma) / math.sqrt(2.0))

    monkeypatch.setattr(direct, "nonperiodic_kernel", wrong)
    gam = math.sqrt(2.0) * 1.0
    assert abs(direct.nonperiodic_kernel(0.0, gam) - 1.0 / SQRTPI) > 1e-3


def test_planted_force_mistake_is_caught(monkeypatch):
    good = direct.nonperiodic_kernel_deriv

    def wrong(r, gamma):   # the Gaussian term dropped from K'
        a = 1.0 / (math.sqrt(2.0) * np.asarray(gamma))
        return good(r, gamma) - 2.0 / SQRTPI * a * np.exp(-(a * r) ** 2) / np.where(r < 1e-4, 1.0, r)

    s = gen.cluster_system(9, q_tot=1.0, seed=31)
    base = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 1.0)
    monkeypatch.setattr(direct, "nonperiodic_kernel_deriv", wrong)
    bad = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 1.0)
    h = 1e-5
    p = s.pos.copy()
    p[0, 0] += h
    ep = direct.qeq_nonperiodic(p, s.sigma, s.J, s.chi, 1.0, forces=False).e_qeq
    p[0, 0] -= 2 * h
    em = direct.qeq_nonperiodic(p, s.sigma, s.J, s.chi, 1.0, forces=False).e_qeq
    fd = -(ep - em) / (2 * h)
    assert abs(fd - base.forces[0, 0]) < 1e-9
    assert abs(fd - bad.forces[0, 0]) > 1e-6


def test_coincident_atoms_finite():
    """Coincident atoms: the kernel takes its r -> 0 limit, forces stay finite
    and still match finite differences of the re-solved energy."""
    s = gen.cluster_system(12, q_tot=0.0, seed=77)
    s.pos[1] = s.pos[0]
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 0.0)
    assert np.all(np.isfinite(res.forces)) and np.all(np.isfinite(res.q))
    h = 1e-5
    for i, c in ((3, 0), (5, 2)):
        e = []
        for sgn in (1, -1):
            p = s.pos.copy()
            p[i, c] += sgn * h
            e.append(direct.qeq_nonperiodic(p, s.sigma, s.J, s.chi, 0.0, forces=False).e_qeq)
        assert abs(-(e[0] - e[1]) / (2 * h) - res.forces[i, c]) < 1e-9
