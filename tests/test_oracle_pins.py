"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, a textbook constant, an independent formula (the plain plane-wave sum,
the paper's non-periodic kernel), a library solver, brute-force minimisation,
or finite differences.  The last group plants plausible mistakes into copies
of the oracle and shows that the pins catch them.
"""
import math

import numpy as np
import pytest

from inputs import gen
from oracle import direct, ewald, matfree

SQRTPI = math.sqrt(math.pi)


def small_triclinic(n=6, seed=3, q_tot=1.0):
    rng = np.random.default_rng(seed)
    cell = np.array([[9.0, 0.0, 0.0], [1.5, 8.5, 0.0], [-1.0, 2.0, 10.0]])
    frac = rng.uniform(0, 1, (n, 3))
    pos = frac @ cell
    sigma = rng.choice([1.0, 1.3, 1.7], n)
    J = rng.choice([0.3, 0.45, 0.6], n)
    chi = rng.normal(0, 0.1, n)
    return pos, cell, sigma, J, chi, q_tot


# ---------------------------------------------------------------------------
# The Ewald split
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("charged", [False, True])
def test_eta_invariance_of_matrix(charged):
    pos, cell, sigma, J, chi, _ = small_triclinic()
    A = [ewald.coulomb_matrix(pos, cell, sigma, eta=e) for e in (1.1, 1.9, 3.2)]
    for other in A[1:]:
        assert np.abs(other - A[0]).max() < 1e-13
    s = gen.system_64()
    B1 = ewald.coulomb_matrix(s.pos, s.cell, s.sigma, eta=1.4)
    B2 = ewald.coulomb_matrix(s.pos, s.cell, s.sigma, eta=2.6)
    assert np.abs(B1 - B2).max() < 1e-13


@pytest.mark.parametrize("q_tot", [0.0, 1.0, -1.0])
def test_ewald_equals_planewave_definition(q_tot):
    """1/2 q^T E q equals the plain k-space sum with Gaussian form factors."""
    pos, cell, sigma, _, _, _ = small_triclinic(n=5, seed=11)
    rng = np.random.default_rng(2)
    q = rng.normal(size=5)
    q += (q_tot - q.sum()) / 5
    E = ewald.coulomb_matrix(pos, cell, sigma)
    e_ewald = 0.5 * q @ E @ q
    e_pw = direct.planewave_energy(q, pos, cell, sigma)
    assert abs(e_ewald - e_pw) < 1e-12 * max(1.0, abs(e_pw))


def test_truncation_converged():
    pos, cell, sigma, _, _, _ = small_triclinic()
    eta = 1.7
    r0, k0 = ewald.default_cutoffs(eta, math.sqrt(2) * sigma.max())
    A0 = ewald.coulomb_matrix(pos, cell, sigma, eta=eta)
    A1 = ewald.coulomb_matrix(pos, cell, sigma, eta=eta, r_max=1.3 * r0, k_max=1.3 * k0)
    assert np.abs(A1 - A0).max() < 1e-14


def test_madelung_rock_salt():
    """sigma -> 0: (E_elec - sum q^2/(2 sigma sqrt pi)) -> -M (N/2) / r0, M = 1.747565."""
    a = 6.0
    pos, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                pos.append([i * a / 2, j * a / 2, k * a / 2])
                q.append((-1.0) ** (i + j + k))
    pos, q = np.array(pos), np.array(q)
    sig = np.full(8, 0.05)
    E = ewald.coulomb_matrix(pos, np.eye(3) * a, sig, eta=0.8)
    e_point = 0.5 * q @ E @ q - np.sum(q * q / (2 * sig * SQRTPI))
    madelung = -e_point * (a / 2) / 4
    assert abs(madelung - 1.747565) < 1e-6


def test_large_box_limit_is_paper_kernel():
    """Neutral cluster in a box of side L: E_per = E_iso - 2 pi |D|^2 / (3 L^3) + O(L^-5).

    E_iso uses the paper's non-periodic kernel (erf / self terms), so this ties
    the periodic Ewald matrix to the paper's E_ij.
    """
    rng = np.random.default_rng(5)
    pos0 = rng.uniform(-2, 2, (4, 3))
    q = rng.normal(size=4)
    q -= q.mean()
    sig = np.array([1.0, 1.5, 1.2, 0.9])
    e_iso = 0.5 * q @ direct.nonperiodic_matrix(pos0, sig) @ q
    D = q @ pos0
    res = []
    for L in (30.0, 60.0, 120.0):
        E = ewald.coulomb_matrix(pos0 + L / 2, np.eye(3) * L, sig)
        e_per = 0.5 * q @ E @ q
        res.append(e_per - e_iso + 2 * math.pi / 3 * (D @ D) / L ** 3)
    assert abs(res[2]) < 1e-7
    # the remainder falls like L^-5 (quadrupole images)
    assert 20 < res[0] / res[1] < 45 and 20 < res[1] / res[2] < 45


def test_gaussian_self_energy_limit():
    """erf(r/(sqrt2 gamma_ii))/r -> 1/(sigma sqrt pi) as r -> 0 (paper's E_ii)."""
    for s in (0.7, 1.0, 1.7):
        g = math.sqrt(2) * s
        r = 1e-7
        assert abs(math.erf(r / (math.sqrt(2) * g)) / r - 1 / (s * SQRTPI)) < 1e-9
        # and the oracle's pair kernel has the matching small-r series
        k_small = ewald.pair_kernel(np.array([5e-5]), g, 2.0)[0]
        k_ref = (math.erf(5e-5 / (math.sqrt(2) * g)) - math.erf(5e-5 / (math.sqrt(2) * 2.0))) / 5e-5
        assert abs(k_small - k_ref) < 1e-12


# ---------------------------------------------------------------------------
# The bordered solve
# ---------------------------------------------------------------------------

def test_gauss_elimination_matches_lapack():
    s = gen.system_64()
    E = ewald.coulomb_matrix(s.pos, s.cell, s.sigma)
    q1, l1 = ewald.solve_qeq(E, s.J, s.chi, 0.3)
    q2, l2 = ewald.solve_qeq(E, s.J, s.chi, 0.3, solver=np.linalg.solve)
    assert np.abs(q1 - q2).max() < 1e-13 and abs(l1 - l2) < 1e-13


def test_constraint_stationarity_closed_form():
    pos, cell, sigma, J, chi, q_tot = small_triclinic(n=7, seed=8, q_tot=-1.0)
    r = ewald.qeq_dense(pos, cell, sigma, J, chi, q_tot, forces=False)
    assert abs(r.q.sum() - q_tot) < 1e-12
    g = (r.E + np.diag(J)) @ r.q + chi
    assert np.abs(g - r.mu).max() < 1e-12
    # E_QEq at the solution = 1/2 chi.q - 1/2 lam Q
    assert abs(r.e_qeq - (0.5 * chi @ r.q - 0.5 * r.lam * q_tot)) < 1e-13


def test_two_atom_closed_form():
    pos = np.array([[0.0, 0.0, 0.0], [2.3, 0.4, -0.7]])
    sigma = np.array([1.0, 1.5])
    J = np.array([0.3, 0.5])
    chi = np.array([0.12, -0.07])
    E = direct.nonperiodic_matrix(pos, sigma)
    q, _ = ewald.solve_qeq(E, J, chi, 0.0)
    assert np.abs(q - direct.two_atom_charges(E, J, chi)).max() < 1e-14


@pytest.mark.parametrize("seed,n", [(1, 3), (2, 5), (4, 8)])
def test_brute_force_minimisation(seed, n):
    pos, cell, sigma, J, chi, _ = small_triclinic(n=n, seed=seed)
    q_tot = float(seed % 3 - 1)
    r = ewald.qeq_dense(pos, cell, sigma, J, chi, q_tot, forces=False)
    qb = direct.brute_force_qeq(r.E + np.diag(J), chi, q_tot)
    assert np.abs(qb - r.q).max() < 1e-9


def test_uniform_lattice_identical_atoms():
    """Identical atoms on a perfect simple-cubic lattice share the charge equally."""
    n_side, a = 3, 4.0
    idx = np.arange(n_side)
    g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3) * a
    n = g.shape[0]
    for q_tot in (0.0, 2.0):
        r = ewald.qeq_dense(g, np.eye(3) * n_side * a, np.full(n, 1.2), np.full(n, 0.4),
                            np.full(n, 0.05), q_tot)
        assert np.abs(r.q - q_tot / n).max() < 1e-12
        assert np.abs(r.forces).max() < 1e-10


def test_translation_and_permutation():
    s = gen.system_64()
    r0 = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, 0.0)
    shift = np.array([1.7, -0.4, 3.1])
    r1 = ewald.qeq_dense(s.pos + shift, s.cell, s.sigma, s.J, s.chi, 0.0)
    assert np.abs(r1.q - r0.q).max() < 1e-12
    assert abs(r1.e_qeq - r0.e_qeq) < 1e-12
    assert np.abs(r1.forces - r0.forces).max() < 1e-11
    perm = np.random.default_rng(0).permutation(s.n)
    r2 = ewald.qeq_dense(s.pos[perm], s.cell, s.sigma[perm], s.J[perm], s.chi[perm], 0.0)
    assert np.abs(r2.q - r0.q[perm]).max() < 1e-12
    assert np.abs(r2.forces - r0.forces[perm]).max() < 1e-11
    # Newton's third law over the periodic system
    assert np.abs(r0.forces.sum(0)).max() < 1e-11


# ---------------------------------------------------------------------------
# Forces and the adjoint gradient against finite differences
# ---------------------------------------------------------------------------

def _small_system(n=8, seed=21):
    s = gen.system_64()
    idx = np.random.default_rng(seed).choice(s.n, n, replace=False)
    return s.pos[idx], s.cell, s.sigma[idx], s.J[idx], s.chi[idx]


def test_adjoint_energy_weights_match_finite_differences():
    """dL/dE_QEq and dL/dE_elec weights (no charge term) against FD of the energies."""
    pos, cell, sigma, J, chi = _small_system(n=6, seed=9)
    q_tot = 1.0
    _, dchi, dpos, dJ = ewald.qeq_adjoint(pos, cell, sigma, J, chi, q_tot, np.zeros(6),
                                           dL_dEelec=0.7, dL_dEqeq=-1.3)

    def loss(p, c, Jv):
        r = ewald.qeq_dense(p, cell, sigma, Jv, c, q_tot, forces=False)
        return 0.7 * r.e_elec - 1.3 * r.e_qeq

    h = 1e-5
    cp = chi.copy(); cp[1] += h
    cm = chi.copy(); cm[1] -= h
    assert abs((loss(pos, cp, J) - loss(pos, cm, J)) / (2 * h) - dchi[1]) < 1e-8
    jp = J.copy(); jp[3] += h
    jm = J.copy(); jm[3] -= h
    assert abs((loss(pos, chi, jp) - loss(pos, chi, jm)) / (2 * h) - dJ[3]) < 1e-8
    pp = pos.copy(); pp[4, 1] += h
    pm = pos.copy(); pm[4, 1] -= h
    assert abs((loss(pp, chi, J) - loss(pm, chi, J)) / (2 * h) - dpos[4, 1]) < 1e-8


def test_forces_are_minus_energy_derivative_with_resolved_charges():
    pos, cell, sigma, J, chi = _small_system()
    q_tot = 0.5
    r = ewald.qeq_dense(pos, cell, sigma, J, chi, q_tot)
    h = 1e-5
    for (i, c) in [(0, 0), (3, 1), (7, 2)]:
        ep = pos.copy(); ep[i, c] += h
        em = pos.copy(); em[i, c] -= h
        fp = ewald.qeq_dense(ep, cell, sigma, J, chi, q_tot, forces=False).e_qeq
        fm = ewald.qeq_dense(em, cell, sigma, J, chi, q_tot, forces=False).e_qeq
        fd = -(fp - fm) / (2 * h)
        assert abs(fd - r.forces[i, c]) < 1e-8 * max(1.0, abs(fd))


def test_adjoint_gradient_matches_finite_differences():
    pos, cell, sigma, J, chi = _small_system(seed=5)
    q_tot = 0.0
    w, q_ref = gen.adjoint_targets(len(J), seed=1003)

    def loss(p, c):
        r = ewald.qeq_dense(p, cell, sigma, J, c, q_tot, forces=False)
        return np.sum(w * (r.q - q_ref) ** 2) + r.e_elec, r

    _, r0 = loss(pos, chi)
    dl_dq = 2 * w * (r0.q - q_ref)
    _, dchi, dpos, dJ = ewald.qeq_adjoint(pos, cell, sigma, J, chi, q_tot, dl_dq, dL_dEelec=1.0)
    h = 1e-5
    for i in (0, 4):
        cp = chi.copy(); cp[i] += h
        cm = chi.copy(); cm[i] -= h
        fd = (loss(pos, cp)[0] - loss(pos, cm)[0]) / (2 * h)
        assert abs(fd - dchi[i]) < 1e-8

    def loss_J(Jv):
        r = ewald.qeq_dense(pos, cell, sigma, Jv, chi, q_tot, forces=False)
        return np.sum(w * (r.q - q_ref) ** 2) + r.e_elec

    for i in (2, 7):
        jp = J.copy(); jp[i] += h
        jm = J.copy(); jm[i] -= h
        fd = (loss_J(jp) - loss_J(jm)) / (2 * h)
        assert abs(fd - dJ[i]) < 1e-8
    for (i, c) in [(1, 0), (6, 2)]:
        pp = pos.copy(); pp[i, c] += h
        pm = pos.copy(); pm[i, c] -= h
        fd = (loss(pp, chi)[0] - loss(pm, chi)[0]) / (2 * h)
        assert abs(fd - dpos[i, c]) < 1e-8


# ---------------------------------------------------------------------------
# Matrix-free oracle against the dense one
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["64", "512", "tri"])
def test_matfree_matches_dense(which):
    if which == "64":
        s = gen.system_64()
        args = (s.pos, s.cell, s.sigma, s.J, s.chi, 0.0)
    elif which == "512":
        s = gen.system_512()
        args = (s.pos, s.cell, s.sigma, s.J, s.chi, 0.0)
    else:
        b = gen.batch_structure(7)
        args = (b.pos, b.cell, b.sigma, b.J, b.chi, b.q_tot)
    d = ewald.qeq_dense(*args)
    m = matfree.qeq_matfree(*args)
    v = np.random.default_rng(1).normal(size=len(args[3]))
    op = matfree.EwaldOperator(args[0], args[1], args[2])
    assert np.abs(op.apply(v) - d.E @ v).max() < 1e-12
    assert np.abs(m.q - d.q).max() < 1e-9
    assert abs(m.e_elec - d.e_elec) < 1e-10 * abs(d.e_elec)
    assert abs(m.e_qeq - d.e_qeq) < 1e-10 * abs(d.e_qeq)
    assert abs(m.mu - d.mu) < 1e-9
    assert np.abs(m.forces - d.forces).max() < 1e-9


def test_matfree_bilinear_gradient_matches_dense():
    s = gen.system_64()
    rng = np.random.default_rng(3)
    q, a = rng.normal(size=s.n), rng.normal(size=s.n)
    op = matfree.EwaldOperator(s.pos, s.cell, s.sigma)
    g1 = op.grad_positions(q, a=a)
    g2 = ewald.energy_gradient_positions(s.pos, s.cell, s.sigma, q, a=a)
    assert np.abs(g1 - g2).max() < 1e-11


# ---------------------------------------------------------------------------
# Planted mistakes: each pin above catches at least one plausible error
# ---------------------------------------------------------------------------

def test_pins_catch_planted_mistakes(monkeypatch):
    pos, cell, sigma, _, _, _ = small_triclinic()

    def eta_spread():
        A1 = ewald.coulomb_matrix(pos, cell, sigma, eta=1.2)
        A2 = ewald.coulomb_matrix(pos, cell, sigma, eta=2.8)
        return np.abs(A1 - A2).max()

    assert eta_spread() < 1e-13
    # (1) k-space prefactor 2 pi instead of 4 pi
    orig_w = ewald.kspace_weights
    monkeypatch.setattr(ewald, "kspace_weights", lambda k2, v, e: 0.5 * orig_w(k2, v, e))
    assert eta_spread() > 1e-4
    monkeypatch.setattr(ewald, "kspace_weights", orig_w)
    # (2) screening Gaussian read as exp(-eta^2 k^2 / 4)
    monkeypatch.setattr(ewald, "kspace_weights",
                        lambda k2, v, e: orig_w(k2, v, e) * np.exp(0.25 * e * e * k2))
    assert eta_spread() > 1e-4
    monkeypatch.setattr(ewald, "kspace_weights", orig_w)
    # (3) pair kernel with gamma = sigma_i + sigma_j instead of sqrt(sum of squares):
    #     eta-invariant, but the plane-wave definition catches it
    orig_k = ewald.pair_kernel
    monkeypatch.setattr(ewald, "pair_kernel", lambda r, g, e: orig_k(r, g * 1.2, e))
    q = np.random.default_rng(2).normal(size=pos.shape[0])
    E = ewald.coulomb_matrix(pos, cell, sigma)
    assert abs(0.5 * q @ E @ q - direct.planewave_energy(q, pos, cell, sigma)) > 1e-4
    monkeypatch.setattr(ewald, "pair_kernel", orig_k)
    # (4) a missing background term: eta-dependence for the charged case
    def no_bg(pos_, cell_, sigma_, eta=None, r_max=None, k_max=None):
        vol = abs(np.linalg.det(cell_))
        A = ewald.coulomb_matrix(pos_, cell_, sigma_, eta=eta)
        s2 = sigma_ ** 2
        return A + (2 * math.pi / vol) * (eta * eta - s2[:, None] - s2[None, :])
    q = np.full(pos.shape[0], 1.0 / pos.shape[0])
    e1 = 0.5 * q @ no_bg(pos, cell, sigma, eta=1.2) @ q
    e2 = 0.5 * q @ no_bg(pos, cell, sigma, eta=2.8) @ q
    assert abs(e1 - e2) > 1e-3


def test_weighted_descriptors_linear_in_weights():
    """Weighted radial descriptors: unit weights give the plain ones, and the
    sum over an element partition of the weights gives the total (each
    neighbour term carries exactly its own weight)."""
    from oracle import mlp as omlp
    s = gen.system_64()
    c = np.linspace(1.0, 9.0, 8)
    G = omlp.radial_descriptors(s.pos, s.cell, c, 0.7, 8.0)
    assert np.abs(omlp.radial_descriptors(s.pos, s.cell, c, 0.7, 8.0, weights=np.ones(s.n)) - G).max() < 1e-14
    parts = [omlp.radial_descriptors(s.pos, s.cell, c, 0.7, 8.0, weights=(s.species == e).astype(float))
             for e in (0, 1)]
    assert np.abs(parts[0] + parts[1] - G).max() < 1e-12
    w = np.random.default_rng(2).normal(size=s.n)
    Gw = omlp.radial_descriptors(s.pos, s.cell, c, 0.7, 8.0, weights=w)
    # brute force for atom 0 over images within the cutoff
    L = s.cell[0, 0]
    d = s.pos - s.pos[0]
    ref = np.zeros(len(c))
    for sh in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).T.reshape(-1, 3):
        dd = d + sh * L
        r = np.linalg.norm(dd, axis=1)
        m = (r < 8.0) & (r > 1e-12)
        fc = 0.5 * (np.cos(np.pi * r[m] / 8.0) + 1.0)
        ref += (w[m][:, None] * np.exp(-(r[m][:, None] - c) ** 2 / (2 * 0.49)) * fc[:, None]).sum(0)
    assert np.abs(Gw[0] - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# Virial W = -dE/d eps (strain of positions and cell at fixed fractional
# coordinates)
# ---------------------------------------------------------------------------

def _energy_at_strain(pos, cell, sigma, q, F):
    p2, c2 = ewald.strained(pos, cell, F)
    return 0.5 * q @ ewald.coulomb_matrix(p2, c2, sigma) @ q


def _strain_fd(fn, h=1e-5):
    """-d fn(F)/dF_ab at F = 1 by central differences, every (a, b)."""
    W = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            Fp, Fm = np.eye(3), np.eye(3)
            Fp[a, b] += h
            Fm[a, b] -= h
            W[a, b] = -(fn(Fp) - fn(Fm)) / (2 * h)
    return W


def _charges(n, q_tot, seed):
    q = np.random.default_rng(seed).normal(0, 0.4, n)
    return q + (q_tot - q.sum()) / n


@pytest.mark.parametrize("q_tot", [0.0, 1.0])
def test_virial_is_minus_strain_derivative(q_tot):
    """All nine components against finite differences of the dense Ewald
    energy under r -> F r (non-symmetric F, so the antisymmetric part, zero by
    rotation invariance, is checked too)."""
    pos, cell, sigma, _, _, _ = small_triclinic(n=6, seed=7)
    q = _charges(6, q_tot, 4)
    W = ewald.virial(pos, cell, sigma, q)
    fd = _strain_fd(lambda F: _energy_at_strain(pos, cell, sigma, q, F))
    scale = np.abs(W).max()
    assert np.abs(W - W.T).max() < 1e-13 * scale
    assert np.abs(W - fd).max() < 1e-8 * scale


def test_virial_eta_invariant():
    pos, cell, sigma, _, _, _ = small_triclinic(n=6, seed=8)
    q = _charges(6, -1.0, 5)
    Ws = [ewald.virial(pos, cell, sigma, q, eta=e) for e in (1.2, 1.9, 2.8)]
    for W in Ws[1:]:
        assert np.abs(W - Ws[0]).max() < 1e-12 * np.abs(Ws[0]).max()


def test_virial_point_charge_homogeneity():
    """Rock salt with sigma -> 0: past the (length-independent) self energies
    the energy is a lattice sum of 1/r, homogeneous of degree -1 in length, so
    tr W = E_elec - sum q^2/(2 sigma sqrt pi); cubic symmetry makes W
    isotropic."""
    a = 6.0
    pos, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                pos.append([i * a / 2, j * a / 2, k * a / 2])
                q.append((-1.0) ** (i + j + k))
    pos, q = np.array(pos), np.array(q)
    sig = np.full(8, 0.05)
    W = ewald.virial(pos, np.eye(3) * a, sig, q, eta=0.8)
    E = ewald.coulomb_matrix(pos, np.eye(3) * a, sig, eta=0.8)
    e_point = 0.5 * q @ E @ q - np.sum(q * q / (2 * sig * SQRTPI))
    assert abs(np.trace(W) - e_point) < 1e-11 * abs(e_point)
    assert np.abs(W - np.trace(W) / 3 * np.eye(3)).max() < 1e-11 * abs(e_point)


def test_qeq_virial_is_total_strain_derivative():
    """At the QEq solution the virial of E_elec at fixed q equals
    -dE_QEq/d eps with the charges re-solved at every strained geometry
    (stationarity on the constraint plane; J and chi do not depend on it)."""
    pos, cell, sigma, J, chi = _small_system(n=7, seed=13)
    q_tot = 0.5
    r = ewald.qeq_dense(pos, cell, sigma, J, chi, q_tot, forces=False)
    W = ewald.virial(pos, cell, sigma, r.q)

    def e_qeq(F):
        p2, c2 = ewald.strained(pos, cell, F)
        return ewald.qeq_dense(p2, c2, sigma, J, chi, q_tot, forces=False).e_qeq

    fd = _strain_fd(e_qeq)
    assert np.abs(W - fd).max() < 1e-8 * np.abs(W).max()


@pytest.mark.parametrize("which", ["64", "tri"])
def test_matfree_virial_matches_dense(which):
    if which == "64":
        s = gen.system_64()
        q = _charges(s.n, 0.0, 6)
    else:
        s = gen.batch_structure(7)
        q = _charges(s.n, s.q_tot, 6)
    Wd = ewald.virial(s.pos, s.cell, s.sigma, q)
    Wm = matfree.EwaldOperator(s.pos, s.cell, s.sigma).virial(q)
    assert np.abs(Wm - Wd).max() < 1e-11 * np.abs(Wd).max()


def test_virial_pins_catch_planted_mistakes(monkeypatch):
    pos, cell, sigma, _, _, _ = small_triclinic(n=6, seed=7)
    q = _charges(6, 1.0, 4)
    fd = _strain_fd(lambda F: _energy_at_strain(pos, cell, sigma, q, F))
    scale = np.abs(fd).max()

    def err():
        return np.abs(ewald.virial(pos, cell, sigma, q) - fd).max() / scale

    assert err() < 1e-8
    # (1) the screening Gaussian's own strain dependence left out
    orig = ewald.kspace_strain_factor
    monkeypatch.setattr(ewald, "kspace_strain_factor", lambda k, k2, e: orig(k, k2, 0.0))
    assert err() > 1e-3
    monkeypatch.setattr(ewald, "kspace_strain_factor", orig)
    # (2) the volume derivative of the k-space prefactor dropped
    monkeypatch.setattr(ewald, "kspace_strain_factor", lambda k, k2, e: orig(k, k2, e) + np.eye(3))
    assert err() > 1e-3
    monkeypatch.setattr(ewald, "kspace_strain_factor", orig)
    # (3) the background's volume dependence dropped (charged cell)
    orig_bg = ewald.background_energy
    monkeypatch.setattr(ewald, "background_energy", lambda *a: 0.0)
    assert err() > 1e-3
    monkeypatch.setattr(ewald, "background_energy", orig_bg)


def test_real_space_pairs_tree_equals_all_pairs():
    """The k-d tree search of the oracle's real-space pair table returns the
    same pairs and displacements as the all-pairs minimum-image loop."""
    from oracle import matfree
    s = gen.system_512()
    for r in (9.0, 11.0, 15.0):
        a = matfree.real_space_pairs(s.pos, s.cell, r, tree=True)
        b = matfree.real_space_pairs(s.pos, s.cell, r, tree=False)
        ka = np.lexsort((a[1], a[0]))
        kb = np.lexsort((b[1], b[0]))
        assert len(ka) == len(kb) > 0
        assert np.array_equal(a[0][ka], b[0][kb]) and np.array_equal(a[1][ka], b[1][kb])
        assert np.abs(a[2][ka] - b[2][kb]).max() == 0.0
