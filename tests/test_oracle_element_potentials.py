"""Pins of the element-resolved potentials Gamma_i^z (ee4G embedding features).

Gamma_i^z is the potential at atom i of the equilibrated charges of element
z, without the atom's own Gaussian self term.  Pinned against: central
differences of the plain plane-wave energy (an independent formula with no
Ewald split), a scalar loop over the paper's non-periodic kernel, the
stationarity of the QEq solution (sum over z of Gamma_i^z + q_i/(sigma_i
sqrt(pi)) + J_i q_i + chi_i = mu for every atom), and a planted mistake.
"""
import math

import numpy as np

from inputs import gen
from oracle import direct, ewald

SQRTPI = math.sqrt(math.pi)


def small_triclinic(n=7, seed=9):
    rng = np.random.default_rng(seed)
    cell = np.array([[9.5, 0.0, 0.0], [1.2, 8.8, 0.0], [-0.8, 1.7, 10.3]])
    pos = rng.uniform(0, 1, (n, 3)) @ cell
    species = rng.integers(0, 3, n)
    sigma = np.array([1.0, 1.3, 1.7])[species]
    J = np.array([0.3, 0.45, 0.6])[species]
    chi = np.array([0.1, 0.0, -0.1])[species] + rng.normal(0, 0.05, n)
    return pos, cell, species, sigma, J, chi


def test_periodic_against_planewave_differences():
    pos, cell, species, sigma, J, chi = small_triclinic()
    res = ewald.qeq_dense(pos, cell, sigma, J, chi, 1.0)
    G = ewald.element_potentials(pos, cell, sigma, res.q, species, 3)
    h = 1e-3
    for z in range(3):
        v = res.q * (species == z)
        for i in (0, 3, 6):
            e = []
            for sgn in (1, -1):
                w = v.copy()
                w[i] += sgn * h
                e.append(direct.planewave_energy(w, pos, cell, sigma))
            phi = (e[0] - e[1]) / (2 * h)   # (E v)_i: exact for a quadratic form
            ref = phi - (species[i] == z) * res.q[i] / (sigma[i] * SQRTPI)
            assert abs(G[i, z] - ref) < 1e-10


def test_nonperiodic_scalar_loop():
    s = gen.cluster_system(9, q_tot=1.0, seed=3)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, 1.0)
    G = direct.element_potentials_nonperiodic(s.pos, s.sigma, res.q, s.species, 2)
    for i in range(s.n):
        for z in range(2):
            acc = 0.0
            for j in range(s.n):
                if j == i or s.species[j] != z:
                    continue
                r = math.dist(s.pos[i], s.pos[j])
                g = math.sqrt(s.sigma[i] ** 2 + s.sigma[j] ** 2)
                acc += math.erf(r / (math.sqrt(2.0) * g)) / r * res.q[j]
            assert abs(G[i, z] - acc) < 1e-14


def test_stationarity_sum_rule():
    for q_tot in (0.0, 1.0):
        pos, cell, species, sigma, J, chi = small_triclinic(n=8, seed=21)
        res = ewald.qeq_dense(pos, cell, sigma, J, chi, q_tot)
        G = ewald.element_potentials(pos, cell, sigma, res.q, species, 3)
        lhs = G.sum(1) + res.q / (sigma * SQRTPI) + J * res.q + chi
        assert np.abs(lhs - res.mu).max() < 1e-12
    s = gen.cluster_system(30, q_tot=-1.0, seed=8)
    res = direct.qeq_nonperiodic(s.pos, s.sigma, s.J, s.chi, -1.0)
    G = direct.element_potentials_nonperiodic(s.pos, s.sigma, res.q, s.species, 2)
    lhs = G.sum(1) + res.q / (s.sigma * SQRTPI) + s.J * res.q + s.chi
    assert np.abs(lhs - res.mu).max() < 1e-12


def test_planted_self_term_is_caught():
    pos, cell, species, sigma, J, chi = small_triclinic(n=8, seed=21)
    res = ewald.qeq_dense(pos, cell, sigma, J, chi, 1.0)
    E = ewald.coulomb_matrix(pos, cell, sigma)
    wrong = np.stack([E @ (res.q * (species == z)) for z in range(3)], 1)   # self term kept
    lhs = wrong.sum(1) + res.q / (sigma * SQRTPI) + J * res.q + chi
    assert np.abs(lhs - res.mu).max() > 1e-3
