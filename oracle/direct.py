"""Independent reference formulas used to pin the Ewald oracle (test infrastructure only).

* ``nonperiodic_matrix``  -- the paper's Coulomb kernel between normalised
  Gaussians, written out literally (Electrostatics and Charge Equilibration
  section, the E_ij cases after eq. elec_energy).
* ``planewave_energy``    -- the periodic energy as a plain sum over reciprocal
  vectors of |Q(k)|^2 / k^2 with Gaussian form factors (Electrostatics Solvers
  section: the potential is obtained from Poisson's equation in Fourier space
  with kernel 4 pi / G^2).  No Ewald split, no real-space term.
* ``brute_force_qeq``     -- minimises E_QEq = 1/2 q^T A q + chi.q on the
  plane sum(q) = Q_tot by pairwise charge-transfer line searches (eq.
  qeq_energy; the constraint of eq. 4G_qeq_prime), with no linear solve.
* ``two_atom_charges``    -- closed-form solution for two atoms.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRTPI = math.sqrt(math.pi)


def nonperiodic_matrix(pos, sigma):
    """E_ii = 1/(sigma_i sqrt(pi)), E_ij = erf(r_ij/(sqrt2 gamma_ij))/r_ij."""
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    gam = np.sqrt(sigma[:, None] ** 2 + sigma[None, :] ** 2)
    n = pos.shape[0]
    E = np.zeros((n, n))
    off = ~np.eye(n, dtype=bool)
    E[off] = erf(r[off] / (math.sqrt(2.0) * gam[off])) / r[off]
    E[np.diag_indices(n)] = 1.0 / (sigma * SQRTPI)
    return E


def planewave_energy(q, pos, cell, sigma, k_max=None):
    """(2 pi / V) sum_{k != 0} |sum_j q_j e^{-sigma_j^2 k^2 / 2} e^{i k.r_j}|^2 / k^2.

    Summed over every reciprocal vector with |k| <= k_max (default: the
    Gaussian form factor of the narrowest charge falls below ~1e-19).
    """
    q = np.asarray(q, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    H = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(H))
    recip = 2.0 * math.pi * np.linalg.inv(H).T
    if k_max is None:
        k_max = 9.5 / float(sigma.min())
    lengths = np.linalg.norm(H, axis=1)
    mmax = [int(math.ceil(k_max * l / (2 * math.pi))) + 1 for l in lengths]
    total = 0.0
    m1 = np.arange(-mmax[0], mmax[0] + 1)
    for a in m1:
        m23 = np.stack(np.meshgrid(np.arange(-mmax[1], mmax[1] + 1),
                                   np.arange(-mmax[2], mmax[2] + 1), indexing="ij"),
                       axis=-1).reshape(-1, 2)
        m = np.concatenate([np.full((m23.shape[0], 1), a), m23], axis=1)
        k = m @ recip
        k2 = (k * k).sum(1)
        keep = (k2 > 0) & (k2 <= k_max * k_max)
        k, k2 = k[keep], k2[keep]
        if k.size == 0:
            continue
        form = np.exp(-0.5 * np.outer(sigma * sigma, k2))
        ph = pos @ k.T
        qr = (q[:, None] * form * np.cos(ph)).sum(0)
        qi = (q[:, None] * form * np.sin(ph)).sum(0)
        total += np.sum((qr * qr + qi * qi) / k2)
    return 2.0 * math.pi / vol * total


def brute_force_qeq(A, chi, q_tot, tol=1e-14, max_moves=1000000):
    """Minimise 1/2 q^T A q + chi.q on sum(q) = q_tot by pairwise transfers.

    Starts from the uniform distribution q_tot/N and repeatedly moves, between
    the pair (i, j) with the lowest and highest energy gradient, the amount of
    charge that minimises the energy along that transfer line.  Stops when the
    gradient spread max(g) - min(g) (zero exactly at the constrained minimum)
    falls below ``tol``.  No linear system is solved.
    """
    A = np.asarray(A, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    n = A.shape[0]
    q = np.full(n, q_tot / n)
    g = A @ q + chi
    dA = np.diag(A)
    for _ in range(max_moves):
        i = int(np.argmin(g))
        j = int(np.argmax(g))
        if g[j] - g[i] <= tol:
            break
        curv = dA[i] + dA[j] - 2.0 * A[i, j]
        delta = (g[j] - g[i]) / curv           # move delta from j to i
        q[i] += delta
        q[j] -= delta
        g = A @ q + chi                        # recompute: no drift
    return q


def two_atom_charges(E, J, chi):
    """q1 = -q2 = (chi2 - chi1) / (J1 + J2 + E11 + E22 - 2 E12) for Q_tot = 0."""
    num = chi[1] - chi[0]
    den = J[0] + J[1] + E[0, 0] + E[1, 1] - 2.0 * E[0, 1]
    q1 = num / den
    return np.array([q1, -q1])
