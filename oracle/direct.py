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
* ``qeq_nonperiodic``     -- QEq of an isolated system (no cell): the bordered
  system of eq. 4G_qeq_prime with the paper's non-periodic kernel written
  out, charges by Gaussian elimination (or projected CG on the same dense
  matrix for large N), energies of eq. qeq_energy and analytic forces
  F_k = -q_k sum_j q_j K'(r_kj) (r_k - r_j) / r_kj (the SI force expression
  at constant chi and J).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRTPI = math.sqrt(math.pi)


def nonperiodic_kernel(r, gamma):
    """K(r) = erf(r / (sqrt2 gamma)) / r, with its r -> 0 limit sqrt(2/pi) / gamma.

    Below 1e-4 bohr the series 2a/sqrt(pi) (1 - (a r)^2 / 3), a = 1/(sqrt2 gamma).
    """
    r = np.asarray(r, dtype=np.float64)
    a = 1.0 / (math.sqrt(2.0) * np.asarray(gamma, dtype=np.float64))
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    return np.where(small, 2.0 / SQRTPI * a * (1.0 - (a * r) ** 2 / 3.0), erf(a * rs) / rs)


def nonperiodic_kernel_deriv(r, gamma):
    """dK/dr of ``nonperiodic_kernel``: (2a/sqrt(pi)) exp(-(a r)^2) / r - K / r (0 at r = 0)."""
    r = np.asarray(r, dtype=np.float64)
    a = 1.0 / (math.sqrt(2.0) * np.asarray(gamma, dtype=np.float64))
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    d = (2.0 / SQRTPI * a * np.exp(-(a * rs) ** 2) - erf(a * rs) / rs) / rs
    return np.where(small, -4.0 / (3.0 * SQRTPI) * a ** 3 * r, d)


def nonperiodic_matrix(pos, sigma):
    """E_ii = 1/(sigma_i sqrt(pi)), E_ij = erf(r_ij/(sqrt2 gamma_ij))/r_ij."""
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    gam = np.sqrt(sigma[:, None] ** 2 + sigma[None, :] ** 2)
    n = pos.shape[0]
    E = nonperiodic_kernel(r, gam)
    E[np.diag_indices(n)] = 1.0 / (sigma * SQRTPI)
    return E


def nonperiodic_gradient(pos, sigma, q):
    """d/dr_k of E_elec = 1/2 q^T E q: sum_j q_k q_j K'(r_kj) (r_k - r_j) / r_kj."""
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    gam = np.sqrt(sigma[:, None] ** 2 + sigma[None, :] ** 2)
    np.fill_diagonal(r, 1.0)
    # K'(r) / r; below 1e-4 bohr its limit -4 a^3 / (3 sqrt(pi)) (finite at r = 0)
    a = 1.0 / (math.sqrt(2.0) * gam)
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    w = np.where(small, -4.0 / (3.0 * SQRTPI) * a ** 3, nonperiodic_kernel_deriv(rs, gam) / rs)
    np.fill_diagonal(w, 0.0)
    w *= np.outer(q, q)
    return (w[:, :, None] * d).sum(1)


def qeq_nonperiodic(pos, sigma, J, chi, q_tot, forces=True, method="dense", tol=1e-12):
    """QEq of an isolated system: charges, mu, E_QEq, E_elec and forces.

    method="dense": the bordered system by the oracle's Gaussian elimination;
    method="cg": Jacobi-projected CG on the same dense matrix (large N).
    Forces are -dE_QEq/dr at the solution = -dE_elec/dr at fixed q.
    """
    from . import ewald, matfree
    J = np.asarray(J, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    E = nonperiodic_matrix(pos, sigma)
    if method == "dense":
        q, lam = ewald.solve_qeq(E, J, chi, q_tot)
        mu = -lam
    else:
        A = E + np.diag(J)
        q, mu, _, _ = matfree.projected_cg(lambda v: A @ v, np.diag(A).copy(), chi, q_tot, tol=tol)
    e_qeq, e_elec = ewald.qeq_energy(E, J, chi, q)
    res = ewald.QEqResult(q=q, mu=mu, lam=-mu, e_qeq=e_qeq, e_elec=e_elec, E=E)
    if forces:
        res["forces"] = -nonperiodic_gradient(pos, sigma, q)
    return res


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


def element_potentials_nonperiodic(pos, sigma, q, species, n_elem):
    """Gamma_i^z of an isolated system: sum over atoms j != i of element z of
    erf(r_ij / (sqrt2 gamma_ij)) / r_ij q_j (the paper's kernel)."""
    from . import ewald
    return ewald._element_potentials_from(nonperiodic_matrix(pos, sigma), sigma, q, species, n_elem)
