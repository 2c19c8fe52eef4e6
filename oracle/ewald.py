"""Dense FP64 Ewald oracle for periodic Gaussian-charge QEq (test infrastructure only).

Quantity (Electrostatics and Charge Equilibration section, eq. elec_energy and
the Coulomb kernel E_ij that follows it; Electrostatics Solvers section, eq.
matvec): the electrostatic energy of normalised Gaussian charges
rho_i(r) = (2 pi sigma_i^2)^(-3/2) exp(-r^2 / 2 sigma_i^2) in a periodic cell
with a neutralising background and tin-foil boundary,

    E_elec(q) = (2 pi / V) sum_{k != 0} |sum_j q_j exp(-sigma_j^2 k^2 / 2) exp(i k.r_j)|^2 / k^2,

whose non-periodic limit is the paper's kernel E_ii = 1/(sigma_i sqrt(pi)),
E_ij = erf(r_ij / (sqrt(2) gamma_ij)) / r_ij, gamma_ij = sqrt(sigma_i^2 + sigma_j^2).

Algorithm (SI, Ewald Summation section): split with a screening Gaussian of
standard deviation ``eta`` into

  real space  K_ij(r) = [erf(r/(sqrt2 gamma_ij)) - erf(r/(sqrt2 eta))] / r over
              all lattice images (skipping i = j in the home cell),
  k space     (4 pi / V) exp(-eta^2 k^2 / 2) / k^2 cos(k.(r_i - r_j)), k != 0,
  self        1/(sigma_i sqrt(pi)) - sqrt(2/pi)/eta on the diagonal,
  background  -(2 pi / V)(eta^2 - sigma_i^2 - sigma_j^2) on every element
              (the k -> 0 remainder of the split; it makes A independent of eta
              for charged cells and drops out of the energy when Q_tot = 0).

QEq (eq. qeq_energy, eq. 4G_qeq_prime; SI eq. qeq): A = E + diag(J) and

    [A 1; 1^T 0] [q; lam] = [-chi; Q_tot],

solved by Gaussian elimination with partial pivoting (Electrostatics Solvers
section: the direct O(N^3) factorisation).  The SI writes the same system as
(A + J) q = -chi + mu 1, so mu = -lam.

Units: bohr, Hartree, e.  Cells are 3x3 with ROWS = lattice vectors.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
SQRTPI = math.sqrt(math.pi)
TWO_OVER_SQRTPI = 2.0 / SQRTPI

# Truncation of both Ewald sums: the neglected tails are ~erfc(6.5) ~ 4e-20
# relative to the retained terms.
TAIL_X = 6.5


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------

def cell_geometry(cell):
    """Volume, inverse cell, reciprocal rows (with 2 pi) and face-to-face widths."""
    H = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(H))
    if not vol > 0.0:
        raise ValueError("singular cell")
    Hinv = np.linalg.inv(H)
    recip = 2.0 * math.pi * Hinv.T          # row a: b_a with a_b . b_a = 2 pi delta
    widths = 2.0 * math.pi / np.linalg.norm(recip, axis=1)
    return vol, Hinv, recip, widths


def default_cutoffs(eta, gamma_max):
    """Real-space radius and k cutoff for which both tails are ~erfc(6.5)."""
    r_max = TAIL_X * SQRT2 * max(eta, gamma_max)
    k_max = TAIL_X * SQRT2 / eta
    return r_max, k_max


def lattice_shifts(cell, r_max):
    """All integer shifts n whose image n.H can lie within r_max of a home-cell pair."""
    _, _, _, widths = cell_geometry(cell)
    nmax = [int(math.ceil(r_max / w)) + 1 for w in widths]
    rng = [np.arange(-m, m + 1) for m in nmax]
    n = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    return n


def half_space_kvectors(cell, k_max):
    """Reciprocal vectors k = m.B with 0 < |k| <= k_max, one of each +-k pair."""
    _, _, recip, _ = cell_geometry(cell)
    H = np.asarray(cell, dtype=np.float64)
    lengths = np.linalg.norm(H, axis=1)
    mmax = [int(math.ceil(k_max * l / (2.0 * math.pi))) + 1 for l in lengths]
    rng = [np.arange(-m, m + 1) for m in mmax]
    m = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    pos_half = (m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0)) | \
               ((m[:, 0] == 0) & (m[:, 1] == 0) & (m[:, 2] > 0))
    m = m[pos_half]
    k = m @ recip
    k2 = np.einsum("ij,ij->i", k, k)
    keep = k2 <= k_max * k_max
    return k[keep], k2[keep]


# ---------------------------------------------------------------------------
# Pair kernel
# ---------------------------------------------------------------------------

def pair_kernel(r, gamma, eta):
    """K(r) = [erf(r/(sqrt2 gamma)) - erf(r/(sqrt2 eta))]/r with its r -> 0 limit."""
    r = np.asarray(r, dtype=np.float64)
    a = 1.0 / (SQRT2 * gamma)
    b = 1.0 / (SQRT2 * eta)
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    out = (erf(a * rs) - erf(b * rs)) / rs
    series = TWO_OVER_SQRTPI * ((a - b) - (a ** 3 - b ** 3) * r * r / 3.0)
    return np.where(small, series, out)


def pair_kernel_deriv(r, gamma, eta):
    """dK/dr of ``pair_kernel`` (0 at r = 0)."""
    r = np.asarray(r, dtype=np.float64)
    a = 1.0 / (SQRT2 * gamma)
    b = 1.0 / (SQRT2 * eta)
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    d = (TWO_OVER_SQRTPI * (a * np.exp(-(a * rs) ** 2) - b * np.exp(-(b * rs) ** 2))
         - (erf(a * rs) - erf(b * rs)) / rs) / rs
    series = -TWO_OVER_SQRTPI * 2.0 * (a ** 3 - b ** 3) * r / 3.0
    return np.where(small, series, d)


# ---------------------------------------------------------------------------
# Dense Coulomb matrix by Ewald summation
# ---------------------------------------------------------------------------

def _real_space(pos, cell, sigma, eta, r_max, want="matrix", q=None, a=None):
    """Real-space Ewald sum over images.

    want="matrix": N x N matrix sum_n K_ij(|r_i - r_j + n.H|).
    want="grad"  : d/dr_i of (1/2) q^T K q (or of a^T K q if ``a`` is given).
    """
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    H = np.asarray(cell, dtype=np.float64)
    sig2 = sigma * sigma
    gam = np.sqrt(sig2[:, None] + sig2[None, :])
    dr0 = pos[:, None, :] - pos[None, :, :]
    eye = np.eye(n, dtype=bool)
    out = np.zeros((n, n)) if want == "matrix" else np.zeros((n, 3))
    for s in lattice_shifts(H, r_max):
        d = dr0 + s @ H
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        mask = r < r_max
        if (s == 0).all():
            mask &= ~eye
        if not mask.any():
            continue
        if want == "matrix":
            kk = np.zeros((n, n))
            kk[mask] = pair_kernel(r[mask], gam[mask], eta)
            out += kk
        else:
            mask &= ~eye      # i = j images do not move with r_i
            dk = np.zeros((n, n))
            rr = np.where(mask, r, 1.0)
            dk[mask] = pair_kernel_deriv(r[mask], gam[mask], eta) / rr[mask]
            if a is None:
                coef = q[:, None] * q[None, :] * dk
            else:
                coef = (a[:, None] * q[None, :] + q[:, None] * a[None, :]) * dk
            out += np.einsum("ij,ijk->ik", coef, d)
    return out


def _kspace_tables(pos, kvec, chunk=4096):
    """Yield (k chunk, cos(k.r) (N,nk), sin(k.r) (N,nk))."""
    for s in range(0, kvec.shape[0], chunk):
        kc = kvec[s:s + chunk]
        ph = pos @ kc.T
        yield s, kc, np.cos(ph), np.sin(ph)


def kspace_weights(k2, vol, eta):
    """Half-space weights 2 (4 pi / V) exp(-eta^2 k^2 / 2) / k^2."""
    return 2.0 * (4.0 * math.pi / vol) * np.exp(-0.5 * eta * eta * k2) / k2


def coulomb_matrix(pos, cell, sigma, eta=None, r_max=None, k_max=None):
    """Dense periodic Coulomb matrix E (without J) by Ewald summation.

    Follows SI Ewald Summation (real + reciprocal + self) with the background
    term described in the module docstring.  ``eta`` is the oracle's own split
    width; the result does not depend on it (checked by the pins).
    """
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    vol, _, _, _ = cell_geometry(cell)
    gmax = SQRT2 * float(sigma.max())
    if eta is None:
        eta = default_eta(pos.shape[0], vol, gmax)
    rm, km = default_cutoffs(eta, gmax)
    r_max = rm if r_max is None else r_max
    k_max = km if k_max is None else k_max
    A = _real_space(pos, cell, sigma, eta, r_max)
    kvec, k2 = half_space_kvectors(cell, k_max)
    w = kspace_weights(k2, vol, eta)
    for s, _, c, sn in _kspace_tables(pos, kvec):
        ww = w[s:s + c.shape[1]]
        A += (c * ww) @ c.T + (sn * ww) @ sn.T
    A[np.diag_indices_from(A)] += 1.0 / (sigma * SQRTPI) - math.sqrt(2.0 / math.pi) / eta
    sig2 = sigma * sigma
    A -= (2.0 * math.pi / vol) * (eta * eta - sig2[:, None] - sig2[None, :])
    return A


def default_eta(n, vol, gamma_max):
    """A split width that keeps the dense sums cheap (any value gives the same A)."""
    return max(0.5 * gamma_max, min(2.0, 0.35 * (vol / max(n, 1)) ** (1.0 / 3.0)))


def energy_gradient_positions(pos, cell, sigma, q, eta=None, a=None):
    """d/dr of E_elec = (1/2) q^T E q at fixed q (or of a^T E q if ``a`` given).

    Analytic derivative of the real- and k-space Ewald terms (SI Ewald
    Summation: the influence matrix and its position derivatives come from the
    same Ewald framework).  Self and background terms do not depend on r.
    """
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    vol, _, _, _ = cell_geometry(cell)
    gmax = SQRT2 * float(sigma.max())
    if eta is None:
        eta = default_eta(pos.shape[0], vol, gmax)
    r_max, k_max = default_cutoffs(eta, gmax)
    g = _real_space(pos, cell, sigma, eta, r_max, want="grad", q=q, a=a)
    kvec, k2 = half_space_kvectors(cell, k_max)
    w = kspace_weights(k2, vol, eta)
    for s, kc, c, sn in _kspace_tables(pos, kvec):
        ww = w[s:s + c.shape[1]]
        Cq, Sq = q @ c, q @ sn
        if a is None:
            # d/dr_i (1/2) sum_k w (Cq^2 + Sq^2) = sum_k w k q_i (c_i Sq - s_i Cq)
            coef = q[:, None] * (c * (ww * Sq) - sn * (ww * Cq))
        else:
            Ca, Sa = a @ c, a @ sn
            coef = (a[:, None] * (c * (ww * Sq) - sn * (ww * Cq))
                    + q[:, None] * (c * (ww * Sa) - sn * (ww * Ca)))
        g += coef @ kc
    return g


# ---------------------------------------------------------------------------
# Bordered system: Gaussian elimination with partial pivoting
# ---------------------------------------------------------------------------

def gauss_solve(M, b):
    """Solve M x = b by Gaussian elimination with partial pivoting (FP64).

    Plain textbook elimination written out; the tests cross-check it against
    LAPACK's dgesv.
    """
    M = np.array(M, dtype=np.float64, copy=True)
    b = np.array(b, dtype=np.float64, copy=True)
    n = M.shape[0]
    for col in range(n):
        piv = col + int(np.argmax(np.abs(M[col:, col])))
        if M[piv, col] == 0.0:
            raise np.linalg.LinAlgError("singular bordered matrix")
        if piv != col:
            M[[col, piv]] = M[[piv, col]]
            b[[col, piv]] = b[[piv, col]]
        f = M[col + 1:, col] / M[col, col]
        M[col + 1:, col:] -= f[:, None] * M[col, col:][None, :]
        b[col + 1:] -= f * b[col]
    x = np.zeros(n)
    for row in range(n - 1, -1, -1):
        x[row] = (b[row] - M[row, row + 1:] @ x[row + 1:]) / M[row, row]
    return x


def bordered_matrix(A):
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    return M


def solve_qeq(E, J, chi, q_tot, solver=gauss_solve):
    """Charges and Lagrange multiplier from eq. 4G_qeq_prime.

    Returns (q, lam) with [E + diag(J), 1; 1^T, 0][q; lam] = [-chi; Q_tot].
    """
    A = E + np.diag(np.asarray(J, dtype=np.float64))
    rhs = np.concatenate([-np.asarray(chi, dtype=np.float64), [float(q_tot)]])
    x = solver(bordered_matrix(A), rhs)
    return x[:-1], x[-1]


def qeq_energy(E, J, chi, q):
    """E_QEq = E_elec + chi.q + (1/2) sum J q^2 (SI, 4G section; eq. qeq_energy)."""
    e_elec = 0.5 * q @ (E @ q)
    return e_elec + chi @ q + 0.5 * np.sum(J * q * q), e_elec


class QEqResult(dict):
    __getattr__ = dict.__getitem__


def qeq_dense(pos, cell, sigma, J, chi, q_tot, eta=None, forces=True, solver=gauss_solve):
    """Full oracle solve: charges, mu, E_QEq, E_elec and forces.

    Forces are -dE_QEq/dr at the solution.  Because E_QEq is stationary in q
    on the constraint plane, they equal -dE_elec/dr at fixed q (the "force
    trick" of the SI 4G section needs no extra solve for the QEq energy
    itself).
    """
    E = coulomb_matrix(pos, cell, sigma, eta=eta)
    q, lam = solve_qeq(E, J, chi, q_tot, solver=solver)
    e_qeq, e_elec = qeq_energy(E, np.asarray(J), np.asarray(chi), q)
    res = QEqResult(q=q, lam=lam, mu=-lam, e_qeq=e_qeq, e_elec=e_elec, E=E)
    if forces:
        res["forces"] = -energy_gradient_positions(pos, cell, sigma, q, eta=eta)
    return res


def qeq_adjoint(pos, cell, sigma, J, chi, q_tot, dL_dq, dL_dEelec=0.0, dL_dEqeq=0.0,
                eta=None, solver=gauss_solve):
    """Gradient of a loss L(q, E_elec, E_QEq) through the QEq solve.

    Lagrange / adjoint route of the SI 4G section (eq. 4g_force_trick): one
    extra solve of the (symmetric) bordered system

        [A 1; 1^T 0][a; nu] = [g; 0],  g = dL/dq + dL/dE_elec * (E q),

    then dL/dchi = -a + dL/dE_QEq * q, dL/dJ = -a q + dL/dE_QEq q^2 / 2 and
    dL/dr = (dL/dE_elec + dL/dE_QEq) dE_elec/dr|_q - d(a^T E q)/dr|_{a,q}.
    The term dE_QEq/dq = mu 1 is orthogonal to every feasible dq and drops out.
    Returns (q, dL_dchi, dL_dpos, dL_dJ).
    """
    pos = np.asarray(pos, dtype=np.float64)
    E = coulomb_matrix(pos, cell, sigma, eta=eta)
    q, _ = solve_qeq(E, J, chi, q_tot, solver=solver)
    g = np.asarray(dL_dq, dtype=np.float64) + dL_dEelec * (E @ q)
    A = E + np.diag(np.asarray(J, dtype=np.float64))
    x = solver(bordered_matrix(A), np.concatenate([g, [0.0]]))
    a = x[:-1]
    dchi = -a + dL_dEqeq * q
    dJ = -a * q + 0.5 * dL_dEqeq * q * q
    de_dr = energy_gradient_positions(pos, cell, sigma, q, eta=eta)
    bil = energy_gradient_positions(pos, cell, sigma, q, eta=eta, a=a)
    dpos = (dL_dEelec + dL_dEqeq) * de_dr - bil
    return q, dchi, dpos, dJ


# ---------------------------------------------------------------------------
# Virial (strain derivative of the energy)
# ---------------------------------------------------------------------------

def background_energy(cell, sigma, q, eta):
    """E_bg = (1/2) q^T B q with B_ij = -(2 pi / V)(eta^2 - sigma_i^2 - sigma_j^2)."""
    vol, _, _, _ = cell_geometry(cell)
    q = np.asarray(q, dtype=np.float64)
    qt = q.sum()
    return -(math.pi / vol) * (eta * eta * qt * qt - 2.0 * qt * np.sum(q * sigma * sigma))


def kspace_strain_factor(kvec, k2, eta):
    """d ln(e^{-eta^2 k^2/2} / (V k^2)) / d eps_ab, per k: -delta_ab + 2 (1/k^2 + eta^2/2) k_a k_b.

    Under r -> (1 + eps) r every k.r is unchanged, so k -> (1 + eps)^{-T} k
    and d(k^2)/d eps_ab = -2 k_a k_b, while dV/d eps_ab = V delta_ab.
    """
    c = 2.0 * (1.0 / k2 + 0.5 * eta * eta)
    return -np.eye(3)[None, :, :] + c[:, None, None] * kvec[:, :, None] * kvec[:, None, :]


def virial(pos, cell, sigma, q, eta=None):
    """W_ab = -dE_elec/d eps_ab at fixed q (3 x 3, symmetric).

    The strain acts on positions and lattice vectors alike (r -> (1 + eps) r,
    fractional coordinates fixed).  The SI's Stress Tensor subsection defines
    the stress as sigma = (1/V) dE/d eps and the virial handed to an MD code
    as -V sigma, which is this W; the Electrostatics Solvers section obtains
    it from the same Fourier-space machinery as the forces.  Term by term from
    the same Ewald split as ``coulomb_matrix``:

      real space  -(1/2) sum_{i,j,n} q_i q_j K'(r)/r d_a d_b,  d = r_i - r_j + n.H,
      k space     -sum_k E_k [-delta_ab + 2 (1/k^2 + eta^2/2) k_a k_b],
                  E_k = (1/2) (4 pi / V) e^{-eta^2 k^2/2} / k^2 |S(k)|^2,
      self        none (no length enters it),
      background  E_bg delta_ab (E_bg is proportional to 1/V).

    The total does not depend on eta (pinned by the tests).
    """
    pos = np.asarray(pos, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    H = np.asarray(cell, dtype=np.float64)
    n = pos.shape[0]
    vol, _, _, _ = cell_geometry(H)
    gmax = SQRT2 * float(sigma.max())
    if eta is None:
        eta = default_eta(n, vol, gmax)
    r_max, k_max = default_cutoffs(eta, gmax)
    W = np.zeros((3, 3))
    # real space
    sig2 = sigma * sigma
    gam = np.sqrt(sig2[:, None] + sig2[None, :])
    dr0 = pos[:, None, :] - pos[None, :, :]
    eye = np.eye(n, dtype=bool)
    qq = q[:, None] * q[None, :]
    for s in lattice_shifts(H, r_max):
        d = dr0 + s @ H
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        mask = r < r_max
        if (s == 0).all():
            mask &= ~eye
        if not mask.any():
            continue
        c = np.zeros((n, n))
        c[mask] = qq[mask] * pair_kernel_deriv(r[mask], gam[mask], eta) / r[mask]
        W -= 0.5 * np.einsum("ij,ija,ijb->ab", c, d, d)
    # k space (half space, weights doubled)
    kvec, k2 = half_space_kvectors(H, k_max)
    w = kspace_weights(k2, vol, eta)
    for s, kc, cs, sn in _kspace_tables(pos, kvec):
        ww = w[s:s + cs.shape[1]]
        Cq, Sq = q @ cs, q @ sn
        ek = 0.5 * ww * (Cq * Cq + Sq * Sq)
        W -= np.einsum("k,kab->ab", ek, kspace_strain_factor(kc, k2[s:s + kc.shape[0]], eta))
    # background
    W += background_energy(H, sigma, q, eta) * np.eye(3)
    return W


def strained(pos, cell, F):
    """Positions and cell after the homogeneous deformation r -> F r (rows are vectors)."""
    F = np.asarray(F, dtype=np.float64)
    return np.asarray(pos, dtype=np.float64) @ F.T, np.asarray(cell, dtype=np.float64) @ F.T


# ---------------------------------------------------------------------------
# Element-resolved electrostatic potentials (ee4G embedding features)
# ---------------------------------------------------------------------------

def element_potentials(pos, cell, sigma, q, species, n_elem, eta=None):
    """Gamma_i^z: potential at atom i of the charges of element z, without the
    atom's own Gaussian self term (Electrostatics and Charge Equilibration
    section: the ee4G variant appends element-specific electrostatic
    potentials at each site, computed from the equilibrated charges).

    Gamma[:, z] = E (q * [s = z]) - [s_i = z] q_i / (sigma_i sqrt(pi)), with E
    the periodic Coulomb matrix (images, background) of ``coulomb_matrix``.
    """
    E = coulomb_matrix(pos, cell, sigma, eta=eta)
    return _element_potentials_from(E, sigma, q, species, n_elem)


def _element_potentials_from(E, sigma, q, species, n_elem):
    q = np.asarray(q, dtype=np.float64)
    species = np.asarray(species)
    sigma = np.asarray(sigma, dtype=np.float64)
    out = np.zeros((q.shape[0], n_elem))
    for z in range(n_elem):
        m = (species == z).astype(np.float64)
        out[:, z] = E @ (q * m) - m * q / (sigma * SQRTPI)
    return out
