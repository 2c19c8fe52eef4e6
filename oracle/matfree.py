"""Matrix-free FP64 Ewald oracle with projected CG (test infrastructure only).

The same Ewald split as ``oracle.ewald`` (real-space images + reciprocal sum +
self + background), applied to a vector without forming the N x N matrix, so
that systems of tens of thousands of atoms can be checked:

* the real-space part is a sparse FP64 matrix over all image pairs within the
  oracle's own cutoff;
* the reciprocal part uses per-axis phase tables exp(2 pi i m_a s_ja) in
  fractional coordinates (k.r = 2 pi m.s for any cell), contracted with
  ordinary complex matrix products;
* the solve is the paper's iterative route (Electrostatics Solvers section:
  conjugate gradients on eq. 4G_qeq_prime): CG restricted to the plane
  sum(q) = Q_tot, Jacobi-preconditioned, to a relative projected residual of
  1e-12 in FP64.

Parity: pinned to the dense oracle (Gaussian elimination) on the 64- and
512-atom systems by the tests; at 32,768 atoms it is the same arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import ewald

SQRTPI = math.sqrt(math.pi)


def _is_orthorhombic(H):
    return np.allclose(H - np.diag(np.diag(H)), 0.0)


def real_space_pairs(pos, cell, r_max, chunk=256, tree=True):
    """All (i, j, d = r_i - r_j + n.H) with |d| < r_max, excluding i = j, n = 0.

    Orthorhombic cells with r_max below half the shortest edge have at most
    one image per pair (the minimum image); there the candidate pairs come
    from scipy's periodic k-d tree (a library search, same pair set as the
    all-pairs loop below, which ``tree=False`` selects and a test compares),
    else every pair and image shift is tested directly."""
    pos = np.asarray(pos, dtype=np.float64)
    H = np.asarray(cell, dtype=np.float64)
    n = pos.shape[0]
    rows, cols, ds = [], [], []
    if tree and _is_orthorhombic(H) and r_max < 0.5 * np.diag(H).min():
        from scipy.spatial import cKDTree
        L = np.diag(H)
        wrapped = pos - L * np.floor(pos / L)
        wrapped[wrapped >= L] -= L[np.nonzero(wrapped >= L)[1]]
        ij = cKDTree(wrapped, boxsize=L).query_pairs(r_max, output_type="ndarray")
        i, j = ij[:, 0], ij[:, 1]
        d = pos[i] - pos[j]
        d -= L * np.round(d / L)
        keep = np.einsum("ij,ij->i", d, d) < r_max * r_max
        i, j, d = i[keep], j[keep], d[keep]
        return np.concatenate([i, j]), np.concatenate([j, i]), np.concatenate([d, -d])
    if _is_orthorhombic(H) and r_max < 0.5 * np.diag(H).min():
        # each pair has at most one image inside r_max: minimum image
        L = np.diag(H)
        for s in range(0, n, chunk):
            d = pos[s:s + chunk, None, :] - pos[None, :, :]
            d -= L * np.round(d / L)
            r2 = np.einsum("ijk,ijk->ij", d, d)
            ii, jj = np.nonzero(r2 < r_max * r_max)
            keep = (ii + s) != jj
            ii, jj = ii[keep], jj[keep]
            rows.append(ii + s)
            cols.append(jj)
            ds.append(d[ii, jj])
    else:
        shifts = ewald.lattice_shifts(H, r_max) @ H
        for s in range(0, n, chunk):
            d0 = pos[s:s + chunk, None, :] - pos[None, :, :]
            for t in shifts:
                d = d0 + t
                r2 = np.einsum("ijk,ijk->ij", d, d)
                ii, jj = np.nonzero(r2 < r_max * r_max)
                if not np.any(t):
                    keep = (ii + s) != jj
                    ii, jj = ii[keep], jj[keep]
                rows.append(ii + s)
                cols.append(jj)
                ds.append(d[ii, jj])
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(ds)


class EwaldOperator:
    """y = E v for the periodic Gaussian Coulomb matrix E, never formed."""

    def __init__(self, pos, cell, sigma, eta=None):
        self.pos = np.asarray(pos, dtype=np.float64)
        self.cell = np.asarray(cell, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        n = self.pos.shape[0]
        self.n = n
        vol, Hinv, recip, _ = ewald.cell_geometry(self.cell)
        self.vol = vol
        gmax = math.sqrt(2.0) * float(self.sigma.max())
        if eta is None:
            eta = self.balanced_eta(n, vol, gmax)
        self.eta = eta
        r_max, k_max = ewald.default_cutoffs(eta, gmax)
        self.r_max, self.k_max = r_max, k_max

        # --- real space: sparse K and dK/dr / r with displacement vectors
        ii, jj, d = real_space_pairs(self.pos, self.cell, r_max)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        gam = np.sqrt(self.sigma[ii] ** 2 + self.sigma[jj] ** 2)
        kv = ewald.pair_kernel(r, gam, eta)
        self.K = sp.csr_matrix((kv, (ii, jj)), shape=(n, n))
        self._pairs = (ii, jj, d, r, gam)

        # --- self and background
        self.diag_self = 1.0 / (self.sigma * SQRTPI) - math.sqrt(2.0 / math.pi) / eta
        self.sig2 = self.sigma ** 2

        # --- reciprocal space, separable phase tables in fractional coords
        s = self.pos @ Hinv
        lengths = np.linalg.norm(self.cell, axis=1)
        M = [int(math.ceil(k_max * l / (2 * math.pi))) + 1 for l in lengths]
        self.M = M
        m1 = np.arange(-M[0], M[0] + 1)
        m2 = np.arange(-M[1], M[1] + 1)
        m3 = np.arange(0, M[2] + 1)
        self.T1 = np.exp(2j * math.pi * np.outer(s[:, 0], m1))
        self.T2 = np.exp(2j * math.pi * np.outer(s[:, 1], m2))
        self.T3 = np.exp(2j * math.pi * np.outer(s[:, 2], m3))
        mm = np.stack(np.meshgrid(m1, m2, m3, indexing="ij"), axis=-1)
        k = mm @ recip                                   # (M1, M2, M3h, 3)
        k2 = np.einsum("...i,...i->...", k, k)
        with np.errstate(divide="ignore"):
            w = (4.0 * math.pi / vol) * np.exp(-0.5 * eta * eta * k2) / k2
        w[(k2 == 0) | (k2 > k_max * k_max)] = 0.0
        w[:, :, 1:] *= 2.0                               # m3 > 0 stands for +-m3
        # the m3 = 0 plane holds both m and -m explicitly
        self.W = w
        self.kvec = k
        self.active = [a for a in range(len(m1)) if np.any(w[a] != 0.0)]

    @staticmethod
    def balanced_eta(n, vol, gmax):
        # cost ~ real-space pairs (eta^3) vs reciprocal modes (eta^-3)
        return max(gmax, 0.55 * (vol / max(n, 1)) ** (1.0 / 3.0) * (n / 512.0) ** (1.0 / 6.0))

    # -- structure factor S(m) = sum_j v_j exp(2 pi i m.s_j)  (m3 >= 0 half)
    def structure_factor(self, v):
        S = np.zeros(self.W.shape, dtype=np.complex128)
        for a in self.active:
            X = v * self.T1[:, a]
            S[a] = self.T2.T @ (X[:, None] * self.T3)
        return S

    def _back(self, U):
        """sum_m exp(2 pi i m.s_i) U(m) for every atom i (complex)."""
        y = np.zeros(self.n, dtype=np.complex128)
        for a in self.active:
            P = self.T2 @ U[a]
            y += self.T1[:, a] * np.einsum("ij,ij->i", P, self.T3)
        return y

    def apply(self, v):
        """E v: real-space images + reciprocal + self + background."""
        v = np.asarray(v, dtype=np.float64)
        y = self.K @ v
        S = self.structure_factor(v)
        y += self._back(self.W * np.conj(S)).real
        y += self.diag_self * v
        y -= (2.0 * math.pi / self.vol) * ((self.eta ** 2 - self.sig2) * v.sum() - self.sig2 @ v)
        return y

    def grad_positions(self, q, a=None):
        """d/dr of (1/2) q^T E q at fixed q, or of a^T E q if ``a`` is given."""
        q = np.asarray(q, dtype=np.float64)
        ii, jj, d, r, gam = self._pairs
        dk = ewald.pair_kernel_deriv(r, gam, self.eta) / r
        if a is None:
            coef = q[ii] * q[jj] * dk
        else:
            coef = (a[ii] * q[jj] + q[ii] * a[jj]) * dk
        g = np.zeros((self.n, 3))
        for c in range(3):
            g[:, c] = np.bincount(ii, weights=coef * d[:, c], minlength=self.n)
        Sq = self.structure_factor(q)
        Sa = Sq if a is None else self.structure_factor(a)
        for c in range(3):
            kc = self.kvec[..., c]
            # (1/2) sum_m w |S|^2 -> -q_i sum_m w k Im(e_i S*)
            tq = self._back(self.W * kc * np.conj(Sq)).imag
            if a is None:
                g[:, c] += -q * tq
            else:
                ta = self._back(self.W * kc * np.conj(Sa)).imag
                g[:, c] += -a * tq - q * ta
        return g


def _virial_method(self, q):
    """W_ab = -dE_elec/d eps_ab at fixed q (same terms as ``ewald.virial``)."""
    q = np.asarray(q, dtype=np.float64)
    ii, jj, d, r, gam = self._pairs
    c = q[ii] * q[jj] * ewald.pair_kernel_deriv(r, gam, self.eta) / r
    W = -0.5 * np.einsum("e,ea,eb->ab", c, d, d)
    S = self.structure_factor(q)
    ek = 0.5 * self.W * (S.real ** 2 + S.imag ** 2)        # zero where the weight is
    k = self.kvec
    k2 = np.einsum("...i,...i->...", k, k)
    with np.errstate(divide="ignore", invalid="ignore"):
        cf = np.where(ek != 0.0, 2.0 * (1.0 / k2 + 0.5 * self.eta ** 2), 0.0)
    kf = k.reshape(-1, 3)
    W += ek.sum() * np.eye(3) - np.einsum("m,ma,mb->ab", (ek * cf).ravel(), kf, kf)
    W += ewald.background_energy(self.cell, self.sigma, q, self.eta) * np.eye(3)
    return W


EwaldOperator.virial = _virial_method


def projected_cg(apply_A, diag, chi, q_tot, tol=1e-12, max_iter=5000, q0=None, rhs=None):
    """Jacobi-preconditioned CG for min 1/2 q^T A q + chi.q on sum(q) = Q_tot.

    Every iterate stays on the constraint plane: the preconditioned residual
    z = D^-1 r - (sum D^-1 r / sum D^-1) D^-1 1 has zero sum.  Stops when
    ||P (A q + chi)|| <= tol ||P chi|| with P the orthogonal projector onto
    sum = 0.  ``rhs`` replaces -chi for adjoint solves (then Q_tot should be 0).
    Returns (q, mu, iterations, relative residual).
    """
    n = diag.shape[0]
    b = -np.asarray(chi, dtype=np.float64) if rhs is None else np.asarray(rhs, dtype=np.float64)
    q = np.full(n, q_tot / n) if q0 is None else np.asarray(q0, dtype=np.float64).copy()
    q += (q_tot - q.sum()) / n
    dinv = 1.0 / diag
    sdinv = dinv.sum()

    def pnorm(x):
        y = x - x.mean()
        return math.sqrt(y @ y)

    bnorm = pnorm(b)
    if bnorm == 0.0:
        bnorm = 1.0
    # The residual is kept projected (zero mean): its constant part only
    # carries the Lagrange multiplier and would swamp the dot products.
    r = b - apply_A(q)
    r -= r.mean()
    z = dinv * r - (dinv @ r / sdinv) * dinv
    p = z.copy()
    rz = r @ z
    it = 0
    res = pnorm(r) / bnorm
    while res > tol and it < max_iter:
        Ap = apply_A(p)
        alpha = rz / (p @ Ap)
        q += alpha * p
        r -= alpha * Ap
        r -= r.mean()
        z = dinv * r - (dinv @ r / sdinv) * dinv
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        res = pnorm(r) / bnorm
    g = apply_A(q) - b                # = A q + chi = mu 1 at the solution
    return q, float(g.mean()), it, pnorm(g) / bnorm


def qeq_matfree(pos, cell, sigma, J, chi, q_tot, eta=None, tol=1e-12, forces=True, op=None):
    """Charges, mu, energies and forces via the matrix-free operator + projected CG."""
    if op is None:
        op = EwaldOperator(pos, cell, sigma, eta=eta)
    J = np.asarray(J, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    diag = J + 1.0 / (op.sigma * SQRTPI)

    def apply_A(v):
        return op.apply(v) + J * v

    q, mu, it, res = projected_cg(apply_A, diag, chi, q_tot, tol=tol)
    Eq = op.apply(q)
    e_elec = 0.5 * q @ Eq
    e_qeq = e_elec + chi @ q + 0.5 * np.sum(J * q * q)
    out = ewald.QEqResult(q=q, mu=mu, lam=-mu, e_elec=e_elec, e_qeq=e_qeq, iters=it,
                          rel_resid=res, phi=Eq)
    if forces:
        out["forces"] = -op.grad_positions(q)
    return out
