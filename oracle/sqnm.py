"""Stabilised quasi-Newton minimisation (SQNM) of the QEq energy (test
infrastructure only: tests, smoke() and the bench's CPU baseline use it).

The paper lists SQNM beside conjugate gradients as a charge-equilibration
solver ("Electrostatics Solvers" benchmarks, SI solver comparison) without
stating it; this follows the published stabilised quasi-Newton scheme
(Schaefer, Mohr, Amsler, Goedecker, J. Chem. Phys. 142, 034112 (2015)),
applied to

    f(q) = 1/2 q^T A q + chi^T q     on the plane sum(q) = Q_tot,

A = E + diag(J) (eq. 4G_qeq_prime; its minimiser on the plane is the QEq
solution), in the coordinates z = D^{1/2} q with D the Jacobi diagonal
(J_i + 1/(sigma_i sqrt(pi))), i.e. with the metric <u, v> = u^T D v for
displacements and <g, h> = g^T D^-1 h for gradients.  One iteration:

1. history: the last m displacements s_i and gradient differences y_i,
   normalised by |s_i|; overlap matrix S_ij = <s_i, s_j>, eigenpairs of S
   with eigenvalues above eps_sig * max keep the well-conditioned subspace
   (orthonormal basis d_k = sum_i v_ik s_i / sqrt(lambda_k));
2. Hessian in that subspace H_kl = (d_k . dg_l + d_l . dg_k) / 2 (dg the
   matching gradient combinations); its eigenpairs (kappa_j, Ritz vectors
   h_j) and residuals res_j = |dg(h_j) - kappa_j D h_j|_{D^-1}; curvatures
   kappa_j' = sqrt(kappa_j^2 + res_j^2);
3. step = -alpha (P g - sum_j (h_j . g) D h_j) mapped back, i.e.
   dq = -alpha (zJ - sum_j c_j h_j) - sum_j c_j / kappa_j' h_j with
   c_j = h_j . (g - c 1) and zJ = D^-1 (g - c 1), c = sum D^-1 g / sum D^-1
   (the Jacobi-projected gradient, zero sum); the step is then projected
   back onto the plane (D metric) so that rounding cannot accumulate off it;
4. energy rise: the step is undone, alpha halved, the history cleared;
   otherwise the pair (s, y) joins the history and alpha grows by 5% when
   consecutive projected gradients still point the same way (cosine in the
   D^-1 metric > 0.2) and halves when they point against each other
   (cosine < 0).
Stop when ||P g||_2 / ||P chi||_2 <= tol (the CG's relative residual).
"""
from __future__ import annotations

import numpy as np

EPS_SIG = 1e-4


def sqnm_minimise(apply_A, diag, chi, q_tot, tol=1e-10, m=10, alpha0=1.0, max_iter=5000, q0=None,
                  record=None):
    """Minimise 1/2 q.A q + chi.q on sum(q) = q_tot.  apply_A(v) -> A v
    (A symmetric positive definite on the plane); diag: the metric D.
    Returns (q, iterations, relative residual).  With record (a list), each
    accepted iteration appends (Ritz values, subspace basis as columns) for
    inspection by the tests."""
    chi = np.asarray(chi, dtype=np.float64)
    D = np.asarray(diag, dtype=np.float64)
    n = chi.size
    Dinv = 1.0 / D
    pchi = chi - chi.mean()
    chi_norm = np.linalg.norm(pchi)
    scale = chi_norm if chi_norm > 0 else 1.0
    q = np.full(n, q_tot / n) if q0 is None else np.asarray(q0, dtype=np.float64).copy()
    q += (q_tot - q.sum()) / n

    def grad_energy(x):
        g = apply_A(x) + chi
        return g, 0.5 * x @ (g + chi)

    g, f = grad_energy(q)
    S, Y = [], []
    alpha = alpha0
    it = 0
    res = np.linalg.norm(g - g.mean()) / scale
    while res > tol and it < max_iter:
        it += 1
        c0 = (Dinv @ g) / Dinv.sum()
        zj = Dinv * (g - c0)                 # Jacobi-projected gradient (sum 0)
        step = -alpha * zj
        if S:
            Sm = np.array(S).T               # n x h
            Ym = np.array(Y).T
            norms = np.sqrt(np.einsum("ij,i,ij->j", Sm, D, Sm))
            Sn, Yn = Sm / norms, Ym / norms
            ov = Sn.T @ (D[:, None] * Sn)
            lam, V = np.linalg.eigh(ov)
            keep = lam > EPS_SIG * lam.max()
            B = V[:, keep] / np.sqrt(lam[keep])          # coefficients of d_k in the s_i
            dvec = Sn @ B
            dg = Yn @ B
            H = 0.5 * (dvec.T @ dg + dg.T @ dvec)
            kap, U = np.linalg.eigh(H)
            hvec = dvec @ U                              # Ritz vectors (columns)
            rvec = dg @ U
            # residuals in the D^-1 metric, with the constraint direction removed
            resid = rvec - kap * (D[:, None] * hvec)
            resid = resid - np.outer(np.ones(n), (Dinv @ resid) / Dinv.sum())
            rn2 = np.einsum("ij,i,ij->j", resid, Dinv, resid)
            kap_s = np.sqrt(kap ** 2 + rn2)
            # c_j = h_j . (g - c0 1): in exact arithmetic sum(h_j) = 0 and the
            # shift drops out, but rounding leaves h_j a small constant
            # component that the multiplier part of g would amplify
            c = hvec.T @ (g - c0)
            step = -alpha * (zj - hvec @ c) - hvec @ (c / kap_s)
            if record is not None:
                record.append((kap.copy(), dvec.copy()))
        # back onto the plane (D-metric projection of the rounding residue)
        step = step - Dinv * (step.sum() / Dinv.sum())
        q_new = q + step
        g_new, f_new = grad_energy(q_new)
        if f_new > f + 1e-14 * abs(f):
            alpha *= 0.5
            S, Y = [], []
            continue
        S.append(step)
        Y.append(g_new - g)
        if len(S) > m:
            S.pop(0)
            Y.pop(0)
        c1 = (Dinv @ g_new) / Dinv.sum()
        zj_new = Dinv * (g_new - c1)
        cosv = (zj_new @ (D * zj)) / np.sqrt((zj_new @ (D * zj_new)) * (zj @ (D * zj)) + 1e-300)
        if cosv > 0.2:
            alpha *= 1.05
        elif cosv < 0.0:
            alpha *= 0.5
        q, g, f = q_new, g_new, f_new
        res = np.linalg.norm(g - g.mean()) / scale
    return q, it, res


def qeq_sqnm(E, J, chi, q_tot, sigma, tol=1e-10, m=10):
    """QEq charges by SQNM on the dense operator E + diag(J); the Jacobi
    metric D = J + 1/(sigma sqrt(pi))."""
    J = np.asarray(J, dtype=np.float64)
    A = np.asarray(E, dtype=np.float64) + np.diag(J)
    D = J + 1.0 / (np.asarray(sigma, dtype=np.float64) * np.sqrt(np.pi))
    return sqnm_minimise(lambda v: A @ v, D, chi, q_tot, tol=tol, m=m)
