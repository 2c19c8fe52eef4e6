"""Pin of the 4G charge-training gradient (electronegativity networks trained
through the QEq solve): the chain-rule gradient of the oracle against central
finite differences of the loss with every QEq re-solved, and a planted
mistake (the adjoint's sign flipped) that the check catches."""
import numpy as np

from inputs import gen
from oracle import mlp as omlp


def setup(seed=2):
    s = gen.lattice_system(3, 14.0, seed)
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (s.n, 16))
    nets = gen.warmstart_init(1005 + seed, 2)
    p = np.zeros(2 * omlp.STRIDE)
    for e, n in enumerate(nets):
        o = e * omlp.STRIDE
        p[o + omlp.OFF_W1:o + omlp.OFF_W1 + 512] = np.asarray(n["W1"]).ravel()
        p[o + omlp.OFF_W2:o + omlp.OFF_W2 + 1024] = np.asarray(n["W2"]).ravel()
        p[o + omlp.OFF_W3:o + omlp.OFF_W3 + 32] = 0.1 * np.asarray(n["W3"])
        p[o + omlp.OFF_B3] = (0.1, -0.1)[e]
    q_ref = rng.normal(0.0, 0.2, s.n)
    q_ref -= q_ref.mean()
    return s, X, p, q_ref


def loss(p, s, X, q_ref):
    return omlp.charge_loss_through_qeq(p, X, s.species, s.pos, s.cell, s.sigma, s.J, 0.0, q_ref)[0]


def fd_check(grad_fn):
    s, X, p, q_ref = setup()
    L, g, q, dchi = grad_fn(p, s, X, q_ref)
    idx = [omlp.OFF_W1 + 5, omlp.OFF_B1 + 3, omlp.OFF_W2 + 100, omlp.OFF_B2 + 7, omlp.OFF_W3 + 2,
           omlp.OFF_B3, omlp.STRIDE + omlp.OFF_W3 + 9, omlp.STRIDE + omlp.OFF_B3]
    h = 1e-5
    err = []
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (loss(pp, s, X, q_ref) - loss(pm, s, X, q_ref)) / (2 * h)
        err.append(abs(fd - g[k]) / max(abs(fd), 1e-8))
    return max(err)


def test_chain_rule_gradient_matches_finite_differences():
    def grad_fn(p, s, X, q_ref):
        return omlp.charge_loss_through_qeq(p, X, s.species, s.pos, s.cell, s.sigma, s.J, 0.0, q_ref)
    assert fd_check(grad_fn) < 1e-6


def test_planted_adjoint_sign_is_caught():
    def wrong(p, s, X, q_ref):
        L, g, q, dchi = omlp.charge_loss_through_qeq(p, X, s.species, s.pos, s.cell, s.sigma, s.J, 0.0, q_ref)
        chi, cache = omlp.forward(p, X, s.species)
        return L, omlp.backward(p, cache, -dchi), q, -dchi
    assert fd_check(wrong) > 0.5


def test_hardness_network_gradient_matches_finite_differences():
    """J_i = J_e exp(0.2 y_i) from a second set of networks: the chain rule
    through dL/dJ of the adjoint against central differences."""
    s, X, p, q_ref = setup()
    _, _, pj, _ = setup(seed=3)
    pj = pj.copy()
    for e in range(2):
        pj[e * omlp.STRIDE + omlp.OFF_B3] = 0.0
    j_elem = s.J

    def L_of(pc, pjj):
        return omlp.charge_loss_through_qeq_chi_j(pc, pjj, X, s.species, s.pos, s.cell, s.sigma, j_elem, 0.2, 0.0,
                                                  q_ref)[0]

    L, gc, gj, q = omlp.charge_loss_through_qeq_chi_j(p, pj, X, s.species, s.pos, s.cell, s.sigma, j_elem, 0.2,
                                                      0.0, q_ref)
    h = 1e-5
    for k in (omlp.OFF_W1 + 7, omlp.OFF_B2 + 2, omlp.OFF_W3 + 4, omlp.OFF_B3, omlp.STRIDE + omlp.OFF_W2 + 33):
        pp, pm = pj.copy(), pj.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L_of(p, pp) - L_of(p, pm)) / (2 * h)
        assert abs(fd - gj[k]) <= 1e-6 * max(abs(fd), 1e-6)
    # the chi part agrees with the chi-only function when J is the element value
    pz = np.zeros_like(pj)
    L1, gc1, _, _ = omlp.charge_loss_through_qeq_chi_j(p, pz, X, s.species, s.pos, s.cell, s.sigma, j_elem, 0.2,
                                                       0.0, q_ref)
    L2, gc2, _, _ = omlp.charge_loss_through_qeq(p, X, s.species, s.pos, s.cell, s.sigma, s.J, 0.0, q_ref)
    assert abs(L1 - L2) <= 1e-14 and np.abs(gc1 - gc2).max() <= 1e-12
