"""Spline orders other than 6 (4 and 8, within the documented 4..8 even range):
the orders the batched autotuner may choose.  Against the FP64 oracle with the
order-6 bars where the discretisation reaches them (order 8 at the configs'
spacing, order 4 on a fine single-structure grid); order 4 in the batched
path at spacing 0.5 misses the 1e-6 energy bar by discretisation (3.5e-6),
so there its code path is checked against the single-structure GPU solve of
the same grid and order instead (tight), and the autotuner's accuracy check
is what keeps such settings out."""
import numpy as np
import pytest

from inputs import gen
from oracle import ewald

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ETA = 2.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def check(q, en, f, ref):
    dq = np.abs(q - ref.q).max()
    de_q = abs(en[0] - ref.e_qeq) / abs(ref.e_qeq)
    de_e = abs(en[1] - ref.e_elec) / abs(ref.e_elec)
    df = np.sqrt(np.mean((f - ref.forces) ** 2)) / np.sqrt(np.mean(ref.forces ** 2))
    assert dq <= 1e-5 and de_q <= 1e-6 and de_e <= 1e-6 and df <= 1e-4, (dq, de_q, de_e, df)
    return dq, de_q, de_e, df


@pytest.mark.parametrize("p,grid", [(8, 24), (4, 48)])
def test_single_structure_orders(dev, p, grid):
    from paper_2607_17978_amd import qeq
    s = gen.system_64()
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    plan = qeq.Plan(s.n, eta=ETA, r_cut=11.0, grid=(grid,) * 3, spline_order=p, tol=1e-8)
    q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
    assert st["rc"] == 0
    print("p", p, "grid", grid, "iters", st["iters"], check(q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy(), ref))
    plan.close()


@pytest.mark.parametrize("p,spacing,members", [(8, 0.8, (3, 17, 40, 5))])
def test_batched_orders(dev, p, spacing, members):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(s) for s in members]
    offs = np.concatenate([[0], np.cumsum([s.n for s in structs])]).astype(np.int32)
    cat = lambda f: np.concatenate([getattr(s, f) for s in structs])
    plan = qeq.Plan(512, eta=ETA, r_cut=12.0, max_spacing=spacing, spline_order=p, tol=1e-8)
    q, en, f, st, rc = plan.solve_batched(T(cat("pos"), dev), offs, np.stack([s.cell for s in structs]),
                                         T(cat("sigma"), dev), T(cat("J"), dev), T(cat("chi"), dev),
                                         np.array([s.q_tot for s in structs]))
    assert rc == 0, st
    q, en, f = q.cpu().numpy(), en.cpu().numpy(), f.cpu().numpy()
    for k, s in enumerate(structs):
        ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
        sl = slice(offs[k], offs[k + 1])
        print("p", p, "member", members[k], "n", s.n, check(q[sl], en[k], f[sl], ref))
    plan.close()


def test_batched_order4_equals_single(dev):
    from paper_2607_17978_amd import qeq
    members = (18, 22, 34, 17)
    structs = [gen.batch_structure(s) for s in members]
    offs = np.concatenate([[0], np.cumsum([s.n for s in structs])]).astype(np.int32)
    cat = lambda f: np.concatenate([getattr(s, f) for s in structs])
    plan = qeq.Plan(512, eta=ETA, r_cut=12.0, max_spacing=0.5, spline_order=4, tol=1e-9)
    q, en, f, st, rc = plan.solve_batched(T(cat("pos"), dev), offs, np.stack([s.cell for s in structs]),
                                         T(cat("sigma"), dev), T(cat("J"), dev), T(cat("chi"), dev),
                                         np.array([s.q_tot for s in structs]))
    assert rc == 0, st
    q, en = q.cpu().numpy(), en.cpu().numpy()
    for k, s in enumerate(structs):
        one = qeq.Plan(s.n, eta=ETA, r_cut=12.0, max_spacing=0.5, spline_order=4, tol=1e-9)
        q1, en1, _, st1 = one.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        sl = slice(offs[k], offs[k + 1])
        dq = np.abs(q[sl] - q1.cpu().numpy()).max()
        de = np.abs(en[k] - en1.cpu().numpy()).max() / np.abs(en1.cpu().numpy()).max()
        print("p 4 member", members[k], "n", s.n, "batched vs single dq", dq, "dE", de)
        assert dq <= 1e-7 and de <= 1e-7
        one.close()
    plan.close()
