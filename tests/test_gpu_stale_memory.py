"""Results must not depend on what a fresh device allocation holds.

With QEQ_POISON_ALLOC set, the library fills every new floating-point
buffer with NaN bytes, so a kernel that reads memory nothing wrote turns the
result into NaN.  Each case runs on a plan created without poisoning and on
one created with it, and the two must agree (the kernels are deterministic
up to the order of FP64 atomic additions; the Gaussian-on-grid spread adds
FP32 values with atomics, so that case is compared to FP32 rounding).
"""
import numpy as np
import pytest

from inputs import gen

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


def T(a, dev, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def both(monkeypatch, run, tol=1e-9):
    monkeypatch.delenv("QEQ_POISON_ALLOC", raising=False)
    clean = run()
    monkeypatch.setenv("QEQ_POISON_ALLOC", "1")
    poisoned = run()
    monkeypatch.delenv("QEQ_POISON_ALLOC", raising=False)
    for name, a in clean.items():
        b = poisoned[name]
        assert np.all(np.isfinite(b)), f"{name}: non-finite with poisoned allocations"
        scale = max(float(np.abs(a).max()), 1e-30)
        err = float(np.abs(np.asarray(a) - np.asarray(b)).max()) / scale
        print(name, "rel max diff", err)
        assert err <= tol, name


def periodic_run(dev, s, rc, spectral=0.0, ewald=False, extras=True, planewave=False, sqnm=False):
    from paper_2607_17978_amd import qeq

    def run():
        plan = qeq.Plan(s.n, eta=ETA, r_cut=rc, grid=s.grid, tol=1e-8, max_iter=3000)
        if ewald:
            plan.use_ewald(True)
        if spectral:
            plan.use_spectral_preconditioner(spectral)
        if planewave:
            plan.use_planewave(True)
        if sqnm:
            plan.use_sqnm(True)
        q, en, f, st = plan.solve(T(s.pos, dev), s.cell, T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        assert st["rc"] == 0, st
        out = {"q": q.cpu().numpy(), "energies": en.cpu().numpy(), "forces": f.cpu().numpy()}
        if extras and not ewald and not planewave:
            out["virial"] = plan.virial().cpu().numpy()
            w = np.random.default_rng(3).uniform(size=s.n)
            dchi, dJ, dpos, st_b = plan.backward(T(w * (q.cpu().numpy() - 0.1), dev), dL_dEelec=1.0)
            out.update(dchi=dchi.cpu().numpy(), dJ=dJ.cpu().numpy(), dpos=dpos.cpu().numpy())
            out["gamma"] = plan.element_potentials(T(s.species, dev, torch.int32), 2).cpu().numpy()
        plan.close()
        return out
    return run


@pytest.mark.parametrize("which", ["n64", "n4096", "n32768"])
def test_periodic_solve_ignores_stale_memory(dev, monkeypatch, which):
    s = {"n64": gen.system_64, "n4096": gen.system_4096, "n32768": gen.system_32k}[which]()
    both(monkeypatch, periodic_run(dev, s, 11.0))


def test_spectral_preconditioner_ignores_stale_memory(dev, monkeypatch):
    both(monkeypatch, periodic_run(dev, gen.system_32k(), 11.0, spectral=0.2, extras=False))


def test_ewald_ignores_stale_memory(dev, monkeypatch):
    both(monkeypatch, periodic_run(dev, gen.system_64(), 11.0, ewald=True))


def test_sqnm_ignores_stale_memory(dev, monkeypatch):
    both(monkeypatch, periodic_run(dev, gen.system_512(), 11.0, sqnm=True))


def test_planewave_ignores_stale_memory(dev, monkeypatch):
    # FP32 atomic additions in the spread: equal up to rounding, not bitwise
    both(monkeypatch, periodic_run(dev, gen.batch_structure(40), 12.0, planewave=True), tol=1e-6)


def test_batched_ignores_stale_memory(dev, monkeypatch):
    from paper_2607_17978_amd import qeq
    structs = [gen.batch_structure(k) for k in (3, 17, 40, 5, 101)]
    offs = np.concatenate([[0], np.cumsum([s.n for s in structs])]).astype(np.int32)
    cat = lambda f: np.concatenate([getattr(s, f) for s in structs])
    a = dict(pos=T(cat("pos"), dev), offsets=offs, cells=np.stack([s.cell for s in structs]),
             sigma=T(cat("sigma"), dev), J=T(cat("J"), dev), chi=T(cat("chi"), dev),
             q_tot=np.array([s.q_tot for s in structs]))

    def run():
        plan = qeq.Plan(int(max(s.n for s in structs)), eta=ETA, r_cut=12.0, tol=1e-8)
        q, en, f, st, rc = plan.solve_batched(**a)
        assert rc == 0, st
        out = {"q": q.cpu().numpy(), "energies": en.cpu().numpy(), "forces": f.cpu().numpy()}
        plan.close()
        return out
    both(monkeypatch, run)


def test_nonperiodic_ignores_stale_memory(dev, monkeypatch):
    from paper_2607_17978_amd import qeq
    s = gen.cluster_system(512, q_tot=1.0)

    def run():
        plan = qeq.Plan(s.n, tol=1e-8, max_iter=3000)
        q, en, f, st = plan.solve_nonperiodic(T(s.pos, dev), T(s.sigma, dev), T(s.J, dev), T(s.chi, dev), s.q_tot)
        assert st["rc"] == 0, st
        out = {"q": q.cpu().numpy(), "energies": en.cpu().numpy(), "forces": f.cpu().numpy(),
               "gamma": plan.element_potentials(T(s.species, dev, torch.int32), 2).cpu().numpy()}
        plan.close()
        return out
    both(monkeypatch, run)
