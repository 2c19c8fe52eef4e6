"""mlp_train_step_noalloc (the allocation-free training step) against
mlp_train_step through the C ABI: two calls in a row, the second on a smaller
batch, each from the same state on both sides.  The two share their kernels;
they differ only in where the partial gradients live, so the results agree up
to the FP32 rounding order of the gradient sums (LDS atomics): loss to 1e-6
relative, gradients to 1e-5 of their largest magnitude, Adam moments
accordingly, parameters to 1e-4 lr except where a gradient component is
within rounding of zero (its Adam step then has an undetermined sign, at most
2 lr apart)."""
import ctypes

import numpy as np
import pytest

from inputs import gen
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_17978_amd import qeq
    qeq.load_library()
    return torch.device("cuda", 0)


def P(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def pack(nets):
    p = np.zeros(len(nets) * omlp.STRIDE, dtype=np.float32)
    for e, nt in enumerate(nets):
        o = e * omlp.STRIDE
        p[o + omlp.OFF_W1:o + omlp.OFF_W1 + 512] = np.asarray(nt["W1"]).ravel()
        p[o + omlp.OFF_B1:o + omlp.OFF_B1 + 32] = nt["b1"]
        p[o + omlp.OFF_W2:o + omlp.OFF_W2 + 1024] = np.asarray(nt["W2"]).ravel()
        p[o + omlp.OFF_B2:o + omlp.OFF_B2 + 32] = nt["b2"]
        p[o + omlp.OFF_W3:o + omlp.OFF_W3 + 32] = nt["W3"]
        p[o + omlp.OFF_B3] = nt["b3"]
    return p


def test_noalloc_train_step_matches_the_workspace_entry(dev):
    from paper_2607_17978_amd import qeq
    L = qeq.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nsp = 2
    rng = np.random.default_rng(11)
    nets = gen.warmstart_init(1005, nsp)
    params0 = torch.as_tensor(pack(nets), device=dev)
    m0 = torch.zeros_like(params0)
    v0 = torch.zeros_like(params0)
    nws = int(L.mlp_workspace_floats(nsp))
    ws = torch.empty(nws, dtype=torch.float32, device=dev)
    lr = 1e-3
    for call, n in enumerate((2048, 500)):
        G = torch.as_tensor(rng.gamma(2.0, 0.6, size=(n, 16)), dtype=torch.float32, device=dev)
        species = torch.as_tensor((rng.uniform(size=n) < 0.5).astype(np.int32), device=dev)
        target = torch.as_tensor(rng.normal(0, 0.2, n), dtype=torch.float64, device=dev)
        stats = torch.empty(nsp * 3 * 16, dtype=torch.float32, device=dev)
        assert L.mlp_feature_stats(P(G), P(species), n, nsp, P(stats), P(ws), stream) == 0
        out = {}
        for name in ("workspace", "noalloc"):
            p, m, v = params0.clone(), m0.clone(), v0.clone()
            loss = torch.zeros(1, dtype=torch.float32, device=dev)
            grad = torch.zeros_like(params0)
            step = call + 1
            if name == "workspace":
                rc = L.mlp_train_step(P(G), P(species), P(target), n, nsp, P(stats), P(p), P(m), P(v), step,
                                      lr, P(ws), nws, P(loss), P(grad), stream)
            else:
                rc = L.mlp_train_step_noalloc(P(G), P(species), P(target), n, nsp, P(stats), P(p), P(m), P(v),
                                              step, lr, P(loss), P(grad), stream)
            torch.cuda.synchronize()
            assert rc == 0, (name, rc)
            out[name] = [t.cpu().numpy().astype(np.float64) for t in (p, m, v, loss, grad)]
        (pa, ma, va, la, ga), (pb, mb, vb, lb, gb) = out["workspace"], out["noalloc"]
        gmax = np.abs(ga).max()
        print(f"call {call} n={n}: loss {la[0]:.6e} vs {lb[0]:.6e}, max |dg| {np.abs(ga - gb).max():.2e} "
              f"(max |g| {gmax:.2e}), max |dp| {np.abs(pa - pb).max():.2e}")
        assert abs(la[0] - lb[0]) <= 1e-6 * abs(la[0])
        assert np.abs(ga - gb).max() <= 1e-5 * gmax
        assert np.abs(ma - mb).max() <= 1e-5 * max(np.abs(ma).max(), 1e-30)
        assert np.abs(va - vb).max() <= 1e-5 * max(np.abs(va).max(), 1e-30)
        stable = np.abs(ga) > 1e-4 * gmax
        assert np.all(np.abs(pa - pb)[stable] <= 1e-4 * lr + 2.0 ** -23 * np.abs(pa[stable]))
        assert np.all(np.abs(pa - pb) <= 2.0 * lr + 2.0 ** -23 * np.abs(pa))
        # the next call starts from the workspace entry's state on both sides
        params0 = torch.as_tensor(pa.astype(np.float32), device=dev)
        m0 = torch.as_tensor(ma.astype(np.float32), device=dev)
        v0 = torch.as_tensor(va.astype(np.float32), device=dev)


def test_noalloc_rejects_bad_arguments(dev):
    from paper_2607_17978_amd import qeq
    L = qeq.load_library()
    x = torch.zeros(16, dtype=torch.float32, device=dev)
    i = torch.zeros(1, dtype=torch.int32, device=dev)
    d = torch.zeros(1, dtype=torch.float64, device=dev)
    big = torch.zeros(5 * omlp.STRIDE, dtype=torch.float32, device=dev)
    # five species exceed the fixed array (and the kernels)
    assert L.mlp_train_step_noalloc(P(x), P(i), P(d), 1, 5, P(big), P(big), P(big), P(big), 1, 1e-3, None, None,
                                    None) == qeq.QEQ_EINVAL
    assert L.mlp_train_step_noalloc(P(x), P(i), P(d), 0, 1, P(x), P(big), P(big), P(big), 1, 1e-3, None, None,
                                    None) == qeq.QEQ_EINVAL
