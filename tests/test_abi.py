"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-only calls behave (no device work here)."""
import ctypes
import os

import pytest

from paper_2607_17978_amd import qeq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(qeq.LIB_PATH):
        pytest.skip("libqeq.so not built")
    return qeq.load_library()


def test_header_declares_the_solver_calls():
    names = qeq.header_functions()
    for required in ("qeq_plan_create", "qeq_plan_destroy", "qeq_solve", "qeq_matvec",
                     "qeq_strerror", "qeq_params_default"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in qeq.header_functions():
        assert hasattr(L, name), name


def test_default_params_and_strerror():
    _lib_or_skip()
    p = qeq.default_params()
    assert p.eta == 2.0 and p.r_cut == 11.0 and p.spline_order == 6 and p.self_correction == 1
    assert p.tol == 1e-6 and tuple(p.grid) == (0, 0, 0)
    assert p.precond == 0 and p.spectral_kcut == 0.2
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert qeq.strerror(code) != "unknown status code"
    assert qeq.strerror(42) == "unknown status code"


def test_plan_create_rejects_bad_params_before_touching_the_device():
    L = _lib_or_skip()
    p = qeq.default_params()
    h = ctypes.c_void_p()
    p.spline_order = 5
    assert L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == qeq.QEQ_EPLAN
    p.spline_order = 6
    p.eta = -1.0
    assert L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == qeq.QEQ_EINVAL
    p.eta = 2.0
    assert L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), 0, None) == qeq.QEQ_EINVAL
    p.precond = 2
    assert L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == qeq.QEQ_EINVAL
    p.precond, p.spectral_kcut = 1, float("nan")
    assert L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == qeq.QEQ_EINVAL


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of qeq_params / qeq_stats agree with the C compiler's layout."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qeq.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(qeq_params), offsetof(qeq_params, grid), offsetof(qeq_params, tol),"
        "offsetof(qeq_params, precond), sizeof(qeq_stats), offsetof(qeq_stats, rel_resid),"
        "offsetof(qeq_stats, mu), offsetof(qeq_stats, e_elec), offsetof(qeq_params, spectral_kcut));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P, S = qeq.Params, qeq.Stats
    want = [ctypes.sizeof(P), P.grid.offset, P.tol.offset, P.precond.offset,
            ctypes.sizeof(S), S.rel_resid.offset, S.mu.offset, S.e_elec.offset, P.spectral_kcut.offset]
    assert got == want


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus above 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_bench_traffic_records_match_the_kernel_sources():
    """The HBM traffic in the bench line comes from rocprofv3 counters taken on
    one version of each kernel that can be the dominant one; the stored source
    hashes must still match (bench.py reports traffic as null otherwise)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert set(bench.MEASURED_TRAFFIC) >= {"spread_r2c", "c2r"}
    for name, rec in bench.MEASURED_TRAFFIC.items():
        assert bench.kernel_source_hash(rec["file"], rec["kernel"]) == rec["source_sha256_16"], name
