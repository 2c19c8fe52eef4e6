"""Thin ctypes binding of the C ABI in include/qeq.h (argument marshalling only).

Every step of the solve runs in the HIP library ``libqeq.so`` that sits next
to this file; the binding only checks tensor placement / dtype / shape and
passes raw device pointers.  If the library is missing, importing works but
every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqeq.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "qeq.h")

QEQ_OK = 0
QEQ_NOT_CONVERGED = 1
QEQ_EINVAL = -1
QEQ_ECELL = -2
QEQ_ENOMEM = -3
QEQ_EHIP = -4
QEQ_EPLAN = -5

PART_RECIP, PART_REAL, PART_SELF, PART_BG = 1, 2, 4, 8
PART_ALL = 15


class Params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double),
        ("r_cut", ctypes.c_double),
        ("max_spacing", ctypes.c_double),
        ("grid", ctypes.c_int32 * 3),
        ("spline_order", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("self_correction", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("spectral_kcut", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("rel_resid", ctypes.c_double),
        ("true_rel_resid", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("e_qeq", ctypes.c_double),
        ("e_elec", ctypes.c_double),
        ("q0_rejected", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class QEqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qeq error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libqeq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i32, f64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.qeq_params_default.argtypes = [ctypes.POINTER(Params)]
    L.qeq_params_default.restype = None
    L.qeq_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), i32, vp]
    L.qeq_plan_create.restype = ctypes.c_int
    L.qeq_plan_destroy.argtypes = [vp]
    L.qeq_plan_destroy.restype = ctypes.c_int
    L.qeq_solve.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_double), dp, dp, dp, f64, dp, dp, dp,
                            dp, ctypes.POINTER(Stats)]
    L.qeq_solve.restype = ctypes.c_int
    L.qeq_solve_nonperiodic.argtypes = [vp, i32, dp, dp, dp, dp, f64, dp, dp, dp, dp, ctypes.POINTER(Stats)]
    L.qeq_solve_nonperiodic.restype = ctypes.c_int
    L.qeq_element_potentials.argtypes = [vp, vp, i32, dp]
    L.qeq_element_potentials.restype = ctypes.c_int
    L.qeq_backward.argtypes = [vp, dp, f64, f64, dp, dp, dp, ctypes.POINTER(Stats)]
    L.qeq_backward.restype = ctypes.c_int
    L.qeq_virial.argtypes = [vp, dp]
    L.qeq_virial.restype = ctypes.c_int
    L.qeq_matvec.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_double), dp, dp, dp, i32]
    L.qeq_matvec.restype = ctypes.c_int
    L.qeq_time_kernel.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
    L.qeq_time_kernel.restype = ctypes.c_int
    L.qeq_use_ewald.argtypes = [vp, i32]
    L.qeq_use_ewald.restype = ctypes.c_int
    L.qeq_use_planewave.argtypes = [vp, i32, ctypes.c_double]
    L.qeq_use_planewave.restype = ctypes.c_int
    L.qeq_use_sqnm.argtypes = [vp, i32, i32]
    L.qeq_use_sqnm.restype = ctypes.c_int
    L.qeq_use_spectral_preconditioner.argtypes = [vp, f64]
    L.qeq_use_spectral_preconditioner.restype = ctypes.c_int
    L.qeq_use_fused_inverse.argtypes = [vp, i32]
    L.qeq_use_fused_inverse.restype = ctypes.c_int
    L.qeq_use_fused_forward.argtypes = [vp, i32]
    L.qeq_use_fused_forward.restype = ctypes.c_int
    L.qeq_use_fused_interp.argtypes = [vp, i32]
    L.qeq_use_fused_interp.restype = ctypes.c_int
    L.qeq_set_tiles.argtypes = [vp, i32, i32, i32]
    L.qeq_set_tiles.restype = ctypes.c_int
    L.qeq_use_graphs.argtypes = [vp, i32]
    L.qeq_use_graphs.restype = ctypes.c_int
    L.qeq_profile.argtypes = [vp, ctypes.c_uint32]
    L.qeq_profile.restype = ctypes.c_int
    L.qeq_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                   i32, i32]
    L.qeq_profile_read.restype = ctypes.c_int
    L.qeq_descriptors.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_double), dp, dp, i32,
                                  ctypes.POINTER(ctypes.c_double), f64, f64, dp]
    L.qeq_descriptors.restype = ctypes.c_int
    L.mlp_workspace_floats.argtypes = [i32]
    L.mlp_workspace_floats.restype = ctypes.c_int64
    L.mlp_feature_stats.argtypes = [dp, dp, i32, i32, dp, dp, vp]
    L.mlp_feature_stats.restype = ctypes.c_int
    L.mlp_forward.argtypes = [dp, dp, i32, i32, dp, dp, dp, vp]
    L.mlp_forward.restype = ctypes.c_int
    L.mlp_train_step.argtypes = [dp, dp, dp, i32, i32, dp, dp, dp, dp, i32, ctypes.c_float, dp,
                                 ctypes.c_int64, dp, dp, vp]
    L.mlp_train_step.restype = ctypes.c_int
    L.mlp_train_step_noalloc.argtypes = [dp, dp, dp, i32, i32, dp, dp, dp, dp, i32, ctypes.c_float, dp, dp, vp]
    L.mlp_train_step_noalloc.restype = ctypes.c_int
    L.qeq_solve_batched.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), dp, ctypes.POINTER(ctypes.c_double),
                                    dp, dp, dp, ctypes.POINTER(ctypes.c_double), dp, dp, dp, dp,
                                    ctypes.POINTER(Stats)]
    L.qeq_solve_batched.restype = ctypes.c_int
    L.qeq_batched_config.argtypes = [vp, i32, i32]
    L.qeq_batched_config.restype = ctypes.c_int
    L.qeq_batched_phase_us.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.qeq_batched_phase_us.restype = ctypes.c_int
    L.qeq_batched_last_ms.argtypes = [vp, i32]
    L.qeq_batched_last_ms.restype = ctypes.c_double
    L.qeq_strerror.argtypes = [ctypes.c_int]
    L.qeq_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/qeq.h."""
    src = open(HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qeq_[a-z_]+|mlp_[a-z_]+)\s*\(", src)))


def strerror(code: int) -> str:
    return load_library().qeq_strerror(code).decode()


def default_params() -> Params:
    p = Params()
    load_library().qeq_params_default(ctypes.byref(p))
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_dev(name, t, n, cols=None, device=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    shape = (n,) if cols is None else (n, cols)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, plan is on {device}")


def _cell_arg(cell):
    c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    return c, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Plan:
    """A solver plan bound to one device and stream (see qeq_plan_create)."""

    def __init__(self, n_max, eta=2.0, r_cut=11.0, grid=None, max_spacing=0.8, spline_order=6,
                 tol=1e-6, max_iter=1000, self_correction=True, stream=None, spectral_kcut=0.0):
        import torch
        L = load_library()
        p = default_params()
        p.eta, p.r_cut, p.max_spacing = eta, r_cut, max_spacing
        g = grid if grid is not None else (0, 0, 0)
        for a in range(3):
            p.grid[a] = int(g[a])
        p.spline_order, p.tol, p.max_iter = spline_order, tol, max_iter
        p.self_correction = 1 if self_correction else 0
        if spectral_kcut > 0.0:
            p.precond, p.spectral_kcut = 1, float(spectral_kcut)
        self.params = p
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = L.qeq_plan_create(ctypes.byref(h), ctypes.byref(p), int(n_max),
                               ctypes.c_void_p(self.stream.cuda_stream))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        self._h = h
        self.n_max = int(n_max)
        self.solve_count = 0      # identifies the tape left by the last solve
        self._last_n = None

    def close(self):
        if getattr(self, "_h", None):
            load_library().qeq_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, pos, cell, sigma, J, chi, q_tot=0.0, q0=None, forces=True, check=True):
        """Charges, [E_QEq, E_elec], forces (or None) and the stats dict."""
        import torch
        n = int(pos.shape[0])
        for name, t, c in (("pos", pos, 3), ("sigma", sigma, None), ("J", J, None), ("chi", chi, None)):
            _check_dev(name, t, n, c, self.device)
        if q0 is not None:
            _check_dev("q0", q0, n, None, self.device)
        q = torch.empty(n, dtype=torch.float64, device=self.device)
        en = torch.empty(2, dtype=torch.float64, device=self.device)
        f = torch.empty((n, 3), dtype=torch.float64, device=self.device) if forces else None
        st = Stats()
        _, cp = _cell_arg(cell)
        rc = load_library().qeq_solve(self._h, n, _ptr(pos), cp, _ptr(sigma), _ptr(J), _ptr(chi),
                                      float(q_tot), _ptr(q0), _ptr(q), _ptr(en), _ptr(f),
                                      ctypes.byref(st))
        self.solve_count += 1
        self._last_n = n
        if check and rc < 0:
            raise QEqError(rc, strerror(rc))
        return q, en, f, dict(st.as_dict(), rc=rc)

    def solve_nonperiodic(self, pos, sigma, J, chi, q_tot=0.0, q0=None, forces=True, check=True):
        """Isolated system (no cell): charges, [E_QEq, E_elec], forces (or None), stats."""
        import torch
        n = int(pos.shape[0])
        for name, t, c in (("pos", pos, 3), ("sigma", sigma, None), ("J", J, None), ("chi", chi, None)):
            _check_dev(name, t, n, c, self.device)
        if q0 is not None:
            _check_dev("q0", q0, n, None, self.device)
        q = torch.empty(n, dtype=torch.float64, device=self.device)
        en = torch.empty(2, dtype=torch.float64, device=self.device)
        f = torch.empty((n, 3), dtype=torch.float64, device=self.device) if forces else None
        st = Stats()
        rc = load_library().qeq_solve_nonperiodic(self._h, n, _ptr(pos), _ptr(sigma), _ptr(J), _ptr(chi),
                                                  float(q_tot), _ptr(q0), _ptr(q), _ptr(en), _ptr(f),
                                                  ctypes.byref(st))
        self.solve_count += 1
        self._last_n = None   # no tape: backward / virial need a periodic solve
        if check and rc < 0:
            raise QEqError(rc, strerror(rc))
        return q, en, f, dict(st.as_dict(), rc=rc)

    def element_potentials(self, species, n_elem):
        """Gamma (n x n_elem float64, device): potentials at each atom of the
        charges of each element, without the atom's own self term (ee4G
        embedding features; see qeq_element_potentials)."""
        import torch
        n = int(species.shape[0])
        if species.device != self.device or species.dtype != torch.int32 or not species.is_contiguous():
            raise QEqError(QEQ_EINVAL, "species must be a contiguous int32 tensor on the plan's device")
        out = torch.empty((n, int(n_elem)), dtype=torch.float64, device=self.device)
        rc = load_library().qeq_element_potentials(self._h, ctypes.c_void_p(species.data_ptr()), int(n_elem),
                                                   _ptr(out))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        return out

    def backward(self, dL_dq=None, dL_dEelec=0.0, dL_dEqeq=0.0, check=True):
        """Adjoint gradients (dL/dchi, dL/dJ, dL/dpos, stats) through the last solve;
        the energy weights come in the C ABI's order, E_elec first."""
        import torch
        n = self._last_n
        if n is None:
            raise QEqError(QEQ_EINVAL, "backward needs a preceding solve")
        if dL_dq is not None:
            _check_dev("dL_dq", dL_dq, n, None, self.device)
        dchi = torch.empty(n, dtype=torch.float64, device=self.device)
        dJ = torch.empty(n, dtype=torch.float64, device=self.device)
        dpos = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        st = Stats()
        rc = load_library().qeq_backward(self._h, _ptr(dL_dq), float(dL_dEelec), float(dL_dEqeq),
                                         _ptr(dchi), _ptr(dJ), _ptr(dpos), ctypes.byref(st))
        if check and rc < 0:
            raise QEqError(rc, strerror(rc))
        return dchi, dJ, dpos, dict(st.as_dict(), rc=rc)

    def virial(self):
        """Virial W = -dE/d eps (3 x 3 float64 on the device) of the last solve;
        the stress is -W / V (see qeq_virial)."""
        import torch
        if self._last_n is None:
            raise QEqError(QEQ_EINVAL, "virial needs a preceding solve")
        W = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        rc = load_library().qeq_virial(self._h, _ptr(W))
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return W

    def descriptors(self, pos, cell, sigma, centers, width, r_cut, weights=None):
        """Radial descriptors G (n x len(centers), float32, device), optionally
        weighted per neighbour; see qeq_descriptors.  pos=None reuses the
        geometry of the last solve / descriptor call (n from sigma or weights)."""
        import torch
        if pos is None:
            n = int((sigma if sigma is not None else weights).shape[0])
        else:
            n = int(pos.shape[0])
            _check_dev("pos", pos, n, 3, self.device)
            _check_dev("sigma", sigma, n, None, self.device)
        if weights is not None:
            _check_dev("weights", weights, n, None, self.device)
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64))
        G = torch.empty((n, len(c)), dtype=torch.float32, device=self.device)
        _, cp = _cell_arg(cell)
        rc = load_library().qeq_descriptors(self._h, n, _ptr(pos), cp, _ptr(sigma), _ptr(weights), len(c),
                                            c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            float(width), float(r_cut), _ptr(G))
        if pos is not None:
            self._last_n = None   # the tape of the last solve is gone
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return G

    def solve_batched(self, pos, offsets, cells, sigma, J, chi, q_tot, q0=None, forces=True, check=True):
        """Solve many structures in one persistent launch (see qeq_solve_batched).

        pos (N_tot x 3), sigma, J, chi (N_tot): device float64; offsets: n_struct + 1
        ints (host); cells: n_struct x 3 x 3 (host); q_tot: n_struct (host).
        Returns q (N_tot), energies (n_struct x 2), forces (N_tot x 3 or None),
        a list of per-structure stats dicts and the return code.
        """
        import torch
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
        ns = off.shape[0] - 1
        ntot = int(off[-1])
        for name, t, c in (("pos", pos, 3), ("sigma", sigma, None), ("J", J, None), ("chi", chi, None)):
            _check_dev(name, t, ntot, c, self.device)
        if q0 is not None:
            _check_dev("q0", q0, ntot, None, self.device)
        cl = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(ns, 9))
        qt = np.ascontiguousarray(np.asarray(q_tot, dtype=np.float64).reshape(ns))
        q = torch.zeros(ntot, dtype=torch.float64, device=self.device)
        en = torch.zeros((ns, 2), dtype=torch.float64, device=self.device)
        f = torch.zeros((ntot, 3), dtype=torch.float64, device=self.device) if forces else None
        st = (Stats * ns)()
        rc = load_library().qeq_solve_batched(
            self._h, ns, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(pos),
            cl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(sigma), _ptr(J), _ptr(chi),
            qt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(q0), _ptr(q), _ptr(en), _ptr(f), st)
        self._last_n = None       # the tape of the last solve is gone
        if check and rc < 0 and rc != QEQ_EINVAL and rc != QEQ_EPLAN:
            raise QEqError(rc, strerror(rc))
        return q, en, f, [st[k].as_dict() for k in range(ns)], rc

    def batched_config(self, threads=1024, wg_per_cu=1):
        """Launch shape of the batched solver (see qeq_batched_config)."""
        rc = load_library().qeq_batched_config(self._h, int(threads), int(wg_per_cu))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))

    BATCH_PHASES = ("setup", "pairs", "mesh_prep", "spread", "fft", "interp", "cg_vec", "total")

    def batched_phase_us(self, n_struct):
        """n_struct x 8 array of per-structure phase microseconds of the last batched call."""
        buf = (ctypes.c_double * (8 * n_struct))()
        rc = load_library().qeq_batched_phase_us(self._h, int(n_struct), buf)
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return np.array(buf[:], dtype=np.float64).reshape(n_struct, 8)

    def batched_ms(self, reset=True):
        """Kernel milliseconds of the batched solves since the last reset."""
        return load_library().qeq_batched_last_ms(self._h, 1 if reset else 0)

    PROFILE_KINDS = ("spread_r2c", "fft_rows_fwd", "fft_cols_green", "fft_rows_inv", "c2r",
                     "interp_pairs", "cg_update", "cg_dir", "final")

    def time_kernel(self, kind, reps=20):
        """Average microseconds of one launch of mesh pass `kind` (0 or 4; see qeq_time_kernel)."""
        us = ctypes.c_double()
        rc = load_library().qeq_time_kernel(self._h, int(kind), int(reps), ctypes.byref(us))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        return us.value

    def use_graphs(self, enable=True):
        """Replay the CG loop as a HIP graph (default) or launch kernels one by one."""
        load_library().qeq_use_graphs(self._h, 1 if enable else 0)

    def use_ewald(self, enable=True):
        """Reciprocal part by direct Ewald sums (True) or the particle mesh (False, default)."""
        rc = load_library().qeq_use_ewald(self._h, 1 if enable else 0)
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        self._last_n = None

    def use_sqnm(self, enable=True, history=10):
        """SQNM (True) or projected CG (False, default) for later solves."""
        rc = load_library().qeq_use_sqnm(self._h, 1 if enable else 0, int(history))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))

    def use_planewave(self, enable=True, support=6.0):
        """Gaussian-on-grid operator without the Ewald split (True) or the
        particle mesh (False, default); support: cut radius in sigma_i."""
        rc = load_library().qeq_use_planewave(self._h, 1 if enable else 0, float(support))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        self._last_n = None

    def use_spectral_preconditioner(self, k_cut=0.2):
        """Spectral (small-k Woodbury) preconditioner with cutoff k_cut in bohr^-1; 0 = Jacobi."""
        rc = load_library().qeq_use_spectral_preconditioner(self._h, float(k_cut))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))
        self._last_n = None

    def use_fused_inverse(self, enable=True):
        """Fused inverse axis-2 + complex-to-real slab pass where it fits (default) or two passes."""
        load_library().qeq_use_fused_inverse(self._h, 1 if enable else 0)

    def use_fused_forward(self, enable=True):
        """Fused spread + axis-3 + axis-2 forward plane pass where it fits (default) or two passes."""
        load_library().qeq_use_fused_forward(self._h, 1 if enable else 0)

    def set_tiles(self, spread_rows=0, tile_rows=0, fft_rows=0):
        """Tile widths of the mesh passes (0 = the built-in rule); see qeq_set_tiles."""
        rc = load_library().qeq_set_tiles(self._h, int(spread_rows), int(tile_rows), int(fft_rows))
        if rc != QEQ_OK:
            raise QEqError(rc, strerror(rc))

    def use_fused_interp(self, enable=True):
        """CG products: complex-to-real pass fused with the interpolation (default) or the grid path."""
        load_library().qeq_use_fused_interp(self._h, 1 if enable else 0)

    def profile(self, mask):
        """Bracket the launch kinds in ``mask`` with HIP events (see qeq_profile)."""
        load_library().qeq_profile(self._h, int(mask))

    def profile_read(self, reset=True):
        """{kind: (total ms, launches)} accumulated since the last reset."""
        ms = (ctypes.c_double * 16)()
        cnt = (ctypes.c_int64 * 16)()
        nk = load_library().qeq_profile_read(self._h, ms, cnt, 16, 1 if reset else 0)
        return {self.PROFILE_KINDS[k]: (ms[k], cnt[k]) for k in range(min(nk, len(self.PROFILE_KINDS)))}

    def matvec(self, pos, cell, sigma, v, parts=PART_ALL):
        """y = E v with the selected operator parts (see qeq_matvec)."""
        import torch
        n = int(pos.shape[0])
        for name, t, c in (("pos", pos, 3), ("sigma", sigma, None), ("v", v, None)):
            _check_dev(name, t, n, c, self.device)
        y = torch.empty(n, dtype=torch.float64, device=self.device)
        _, cp = _cell_arg(cell)
        rc = load_library().qeq_matvec(self._h, n, _ptr(pos), cp, _ptr(sigma), _ptr(v), _ptr(y),
                                       int(parts))
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return y


def _autograd_function():
    import torch

    class QEqFunction(torch.autograd.Function):
        """Differentiable QEq solve: (pos, chi, J) -> (q, [E_QEq, E_elec]).

        Forward runs qeq_solve; backward runs the adjoint (qeq_backward) on the
        same plan.  If another solve used the plan in between, the forward is
        replayed first to restore the tape.  sigma, the cell and Q_tot are
        treated as constants.
        """

        @staticmethod
        def forward(ctx, pos, chi, J, sigma, plan, cell, q_tot):
            q, en, _, st = plan.solve(pos.detach(), cell, sigma, J.detach(), chi.detach(), q_tot,
                                      forces=False)
            ctx.plan, ctx.cell, ctx.q_tot = plan, cell, q_tot
            ctx.solve_id = plan.solve_count
            ctx.save_for_backward(pos.detach(), chi.detach(), J.detach(), sigma)
            ctx.stats = st
            return q, en

        @staticmethod
        def backward(ctx, gq, gen):
            plan = ctx.plan
            pos, chi, J, sigma = ctx.saved_tensors
            if plan.solve_count != ctx.solve_id:
                plan.solve(pos, ctx.cell, sigma, J, chi, ctx.q_tot, forces=False)
            dq = gq.contiguous() if gq is not None else None
            e_qeq = float(gen[0]) if gen is not None else 0.0
            e_elec = float(gen[1]) if gen is not None else 0.0
            dchi, dJ, dpos, _ = plan.backward(dq, dL_dEelec=e_elec, dL_dEqeq=e_qeq)
            return dpos, dchi, dJ, None, None, None, None

    return QEqFunction


def qeq_autograd(pos, chi, J, sigma, plan, cell, q_tot=0.0):
    """q, energies = QEq(pos, chi, J) with gradients through the adjoint solve."""
    return _autograd_function().apply(pos, chi, J, sigma, plan, cell, q_tot)


MLP_STRIDE = 1664
MLP_OFFSETS = {"W1": (0, (32, 16)), "b1": (512, (32,)), "W2": (544, (32, 32)), "b2": (1568, (32,)),
               "W3": (1600, (32,)), "b3": (1632, ())}


def pack_mlp_params(nets):
    """Pack per-element {W1, b1, W2, b2, W3, b3} into the flat layout of include/qeq.h."""
    p = np.zeros(len(nets) * MLP_STRIDE, dtype=np.float32)
    for e, net in enumerate(nets):
        for k, (off, shape) in MLP_OFFSETS.items():
            a = np.asarray(net[k], dtype=np.float32).reshape(-1)
            p[e * MLP_STRIDE + off:e * MLP_STRIDE + off + a.size] = a
    return p


class WarmStartNet:
    """Per-element 16-32-32-1 warm-start networks on the device (mlp_* calls)."""

    def __init__(self, nets, device=None, stream=None):
        import torch
        self.n_species = len(nets)
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.params = torch.as_tensor(pack_mlp_params(nets), device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.stats = torch.zeros(self.n_species * 3 * 16, dtype=torch.float32, device=self.device)
        nws = load_library().mlp_workspace_floats(self.n_species)
        self.workspace = torch.empty(int(nws), dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def fit_scaling(self, G, species):
        rc = load_library().mlp_feature_stats(_ptr(G), _ptr(species), int(G.shape[0]), self.n_species,
                                              _ptr(self.stats), _ptr(self.workspace), self._s())
        if rc < 0:
            raise QEqError(rc, strerror(rc))

    def predict(self, G, species):
        import torch
        out = torch.empty(int(G.shape[0]), dtype=torch.float64, device=self.device)
        rc = load_library().mlp_forward(_ptr(G), _ptr(species), int(G.shape[0]), self.n_species,
                                        _ptr(self.params), _ptr(self.stats), _ptr(out), self._s())
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return out

    def train_step(self, G, species, target, lr=1e-3, update=True, grad_out=None):
        """One Adam step on the batch (or only loss / gradients if update=False)."""
        if update:
            self.step += 1
        rc = load_library().mlp_train_step(_ptr(G), _ptr(species), _ptr(target), int(G.shape[0]),
                                           self.n_species, _ptr(self.stats), _ptr(self.params),
                                           _ptr(self.m), _ptr(self.v), self.step if update else 0,
                                           float(lr), _ptr(self.workspace), int(self.workspace.numel()),
                                           _ptr(self.loss), _ptr(grad_out), self._s())
        if rc < 0:
            raise QEqError(rc, strerror(rc))
        return self.loss
