"""Seeded synthetic QEq workloads.

This module only draws random numbers and places atoms: it holds none of the
charge-equilibration arithmetic, so both the FP64 CPU oracle and the GPU path
can take their inputs from it without sharing any method code.

Units are atomic units throughout (bohr, Hartree, e), as in the paper's SI
(ZBL / data-storage paragraphs).  A cell is a 3x3 array whose ROWS are the
lattice vectors.  Positions are Cartesian, inside the cell.

Workloads (sizes and distributions follow the benchmark configurations):

* ``lattice_system`` -- jittered simple-cubic lattice, two elements with an
  exact 50/50 split assigned by a seeded permutation; sigma = {1.0, 1.5} bohr,
  J = {0.3, 0.5} Ha/e^2, chi ~ N(+-0.1, 0.05) Ha/e, Q_tot = 0.
  n_side=4, L=18.6 is the 64-atom case; n_side=32, L=148.6 the 32,768-atom
  case (density 0.01 bohr^-3); n_side=8, L=37.15 a 512-atom subset at the same
  density.
* ``batch_structure`` -- one member of the batched workload: triclinic cell,
  N ~ U{32..512}, three elements with Dirichlet(1,1,1) fractions.
* ``adjoint_targets`` -- loss weights w ~ U(0,1) and reference charges
  Q_ref ~ N(0, 0.2) for the differentiated workload.
* ``md_frames`` -- the 131,072-atom trajectory lattice and its displacements.
* ``cluster_system`` -- an isolated cluster (no cell) for non-periodic QEq:
  the N sites of a simple-cubic lattice at density 0.01 bohr^-3 nearest to the
  origin, jittered, two elements 50/50, a chosen total charge.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SIGMA_2EL = (1.0, 1.5)
J_2EL = (0.3, 0.5)
CHI_MEAN_2EL = (0.1, -0.1)

SIGMA_3EL = (1.0, 1.3, 1.7)
J_3EL = (0.3, 0.45, 0.6)
CHI_MEAN_3EL = (0.1, 0.0, -0.1)

CHI_SD = 0.05


@dataclasses.dataclass
class System:
    pos: np.ndarray        # (N,3) float64, Cartesian, bohr
    cell: np.ndarray       # (3,3) float64, rows = lattice vectors
    species: np.ndarray    # (N,) int32
    sigma: np.ndarray      # (N,) float64
    J: np.ndarray          # (N,) float64
    chi: np.ndarray        # (N,) float64
    q_tot: float
    grid: tuple            # FFT grid (K1, K2, K3)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def lattice_system(n_side: int, L: float, seed: int, grid=None, name="") -> System:
    """Jittered simple-cubic lattice, 2 elements 50/50, Q_tot = 0.

    Draw order: element permutation, jitter (N,3), chi noise (N,).
    Sites sit at (i + 1/2) * L / n_side; site order is x-major, z fastest.
    """
    rng = np.random.default_rng(seed)
    n = n_side ** 3
    a = L / n_side
    idx = np.arange(n_side)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    sites = (np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) + 0.5) * a
    species = rng.permutation(np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.int32))
    jitter = rng.uniform(-0.6, 0.6, size=(n, 3))
    noise = rng.normal(0.0, CHI_SD, size=n)
    pos = sites + jitter
    sigma = np.asarray(SIGMA_2EL)[species]
    J = np.asarray(J_2EL)[species]
    chi = np.asarray(CHI_MEAN_2EL)[species] + noise
    cell = np.eye(3) * L
    if grid is None:
        k = grid_dim(L, 0.8)
        grid = (k, k, k)
    return System(pos, cell, species.astype(np.int32), sigma, J, chi, 0.0, tuple(int(g) for g in grid), name)


def system_64() -> System:
    """64 atoms, 4^3 lattice, L = 18.6 bohr, 24^3 grid (seed 1000)."""
    return lattice_system(4, 18.6, 1000, grid=(24, 24, 24), name="n64_L18.6")


def system_32k() -> System:
    """32,768 atoms, 32^3 lattice, L = 148.6 bohr, 192^3 grid (seed 1001)."""
    return lattice_system(32, 148.6, 1001, grid=(192, 192, 192), name="n32768_L148.6")


def system_512(seed: int = 1001) -> System:
    """512 atoms, 8^3 lattice at the 32,768-atom density (L = 37.15), 48^3 grid."""
    return lattice_system(8, 8 * 148.6 / 32, seed, grid=(48, 48, 48), name="n512_L37.15")


def system_4096(seed: int = 1001) -> System:
    """4,096 atoms, 16^3 lattice at the same density (L = 74.3), 96^3 grid."""
    return lattice_system(16, 16 * 148.6 / 32, seed, grid=(96, 96, 96), name="n4096_L74.3")


# ---------------------------------------------------------------------------
# Grid sizing: dimensions are multiples of 4 whose prime factors are in {2,3,5}
# (the paper restricts grid dims to multiples of 4; radix set of the FFT).
# ---------------------------------------------------------------------------

def _smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def grid_dim(length: float, max_spacing: float) -> int:
    """Smallest multiple of 4 with factors in {2,3,5} and length/n <= max_spacing."""
    n = max(4, int(math.ceil(length / max_spacing - 1e-12)))
    n = (n + 3) // 4 * 4
    while not _smooth(n):
        n += 4
    return n


def perpendicular_widths(cell: np.ndarray) -> np.ndarray:
    """Distances between opposite faces of the cell (V / |a_b x a_c|)."""
    a, b, c = cell
    vol = abs(np.linalg.det(cell))
    return np.array([vol / np.linalg.norm(np.cross(b, c)),
                     vol / np.linalg.norm(np.cross(c, a)),
                     vol / np.linalg.norm(np.cross(a, b))])


def batch_structure(s: int, min_width: float = 18.0, max_spacing: float = 0.8) -> System:
    """Structure s of the batched workload (rng = default_rng([1002, s])).

    Draw order: N ~ U{32..512}; p ~ Dir(1,1,1); species ~ Cat(p); chi noise;
    Q_tot ~ U{-1,0,+1}; edge ratios U(0.8,1.25)^3; angles U(75,105)^3 deg;
    fractional positions U(0,1)^(N,3).  The cell is scaled to density 0.01
    bohr^-3, then scaled up further if a perpendicular width is below
    ``min_width`` (twice the 9-bohr cutoff), which lowers the density of the
    smallest structures.
    """
    rng = np.random.default_rng([1002, s])
    n = int(rng.integers(32, 513))
    p = rng.dirichlet([1.0, 1.0, 1.0])
    species = rng.choice(3, size=n, p=p).astype(np.int32)
    noise = rng.normal(0.0, CHI_SD, size=n)
    q_tot = float(rng.choice([-1, 0, 1]))
    ratios = rng.uniform(0.8, 1.25, size=3)
    angles = np.deg2rad(rng.uniform(75.0, 105.0, size=3))   # alpha(b,c), beta(a,c), gamma(a,b)
    frac = rng.uniform(0.0, 1.0, size=(n, 3))
    al, be, ga = angles
    ca, cb, cg = math.cos(al), math.cos(be), math.cos(ga)
    sg = math.sin(ga)
    cz2 = 1.0 - cb * cb - ((ca - cb * cg) / sg) ** 2
    if cz2 <= 0.05:       # keep the cell comfortably non-degenerate
        cz2 = 0.05
    unit = np.array([[1.0, 0.0, 0.0],
                     [cg, sg, 0.0],
                     [cb, (ca - cb * cg) / sg, math.sqrt(cz2)]])
    cell = unit * ratios[:, None]
    vol = abs(np.linalg.det(cell))
    cell = cell * (n / 0.01 / vol) ** (1.0 / 3.0)
    w = perpendicular_widths(cell).min()
    if w < min_width:
        cell = cell * (min_width / w)
    pos = frac @ cell
    sigma = np.asarray(SIGMA_3EL)[species]
    J = np.asarray(J_3EL)[species]
    chi = np.asarray(CHI_MEAN_3EL)[species] + noise
    lengths = np.linalg.norm(cell, axis=1)
    grid = tuple(grid_dim(float(l), max_spacing) for l in lengths)
    return System(pos, cell, species, sigma, J, chi, q_tot, grid, name=f"batch{s}")


def batch(n_struct: int = 1024, **kw) -> list:
    return [batch_structure(s, **kw) for s in range(n_struct)]


def adjoint_targets(n: int, seed: int = 1003):
    """Loss weights w ~ U(0,1) and reference charges Q_ref ~ N(0, 0.2)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 1.0, size=n)
    q_ref = rng.normal(0.0, 0.2, size=n)
    return w, q_ref


# ---------------------------------------------------------------------------
# MD-like trajectory workload (131,072 atoms, 51^3 lattice subset, L = 235.7)
# ---------------------------------------------------------------------------

MD_N = 131072
MD_SIDE = 51
MD_SPACING = 4.6216
MD_L = MD_SIDE * MD_SPACING


def md_initial(n: int = MD_N, side: int = MD_SIDE, spacing: float = MD_SPACING, seed: int = 1004):
    """Initial frame: a seeded n-subset of a side^3 simple-cubic lattice.

    Draw order (rng = default_rng(seed)): site subset, jitter U(-0.6,0.6),
    element permutation (exact 50/50).  Returns (pos_unwrapped, cell, species,
    sigma, J).  Electronegativities are produced per frame by a fixed network
    elsewhere, so none are drawn here.
    """
    rng = np.random.default_rng(seed)
    L = side * spacing
    n_sites = side ** 3
    chosen = np.sort(rng.choice(n_sites, size=n, replace=False))
    iz = chosen % side
    iy = (chosen // side) % side
    ix = chosen // (side * side)
    sites = (np.stack([ix, iy, iz], axis=1) + 0.5) * spacing
    jitter = rng.uniform(-0.6, 0.6, size=(n, 3))
    species = rng.permutation(np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.int32))
    pos = sites + jitter
    sigma = np.asarray(SIGMA_2EL)[species]
    J = np.asarray(J_2EL)[species]
    return pos, np.eye(3) * L, species.astype(np.int32), sigma, J


def md_displacement(t: int, n: int = MD_N, seed: int = 1004) -> np.ndarray:
    """Displacement from frame t to t+1: N(0, 0.05 bohr) per component."""
    rng = np.random.default_rng([seed, t])
    return rng.normal(0.0, 0.05, size=(n, 3))


def md_frame_positions(t: int, pos0: np.ndarray, n: int = MD_N, seed: int = 1004) -> np.ndarray:
    """Unwrapped positions of frame t (frame 0 = pos0)."""
    pos = pos0.copy()
    for s in range(t):
        pos += md_displacement(s, n, seed)
    return pos


def xavier_uniform(rng, fan_in: int, fan_out: int) -> np.ndarray:
    """Xavier/Glorot uniform initialisation (paper SI, initialisation section)."""
    lim = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-lim, lim, size=(fan_out, fan_in))


def chi_network_weights(seed: int = 1004):
    """Weights of the fixed random 16-32-1 tanh network that sets chi per frame.

    Drawn from default_rng([seed, 0]) in the order W1 (32x16), W2 (1x32);
    biases are zero.
    """
    rng = np.random.default_rng([seed, 0])
    W1 = xavier_uniform(rng, 16, 32)
    W2 = xavier_uniform(rng, 32, 1)
    return W1, np.zeros(32), W2, np.zeros(1)


def wrap_positions(pos: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """Wrap Cartesian positions into the cell (fractional coords in [0,1))."""
    frac = pos @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    return frac @ cell


def warmstart_init(seed: int = 1005, n_species: int = 2):
    """Initial weights of the per-element 16-32-32-1 warm-start networks.

    Xavier-uniform weights, zero biases (paper SI, initialisation section),
    drawn from default_rng(seed) in the order element, W1 (32x16), W2 (32x32),
    W3 (1x32).  Returns a list of dicts {W1, b1, W2, b2, W3, b3} per element.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_species):
        W1 = xavier_uniform(rng, 16, 32)
        W2 = xavier_uniform(rng, 32, 32)
        W3 = xavier_uniform(rng, 32, 1)
        out.append(dict(W1=W1, b1=np.zeros(32), W2=W2, b2=np.zeros(32), W3=W3[0], b3=0.0))
    return out


def chi_from_descriptors(G, species, weights, scaling=None, y_std=None):
    """Electronegativities of the trajectory workload from its descriptors.

    chi_i = m_e + 0.05 y_i / y_std with m_e = +0.1 / -0.1 for the two
    elements and y the fixed random 16-32-1 tanh network (``chi_network_weights``)
    applied to the descriptors scaled per feature by ``scaling`` = (mean, min,
    max) over all atoms.  With scaling / y_std None they are taken from this
    frame (the first frame) and returned, so that later frames reuse them.
    """
    W1, b1, W2, b2 = weights
    G = np.asarray(G, dtype=np.float64)
    if scaling is None:
        scaling = (G.mean(0), G.min(0), G.max(0))
    mean, mn, mx = scaling
    x = (G - mean) / np.where(mx - mn > 0, mx - mn, 1.0)
    y = (np.tanh(x @ W1.T + b1) @ W2.T + b2)[:, 0]
    if y_std is None:
        y_std = float(y.std())
    chi = np.asarray(CHI_MEAN_2EL)[species] + CHI_SD * y / y_std
    return chi, scaling, y_std


# ---------------------------------------------------------------------------
# Isolated clusters (non-periodic QEq)
# ---------------------------------------------------------------------------
CLUSTER_SPACING = 100.0 ** (1.0 / 3.0)   # bohr: density 0.01 bohr^-3


def cluster_system(n: int, q_tot: float = 0.0, seed: int = 1007, jitter: float = 0.6) -> System:
    """n atoms of a jittered simple-cubic lattice cut to a near-spherical cluster.

    Sites are the n lattice points (spacing 4.6416 bohr) nearest the origin,
    ordered by distance then x, y, z index (deterministic); draw order:
    element permutation (exact 50/50 split), jitter U(-jitter, jitter) per
    axis, chi noise.  sigma / J / chi means as the two-element workloads.
    ``cell`` and ``grid`` are None: the system is isolated.
    """
    rng = np.random.default_rng(seed)
    m = int(math.ceil((3.0 * n / (4.0 * math.pi)) ** (1.0 / 3.0))) + 2
    idx = np.arange(-m, m + 1)
    g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    r2 = (g * g).sum(1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], r2))
    sites = g[order[:n]].astype(np.float64) * CLUSTER_SPACING
    species = rng.permutation(np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.int32))
    pos = sites + rng.uniform(-jitter, jitter, size=(n, 3))
    noise = rng.normal(0.0, CHI_SD, size=n)
    sigma = np.asarray(SIGMA_2EL)[species]
    J = np.asarray(J_2EL)[species]
    chi = np.asarray(CHI_MEAN_2EL)[species] + noise
    return System(pos, None, species.astype(np.int32), sigma, J, chi, float(q_tot), None, f"cluster_n{n}")
