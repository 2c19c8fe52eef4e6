"""Writes tests/golden/n131072_frame100_reference.npz with the FP64 oracle (no GPU involved).

System: frame t = 100 (the first frame of the evaluation half) of the
131,072-atom trajectory workload (inputs.gen.md_initial, seed 1004; frame
t + 1 = frame t + N(0, 0.05 bohr) displacements; L = 235.7 bohr).  Its
electronegativities come from the workload's fixed random network applied to
radial descriptors (16 Gaussians of width 0.5 bohr centred at 1..9 bohr,
cosine cutoff 9 bohr: eq. g2 with the SI cosine cutoff), scaled by the
statistics of frame 0.  Here those descriptors are the oracle's own FP64
ones (oracle.mlp.radial_descriptors), so the stored chi is an oracle input,
not a GPU output.

The frame is solved with the matrix-free Ewald oracle (its own splitting
width eta_o = 4 bohr: the charges do not depend on it, which the oracle pins
prove, and 4 bohr keeps the real-space pair table within memory) and
projected CG to a relative residual of 1e-10.  Stored: chi (FP64, the input),
q (FP64), mu, E_QEq, E_elec, forces (FP32: the parity bar is a relative RMS
of 1e-4), CG iterations and residual.  Takes one to two hours on 8 CPU cores
and about 35 GB of memory.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import gen  # noqa: E402
from oracle import matfree, mlp  # noqa: E402

PATH = os.path.join(HERE, "n131072_frame100_reference.npz")
FRAME = 100
CENTERS = np.linspace(1.0, 9.0, 16)
WIDTH, R_DESC = 0.5, 9.0
ETA_ORACLE = 4.0


def frame_inputs(frame=FRAME):
    """(wrapped positions, cell, species, sigma, J, chi) of one trajectory frame."""
    pos0, cell, species, sigma, J = gen.md_initial()
    pos = pos0.copy()
    for t in range(frame):
        pos = pos + gen.md_displacement(t)
    t0 = time.time()
    G0 = mlp.radial_descriptors(gen.wrap_positions(pos0, cell), cell, CENTERS, WIDTH, R_DESC)
    _, scaling, y_std = gen.chi_from_descriptors(G0, species, gen.chi_network_weights(1004))
    del G0
    posw = gen.wrap_positions(pos, cell)
    G = mlp.radial_descriptors(posw, cell, CENTERS, WIDTH, R_DESC)
    chi, _, _ = gen.chi_from_descriptors(G, species, gen.chi_network_weights(1004), scaling, y_std)
    print(f"oracle descriptors (frames 0 and {frame}): {time.time() - t0:.0f} s", flush=True)
    return posw, cell, species, sigma, J, chi


def main():
    posw, cell, species, sigma, J, chi = frame_inputs()
    t0 = time.time()
    op = matfree.EwaldOperator(posw, cell, sigma, eta=ETA_ORACLE)
    print(f"oracle operator: {time.time() - t0:.0f} s, r_max {op.r_max:.1f}, "
          f"{op.K.nnz} pairs, modes {op.W.shape}", flush=True)
    apply0, calls, t0 = op.apply, [0], time.time()

    def apply_logged(v):
        calls[0] += 1
        if calls[0] % 10 == 0:
            print(f"  operator products: {calls[0]}, {time.time() - t0:.0f} s", flush=True)
        return apply0(v)

    op.apply = apply_logged
    r = matfree.qeq_matfree(posw, cell, sigma, J, chi, 0.0, tol=1e-10, forces=True, op=op)
    print(f"oracle solve: {time.time() - t0:.0f} s, {r.iters} CG iterations, "
          f"resid {r.rel_resid:.2e}", flush=True)
    np.savez_compressed(PATH, chi=chi, q=r.q, mu=r.mu, e_qeq=r.e_qeq, e_elec=r.e_elec,
                        forces=r.forces.astype(np.float32), rel_resid=r.rel_resid,
                        iters=r.iters, eta_oracle=ETA_ORACLE, frame=FRAME)


if __name__ == "__main__":
    main()
