"""Writes tests/golden/n32768_reference.npz with the FP64 oracle (no GPU involved).

System: the 32,768-atom jittered-lattice workload (seed 1001, L = 148.6 bohr)
from inputs.gen.system_32k().  Solved with the matrix-free Ewald oracle and
projected CG to a relative residual of 1e-10; stores charges, mu, E_QEq,
E_elec and forces.  Takes tens of minutes on a few CPU cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import gen  # noqa: E402
from oracle import matfree  # noqa: E402


def main():
    s = gen.system_32k()
    t0 = time.time()
    r = matfree.qeq_matfree(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot, tol=1e-10, forces=True)
    print(f"oracle solve: {time.time() - t0:.0f} s, {r.iters} CG iterations, resid {r.rel_resid:.2e}")
    np.savez_compressed(os.path.join(HERE, "n32768_reference.npz"), q=r.q, mu=r.mu, e_qeq=r.e_qeq,
                        e_elec=r.e_elec, forces=r.forces, rel_resid=r.rel_resid, iters=r.iters)


if __name__ == "__main__":
    main()
