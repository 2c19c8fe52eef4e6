"""Writes tests/golden/n32768_reference.npz with the FP64 oracle (no GPU involved).

System: the 32,768-atom jittered-lattice workload (seed 1001, L = 148.6 bohr)
from inputs.gen.system_32k().  Solved with the matrix-free Ewald oracle and
projected CG to a relative residual of 1e-10; stores charges, mu, E_QEq,
E_elec, forces and the virial W = -dE_elec/d eps at those charges.  Takes
tens of minutes on a few CPU cores.  ``--virial-only`` adds the virial to an
existing file from its stored (oracle) charges.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import gen  # noqa: E402
from oracle import matfree  # noqa: E402


PATH = os.path.join(HERE, "n32768_reference.npz")


def oracle_virial(s, q):
    t0 = time.time()
    W = matfree.EwaldOperator(s.pos, s.cell, s.sigma).virial(q)
    print(f"oracle virial: {time.time() - t0:.0f} s")
    return W


def main():
    s = gen.system_32k()
    t0 = time.time()
    r = matfree.qeq_matfree(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot, tol=1e-10, forces=True)
    print(f"oracle solve: {time.time() - t0:.0f} s, {r.iters} CG iterations, resid {r.rel_resid:.2e}")
    np.savez_compressed(PATH, q=r.q, mu=r.mu, e_qeq=r.e_qeq, e_elec=r.e_elec, forces=r.forces,
                        rel_resid=r.rel_resid, iters=r.iters, virial=oracle_virial(s, r.q))


def add_virial():
    d = dict(np.load(PATH))
    d["virial"] = oracle_virial(gen.system_32k(), d["q"])
    np.savez_compressed(PATH, **d)


if __name__ == "__main__":
    if "--virial-only" in sys.argv[1:]:
        add_virial()
    else:
        main()
