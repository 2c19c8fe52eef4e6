"""Writes tests/golden/grid320_reference.npz with the FP64 oracle (no GPU involved).

System: 64 atoms on a 4^3 jittered lattice in the 235.7-bohr cube of the
131,072-atom trajectory workload (inputs.gen.lattice_system(4, 235.7, 1009)),
solved on the GPU with that workload's 320^3 grid: the mesh passes at this
grid length (their tile shapes differ from the smaller grids') are checked
against dense Ewald + Gaussian elimination.  Stores charges, mu, E_QEq,
E_elec, forces, and E v for a seeded vector v.  About a minute on one core.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import gen  # noqa: E402
from oracle import ewald  # noqa: E402

PATH = os.path.join(HERE, "grid320_reference.npz")


def system():
    return gen.lattice_system(4, 235.7, 1009, grid=(320, 320, 320), name="n64_L235.7")


def main():
    s = system()
    E = ewald.coulomb_matrix(s.pos, s.cell, s.sigma)
    q, lam = ewald.solve_qeq(E, s.J, s.chi, s.q_tot)
    ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
    assert np.abs(ref.q - q).max() < 1e-12
    v = np.random.default_rng(1010).normal(size=s.n)
    np.savez_compressed(PATH, q=ref.q, mu=ref.mu, e_qeq=ref.e_qeq, e_elec=ref.e_elec, forces=ref.forces,
                        v=v, Ev=E @ v)
    print("wrote", PATH)


if __name__ == "__main__":
    main()
