"""Writes batch1024_samples.npz: FP64 oracle solutions of sampled structures
of the 1,024-structure batched workload (inputs.gen.batch).

Calls only the oracle (dense Ewald matrix + Gaussian elimination).  Samples:
the largest and the smallest structure, the first neutral, first anion and
first cation structure, and structures 511 and 1023.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
from inputs import gen          # noqa: E402
from oracle import ewald        # noqa: E402


def main():
    structs = gen.batch(1024)
    ns = np.array([s.n for s in structs])
    qt = np.array([s.q_tot for s in structs])
    idx = [int(ns.argmax()), int(ns.argmin()), int(np.flatnonzero(qt == 0)[0]),
           int(np.flatnonzero(qt == -1)[0]), int(np.flatnonzero(qt == 1)[0]), 511, 1023]
    idx = sorted(set(idx))
    out = {"index": np.array(idx)}
    for k in idx:
        s = structs[k]
        ref = ewald.qeq_dense(s.pos, s.cell, s.sigma, s.J, s.chi, s.q_tot)
        out[f"q{k}"] = ref.q
        out[f"e{k}"] = np.array([ref.e_qeq, ref.e_elec])
        out[f"f{k}"] = ref.forces
        print(k, s.n, s.grid, s.q_tot, ref.e_qeq, flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(__file__), "batch1024_samples.npz"), **out)


if __name__ == "__main__":
    main()
