"""Write config3_scf2.txt: two FP64 SCF iterations (protocol S) of config 3
(64-atom displaced diamond supercell, 90^3 box, 128 bands, Gamma) computed by
the oracle alone, for the GPU parity tests of the 128-band path: energies,
eigenvalues, and the output density at 2048 seeded grid points.

Usage (from the repository root): python tests/golden/make_config3_scf.py
Takes a few minutes on one core.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import energy as oe, scf as oscf  # noqa: E402

NIT = 2
NSAMPLE = 2048
SAMPLE_SEED = 3031


def sample_indices(size):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(size, NSAMPLE, replace=False))


def main():
    cell = W.config3()
    s = oe.build_system(cell)
    blocks = W.initial_wavefunctions(cell.y0_seed, [(cell.nb, b.npw) for b in s.bases])
    t0 = time.time()
    res = oscf.scf(s, [b.T.copy() for b in blocks], oe.start_density(cell, W.START_SIGMA), NIT)
    dt = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_scf2.txt")
    with open(out, "w") as f:
        f.write("# Config 3 (64-atom displaced diamond supercell, Ecut 15 Ha, 90^3, 128 bands, Gamma):\n")
        f.write(f"# {NIT} SCF iterations of protocol S (3 band-CG steps per iteration, Pulay mixing),\n")
        f.write("# FP64 oracle from the seeded start (written by tests/golden/make_config3_scf.py,\n")
        f.write(f"# which calls only oracle/; {dt:.0f} s).\n")
        for i, e in enumerate(res["energies"]):
            f.write(f"E_el {i} {e:.15e}\n")
        for i, e in enumerate(res["eigs"][0]):
            f.write(f"eig {i} {e:.15e}\n")
        f.write(f"n_out_abs_sum {float(np.sum(np.abs(res['n_out']))):.15e}\n")
        # the output density at NSAMPLE seeded grid points (flat row-major index)
        n = np.asarray(res["n_out"]).reshape(-1)
        for j in sample_indices(n.size):
            f.write(f"n_out {j} {n[j]:.15e}\n")
    print("wrote", out, f"{dt:.0f} s")


if __name__ == "__main__":
    main()
