"""Writes tests/golden/water64_oracle.npz: the CPU oracle's whole step on the
64-water workload (256 orbitals, 128^3 grid, R_pair = 5 A, R_PE = 4 A,
R_ME = 5 A, FP64, CG to 1e-10), every pair: its orbitals, energy
e_ij = h^3 sum_PE rho_ij v_ij (Sec. III.C Step V), CG iterations, flag and
true relative residual, and E_xx (Eq. exx_omega).

Calls only oracle/ and the seeded input generator; nothing of the HIP path.
About 2.5 CPU-hours (roughly 1 s per pair per core); run with
    python tests/golden/make_water64_oracle.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1911_10630_amd import synth as S         # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "water64_oracle.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    wl = S.c2_water64()
    phi = S.orbitals_np(wl)
    t0 = time.time()
    E, _, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi,
                      tol=wl.cg_rtol, nthreads=threads, want_D=False)
    dt = time.time() - t0
    np.savez_compressed(OUT, i=out["i"], j=out["j"], e=out["e"], iters=out["iters"], converged=out["converged"],
                        relres=out["relres"], E=np.float64(E), seconds=np.float64(dt),
                        workload=np.array(wl.name))
    print(f"{wl.name}: {len(out['e'])} pairs, E_xx = {E:.15f}, {dt:.0f} s -> {OUT}", flush=True)


if __name__ == "__main__":
    main()
