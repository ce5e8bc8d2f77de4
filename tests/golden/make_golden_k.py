#!/usr/bin/env python3
"""Write the stored exchange matrices that the workload-scale parity tests
compare against.  Calls only the CPU oracle and the seeded input generators.

The system is the lattice recipe of the 256-atom benchmark workload (jittered
simple-cubic lattice, 4-bohr spacing, 2s+2p+1d shells of 3-6 primitives,
exponents log-uniform in [0.05, 20], sparse distance-damped P) at 27 atoms:
one full 3x3x3 block, 135 shells, 351 spherical functions.  The kernel is the
attenuated erfc(omega r)/r of HSE06 with omega = 0.11, the Schwarz threshold
1e-10, every primitive quartet evaluated (the oracle is exact).

Usage:  python tests/golden/make_golden_k.py [--threads N]
Output: tests/golden/k_lattice27_erfc.npz with K, Q and the screened quartet
counts, plus the generator arguments and a SHA-256 of K's bytes.
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import hfx_inputs as hi  # noqa: E402
import oracle  # noqa: E402

NATOM, SEED, TAU, OMEGA = 27, 1, 1e-10, 0.11
OUT = os.path.join(HERE, "k_lattice27_erfc.npz")


def system():
    return hi.lattice_system(NATOM, seed=SEED, name="lattice_dzp27")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    s = system()
    t0 = time.time()
    K, Q, cnt = oracle.build_K(s, tau=TAU, omega=OMEGA, nthreads=a.threads)
    dt = time.time() - t0
    sha = hashlib.sha256(np.ascontiguousarray(K).tobytes()).hexdigest()
    np.savez_compressed(OUT, K=K, Q=Q, quartets=np.int64(cnt["quartets"]),
                        prim_quartets=np.int64(cnt["prim_quartets"]),
                        class_quartets=np.asarray(cnt["per_class"], dtype=np.int64),
                        natom=NATOM, seed=SEED, tau=TAU, omega=OMEGA, sha256=sha,
                        oracle_seconds=dt)
    print(f"{OUT}: {s.nbf} functions, {cnt['quartets']} quartets, {dt:.0f} s, sha256 {sha}")


if __name__ == "__main__":
    main()
