"""Inputs for the host-sanitizer driver: seeded systems and their oracle K
(test infrastructure: only the oracle computes the expected values).

File layout (little-endian): int32 nsys; per system int32 natom, nshell,
nprim, nbf, nhome_shell (0: molecular), nrow (rows of the reference K);
float64 xyz[3 natom]; int32 shells[4 nshell] (atom, l, nprim, prim_off);
float64 exps[nprim], coefs[nprim], P[nbf nbf], Kref[nrow nbf] (erfc omega
0.11, tau 1e-10; periodic systems: the home-cell rows of K^G)."""

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import hfx_inputs as hi  # noqa: E402
import oracle  # noqa: E402

OMEGA, TAU = 0.11, 1e-10


def systems():
    yield hi.sp8_cluster(), 0
    yield hi.lattice_system(8, seed=23, nprim_range=(1, 3)), 0
    cl = hi.periodic_cluster(natom_cell=1, reach=(1, 0, 0), lmax=2, nprim_range=(1, 2))
    yield cl, int(cl.meta["nhome_shell"])


def write(path):
    out = []
    for s, nh in systems():
        if nh:
            K, _ = oracle.build_K_periodic(s, tau=TAU, omega=OMEGA)
        else:
            K = oracle.build_K(s, tau=TAU, omega=OMEGA)[0]
        shells = np.stack([s.shell_atom, s.shell_l, s.shell_nprim, s.shell_off], axis=1).astype(np.int32)
        out.append((s, nh, shells, np.ascontiguousarray(K)))
    with open(path, "wb") as f:
        np.array([len(out)], dtype=np.int32).tofile(f)
        for s, nh, shells, K in out:
            np.array([s.natom, s.nshell, len(s.exps), s.nbf, nh, K.shape[0]], dtype=np.int32).tofile(f)
            for a, t in ((s.xyz, np.float64), (shells, np.int32), (s.exps, np.float64), (s.coefs, np.float64),
                         (s.P, np.float64), (K, np.float64)):
                np.ascontiguousarray(a, dtype=t).tofile(f)


if __name__ == "__main__":
    write(sys.argv[1])
    print("wrote", sys.argv[1], flush=True)
