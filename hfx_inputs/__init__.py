"""Seeded synthetic systems for the screened exchange build.

This module only draws random geometry, Gaussian shells and density matrices.
It holds none of the integral arithmetic: contraction coefficients are returned
raw (not normalised) and every consumer normalises them itself.

The paper's benchmark (bulk Si64 with SZ/DZP NAO2GTO shells and HSE06, Sec. 4)
needs pseudopotentials and fitted Gaussians that are not available here, so
these systems stand in for it: a DZP-like 2s+2p+1d shell set (13 spherical
functions per atom, the DZP count of the Si64 basis table in Sec. 4) on a
jittered cubic lattice, and a small s+p cluster for exact checks.

Basis-function order: shells in the order given, each shell contributing
2l+1 spherical functions (s: 1; p: x, y, z; d: m = -2..2, i.e. xy, yz, z2, xz,
x2-y2).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

__all__ = [
    "System",
    "tiny_sp_cluster",
    "lattice_system",
    "sp8_cluster",
    "dzp256_lattice",
    "dzp1024_lattice",
    "central_subset",
    "uneven_batch",
    "served_requests",
    "si64_like",
    "periodic_cluster",
    "OMEGA_HSE",
]

OMEGA_HSE = 0.11  # bohr^-1, the screening parameter of HSE06


@dataclasses.dataclass
class System:
    xyz: np.ndarray          # (natom, 3) float64, bohr
    shell_atom: np.ndarray   # (nshell,) int32
    shell_l: np.ndarray      # (nshell,) int32, 0..2
    shell_nprim: np.ndarray  # (nshell,) int32
    shell_off: np.ndarray    # (nshell,) int32, offset into exps/coefs
    exps: np.ndarray         # (nprim_total,) float64
    coefs: np.ndarray        # (nprim_total,) float64, raw (unnormalised)
    P: np.ndarray            # (nbf, nbf) float64, symmetric
    meta: dict

    @property
    def natom(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        return int(np.sum(2 * self.shell_l + 1))

    def bf_offsets(self) -> np.ndarray:
        n = 2 * self.shell_l.astype(np.int64) + 1
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)

    def bf_atom(self) -> np.ndarray:
        n = 2 * self.shell_l + 1
        return np.repeat(self.shell_atom, n)

    def subset_atoms(self, atoms) -> "System":
        """The same system restricted to `atoms` (shells and P rows/cols)."""
        atoms = np.asarray(sorted(int(a) for a in atoms))
        remap = -np.ones(self.natom, dtype=np.int64)
        remap[atoms] = np.arange(len(atoms))
        keep = np.isin(self.shell_atom, atoms)
        bfo = self.bf_offsets()
        bf_keep = np.concatenate([
            np.arange(bfo[s], bfo[s] + 2 * self.shell_l[s] + 1)
            for s in np.nonzero(keep)[0]
        ])
        sh = np.nonzero(keep)[0]
        nprim = self.shell_nprim[sh]
        off_new = np.concatenate([[0], np.cumsum(nprim)[:-1]]).astype(np.int32)
        exps = np.concatenate([self.exps[self.shell_off[s]:self.shell_off[s] + self.shell_nprim[s]] for s in sh])
        coefs = np.concatenate([self.coefs[self.shell_off[s]:self.shell_off[s] + self.shell_nprim[s]] for s in sh])
        return System(
            xyz=self.xyz[atoms].copy(),
            shell_atom=remap[self.shell_atom[sh]].astype(np.int32),
            shell_l=self.shell_l[sh].copy(),
            shell_nprim=nprim.astype(np.int32),
            shell_off=off_new,
            exps=exps,
            coefs=coefs,
            P=np.ascontiguousarray(self.P[np.ix_(bf_keep, bf_keep)]),
            meta=dict(self.meta, subset_of=self.meta.get("name"), natom=len(atoms)),
        )


def _pack(xyz, shells, P, meta) -> System:
    """shells: list of (atom, l, exps, coefs)."""
    nprim = np.array([len(s[2]) for s in shells], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(nprim)[:-1]]).astype(np.int32)
    return System(
        xyz=np.ascontiguousarray(xyz, dtype=np.float64),
        shell_atom=np.array([s[0] for s in shells], dtype=np.int32),
        shell_l=np.array([s[1] for s in shells], dtype=np.int32),
        shell_nprim=nprim,
        shell_off=off,
        exps=np.concatenate([np.asarray(s[2], dtype=np.float64) for s in shells]),
        coefs=np.concatenate([np.asarray(s[3], dtype=np.float64) for s in shells]),
        P=np.ascontiguousarray(P, dtype=np.float64),
        meta=meta,
    )


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))


def tiny_sp_cluster(seed: int = 0, natom: int = 8, box: float = 10.0, min_sep: float = 1.8,
                    nprim: int = 3, ls=(0, 1), alpha_range=(0.1, 10.0)) -> System:
    """Random cluster: atoms uniform in a cube (rejection-sampled to a minimum
    separation), each carrying one contracted shell per entry of `ls`.
    P = 2 C C^T with C the Q factor of a Gaussian random (nbf x nbf/4) matrix,
    so P is symmetric positive semidefinite."""
    rng = np.random.default_rng(seed)
    xyz = []
    while len(xyz) < natom:
        c = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(c - x) >= min_sep for x in xyz):
            xyz.append(c)
    xyz = np.array(xyz)
    shells = []
    for a in range(natom):
        for l in ls:
            e = _log_uniform(rng, alpha_range[0], alpha_range[1], nprim)
            c = rng.uniform(0.1, 1.0, size=nprim)
            shells.append((a, l, e, c))
    nbf = sum(2 * s[1] + 1 for s in shells)
    nocc = max(1, nbf // 4)
    q, _ = np.linalg.qr(rng.standard_normal((nbf, nocc)))
    P = 2.0 * q @ q.T
    P = 0.5 * (P + P.T)
    return _pack(xyz, shells, P, dict(name="tiny_sp_cluster", seed=seed, natom=natom))


def sp8_cluster(seed: int = 0) -> System:
    """8 atoms in a 10-bohr cube (min separation 1.8), one s and one p shell of
    3 primitives each (alpha log-uniform in [0.1, 10], c uniform in [0.1, 1]),
    32 functions; P = 2 C C^T from 8 random orthonormal columns."""
    s = tiny_sp_cluster(seed=seed)
    s.meta["name"] = "sp8_cluster"
    return s


def _lattice_xyz(natom: int, rng, spacing=4.0, jitter=0.3) -> np.ndarray:
    n = int(math.ceil(natom ** (1.0 / 3.0) - 1e-12))
    while n ** 3 < natom:
        n += 1
    sites = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                sites.append((i, j, k))
                if len(sites) == natom:
                    break
            if len(sites) == natom:
                break
        if len(sites) == natom:
            break
    base = spacing * np.array(sites, dtype=np.float64)
    return base + rng.uniform(-jitter, jitter, size=base.shape)


def lattice_system(natom: int, seed: int, lmax: int = 2, name: str = "lattice_dzp",
                   nprim_range=(3, 6), alpha_range=(0.05, 20.0), p_cut: float = 12.0,
                   p_decay: float = 3.0) -> System:
    """Jittered simple-cubic lattice (spacing 4 bohr, jitter +-0.3 bohr, x fastest),
    per atom 2s+2p(+1d if lmax==2) contracted shells with 3..6 primitives
    (alpha log-uniform in [0.05, 20], c uniform in [0.1, 1]).
    P: symmetric, entries uniform in [-1, 1] scaled by exp(-r_AB/3) and zeroed
    where the two functions' atoms are more than 12 bohr apart."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_xyz(natom, rng)
    ls = [0, 0, 1, 1] + ([2] if lmax >= 2 else [])
    shells = []
    for a in range(natom):
        for l in ls:
            npr = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            e = np.sort(_log_uniform(rng, alpha_range[0], alpha_range[1], npr))[::-1].copy()
            c = rng.uniform(0.1, 1.0, size=npr)
            shells.append((a, l, e, c))
    nbf = sum(2 * s[1] + 1 for s in shells)
    bf_atom = np.repeat(np.array([s[0] for s in shells]), [2 * s[1] + 1 for s in shells])
    S = rng.uniform(-1.0, 1.0, size=(nbf, nbf))
    S = np.triu(S) + np.triu(S, 1).T
    d = np.linalg.norm(xyz[bf_atom][:, None, :] - xyz[bf_atom][None, :, :], axis=-1)
    P = S * np.exp(-d / p_decay)
    P[d > p_cut] = 0.0
    return _pack(xyz, shells, P, dict(name=name, seed=seed, natom=natom, lmax=lmax))


def dzp256_lattice(seed: int = 1) -> System:
    """256-atom DZP-like lattice system, 1280 shells, 3328 functions."""
    return lattice_system(256, seed, name="dzp256_lattice")


def dzp1024_lattice(seed: int = 2) -> System:
    """The 256-atom lattice recipe at 1024 atoms, 13312 functions."""
    return lattice_system(1024, seed, name="dzp1024_lattice")


def central_subset(sys: System, natom: int = 128) -> System:
    """The `natom` atoms nearest the centroid (ties by index)."""
    c = sys.xyz.mean(axis=0)
    d = np.linalg.norm(sys.xyz - c, axis=1)
    order = np.lexsort((np.arange(sys.natom), d))
    return sys.subset_atoms(order[:natom])


def uneven_batch(seed: int = 3, nsys: int = 64, natom_range=(20, 400)) -> List[System]:
    """Independent systems of uneven size: atom counts uniform in natom_range,
    l_max uniform in {1, 2}, shells and P as in the 256-atom lattice (child seeds)."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nsys)
    out = []
    for i, ch in enumerate(children):
        r = np.random.default_rng(ch)
        n = int(r.integers(natom_range[0], natom_range[1] + 1))
        lmax = int(r.integers(1, 3))
        sub_seed = int(r.integers(0, 2**31 - 1))
        out.append(lattice_system(n, sub_seed, lmax=lmax, name=f"batch_sys{i}"))
    return out


def served_requests(seed: int = 4, nreq: int = 16, natom_range=(50, 2000), iters: int = 10):
    """Request descriptors for the serving workload: atom counts log-uniform in
    natom_range; each request is `iters` K-builds whose density matrices are
    P0 * (1 + 1e-3 E_t) with E_t symmetric standard normal. Returns a list of
    dicts with the child seed and size; the systems are built lazily by
    `lattice_system`."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nreq):
        n = int(round(math.exp(rng.uniform(math.log(natom_range[0]), math.log(natom_range[1])))))
        out.append(dict(id=i, natom=n, seed=int(rng.integers(0, 2**31 - 1)), iters=iters))
    return out


def perturbed_density(P0: np.ndarray, rng, rel: float = 1e-3) -> np.ndarray:
    E = rng.standard_normal(P0.shape)
    E = np.triu(E) + np.triu(E, 1).T
    return P0 * (1.0 + rel * E)


def periodic_cluster(natom_cell: int = 2, cell_len: float = 5.0, reach=(1, 1, 1), seed: int = 6,
                     lmax: int = 2, nprim_range=(1, 2), alpha_range=(0.3, 8.0), p_cut: float = 9.0,
                     p_decay: float = 2.0) -> System:
    """A periodic crystal (simple-cubic cell of side cell_len bohr holding
    natom_cell atoms, jittered lattice sites of the cell) written as a finite
    cluster of image cells n in [-reach, reach] (per axis), home cell first:
    atoms, shells and functions of cell (0, 0, 0) come first, then the other
    cells in lexicographic order of n.  Shells per atom as lattice_system
    (2s+2p+1d, or 2s+2p for lmax 1), identical in every image.

    The density matrix is periodic and Hermitian: P^R_{nu sigma} between
    nu of cell 0 and sigma of cell R is u * exp(-r/p_decay), zero beyond
    p_cut, with r the distance of the two functions' atoms and u uniform in
    [-1, 1] drawn once per (R, nu, sigma) with u(R, nu, sigma) = u(-R, sigma, nu).
    The cluster's P is P_big[(N, nu)][(H, sigma)] = P^{H-N}_{nu sigma}.
    meta: nhome_shell, ncell, cells (integer offsets in cluster order),
    nf_cell (functions per cell)."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(natom_cell ** (1.0 / 3.0) - 1e-12))
    sub = cell_len / max(m, 1)
    sites = [(i, j, k) for k in range(m) for j in range(m) for i in range(m)][:natom_cell]
    cell_xyz = (np.array(sites, dtype=np.float64) + 0.5) * sub + rng.uniform(-0.3, 0.3, size=(natom_cell, 3))
    ls = [0, 0, 1, 1] + ([2] if lmax >= 2 else [])
    cell_shells = []
    for a in range(natom_cell):
        for l in ls:
            npr = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            e = np.sort(_log_uniform(rng, alpha_range[0], alpha_range[1], npr))[::-1].copy()
            c = rng.uniform(0.1, 1.0, size=npr)
            cell_shells.append((a, l, e, c))
    rx, ry, rz = reach
    cells = [(0, 0, 0)] + [(i, j, k) for i in range(-rx, rx + 1) for j in range(-ry, ry + 1)
                           for k in range(-rz, rz + 1) if (i, j, k) != (0, 0, 0)]
    xyz, shells = [], []
    for ci, n in enumerate(cells):
        shift = cell_len * np.array(n, dtype=np.float64)
        xyz.extend(cell_xyz + shift)
        for (a, l, e, c) in cell_shells:
            shells.append((ci * natom_cell + a, l, e, c))
    xyz = np.array(xyz)
    nf = sum(2 * sh[1] + 1 for sh in cell_shells)
    f_atom = np.repeat([sh[0] for sh in cell_shells], [2 * sh[1] + 1 for sh in cell_shells])
    # u per cell difference R in [-2 reach, 2 reach], Hermitian: u(R) = u(-R)^T
    span = [2 * r for r in reach]
    diffs = [(i, j, k) for i in range(-span[0], span[0] + 1) for j in range(-span[1], span[1] + 1)
             for k in range(-span[2], span[2] + 1)]
    U = {R: rng.uniform(-1.0, 1.0, size=(nf, nf)) for R in diffs}
    PR = {}
    for R in diffs:
        mR = tuple(-x for x in R)
        u = 0.5 * (U[R] + U[mR].T)
        shift = cell_len * np.array(R, dtype=np.float64)
        d = np.linalg.norm(cell_xyz[f_atom][:, None, :] - (cell_xyz[f_atom][None, :, :] + shift), axis=-1)
        P = u * np.exp(-d / p_decay)
        P[d > p_cut] = 0.0
        PR[R] = P
    nc = len(cells)
    Pbig = np.zeros((nc * nf, nc * nf))
    for a, Na in enumerate(cells):
        for b, Hb in enumerate(cells):
            R = tuple(h - n_ for h, n_ in zip(Hb, Na))
            Pbig[a * nf:(a + 1) * nf, b * nf:(b + 1) * nf] = PR[R]
    Pbig = 0.5 * (Pbig + Pbig.T)  # exact symmetry (already Hermitian up to rounding)
    sysm = _pack(xyz, shells, Pbig, dict(name="periodic_cluster", seed=seed, natom_cell=natom_cell,
                                           cell_len=cell_len, reach=tuple(reach)))
    sysm.meta.update(nhome_shell=len(cell_shells), ncell=nc, cells=cells, nf_cell=nf)
    return sysm


def si64_like(basis: str = "SZ", seed: int = 5) -> System:
    """64 atoms with the Si64 shell counts of the paper's basis table:
    SZ = 1s+1p per atom, DZP = 2s+2p+1d per atom."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_xyz(64, rng, spacing=4.4)
    ls = [0, 1] if basis == "SZ" else [0, 0, 1, 1, 2]
    shells = []
    for a in range(64):
        for l in ls:
            shells.append((a, l, np.array([1.0, 0.3]), np.array([0.5, 0.5])))
    nbf = sum(2 * s[1] + 1 for s in shells)
    return _pack(xyz, shells, np.eye(nbf), dict(name=f"si64_like_{basis}", seed=seed))
