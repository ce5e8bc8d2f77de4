#!/usr/bin/env python3
"""Generate the per-class device code of the shell-quartet kernels.

For every angular-momentum class (la lb | lc ld) with l <= 2, la >= lb,
lc >= ld, this writes a struct with two straight-line device functions:

  vrr   one primitive quartet: the Obara-Saika vertical recurrence from the
        auxiliary integrals [00|00]^(m) to the targets [e0|f0]^(0) with
        la <= |e| <= la+lb and lc <= |f| <= lc+ld, accumulated into the
        contracted array (Head-Gordon-Pople order: vertical on primitives,
        horizontal after contraction).  Only the nodes the targets depend on
        are emitted; the decrement direction of every node is chosen so the
        dependency graph stays small.
  post  one contracted quartet: horizontal recurrence on the bra
        (b+1_i from a+1_i and A-B), spherical transform of the bra, then the
        same on the ket (C-D), giving (2la+1)(2lb+1)(2lc+1)(2ld+1) values.

The ket vertical step is optionally split into groups of f components
(`--split`): group g emits only the nodes its f targets need, so several lanes
can share one quartet, each holding a slice of the contracted array.

All index tables and coefficients are compile-time constants in the output,
so the device compiler keeps every intermediate in registers.  The file also
reports operation counts (an FMA counts two) used for the FLOP model.
"""

from __future__ import annotations

import argparse
import functools
import json
import math
import os
import random
import sys

LMAX = 2


def cart(l):
    """Cartesian monomials of degree l: x descending, then y descending."""
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def ncart(l):
    return (l + 1) * (l + 2) // 2


# Spherical rows on Cartesians normalised like x^l (p: x, y, z; d: m = -2..2).
R3 = math.sqrt(3.0)
SPH = {
    0: [{(0, 0, 0): 1.0}],
    1: [{(1, 0, 0): 1.0}, {(0, 1, 0): 1.0}, {(0, 0, 1): 1.0}],
    2: [{(1, 1, 0): R3}, {(0, 1, 1): R3}, {(0, 0, 2): 1.0, (2, 0, 0): -0.5, (0, 2, 0): -0.5},
        {(1, 0, 1): R3}, {(2, 0, 0): 0.5 * R3, (0, 2, 0): -0.5 * R3}],
}


def sub(t, i, k=1):
    l = list(t)
    l[i] -= k
    return tuple(l)


def add(t, i, k=1):
    l = list(t)
    l[i] += k
    return tuple(l)


def classes():
    pcs = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    out = []
    for cb in range(6):
        for ck in range(cb + 1):
            out.append(pcs[cb] + pcs[ck])
    return out


def fmt(x):
    r = repr(float(x))
    return r if ("." in r or "e" in r) else r + ".0"


class Emitter:
    def __init__(self, T="double"):
        self.lines = []
        self.flops = 0
        self.T = T

    def lit(self, x):
        s = fmt(x)
        return s + "f" if self.T == "float" else s


# ------------------------------------------------------------------ VRR ----
def vrr_graph(la, lb, lc, ld, f_targets=None, policy="auto", last="auto"):
    """Needed nodes (e, f, m) and each node's recurrence (direction, preds).

    `last` picks the side whose steps are applied last when both e and f are
    non-zero: "ket" builds [e0|00] first and raises f on top of it (with the
    coupling term to e - 1_i); "bra" builds [00|f0] first and raises e on top
    (coupling to f - 1_i).  For a slice that holds only some f components the
    "bra" order needs only the ket base of those components, while "ket"
    rebuilds the whole bra table in every slice."""
    E, F = la + lb, lc + ld
    L = E + F
    e_t = [e for d in range(la, E + 1) for e in cart(d)]
    f_all = [f for d in range(lc, F + 1) for f in cart(d)]
    f_t = f_all if f_targets is None else f_targets
    best = None
    policies = ["first", "small", "large", "last"] if policy == "auto" else [policy]
    lasts = ["ket", "bra"] if last == "auto" else [last]
    for pol, side in ((p_, s_) for s_ in lasts for p_ in policies):
        rec = {}

        def pick(t):
            nz = [i for i in range(3) if t[i] > 0]
            if pol == "first":
                return nz[0]
            if pol == "last":
                return nz[-1]
            if pol == "small":
                return min(nz, key=lambda i: (t[i], i))
            return max(nz, key=lambda i: (t[i], -i))

        order = []
        seen = set()

        def need(node):
            if node in seen:
                return
            e, f, m = node
            if sum(e) == 0 and sum(f) == 0:
                seen.add(node)
                rec[node] = ("base",)
                order.append(node)
                return
            if sum(f) > 0 and (side == "ket" or sum(e) == 0):
                i = pick(f)
                f1 = sub(f, i)
                preds = [("QC", i, (e, f1, m)), ("WQ", i, (e, f1, m + 1))]
                if f1[i] > 0:
                    f2 = sub(f1, i)
                    preds.append(("F2", i, f1[i], (e, f2, m), (e, f2, m + 1)))
                if e[i] > 0:
                    preds.append(("EX", i, e[i], (sub(e, i), f1, m + 1)))
                kind = "ket"
            else:
                i = pick(e)
                e1 = sub(e, i)
                preds = [("PA", i, (e1, f, m)), ("WP", i, (e1, f, m + 1))]
                if e1[i] > 0:
                    e2 = sub(e1, i)
                    preds.append(("E2", i, e1[i], (e2, f, m), (e2, f, m + 1)))
                if f[i] > 0:
                    preds.append(("FX", i, f[i], (e1, sub(f, i), m + 1)))
                kind = "bra"
            for p in preds:
                for x in p:
                    if isinstance(x, tuple) and len(x) == 3 and isinstance(x[0], tuple):
                        need(x)
            seen.add(node)
            rec[node] = (kind, preds)
            order.append(node)

        for f in f_t:
            for e in e_t:
                need((e, f, 0))
        cost = sum(_node_cost(rec[n]) for n in order)
        if best is None or cost < best[0]:
            best = (cost, rec, order, (pol, side))
    return best[1], best[2], e_t, f_t, best[0]


def _node_cost(r):
    """Selection weight of a node (recurrence order, slice partitions): twice
    its instruction count (a product-sum of t terms issues t instructions,
    a c (v - r w) term one more)."""
    if r[0] == "base":
        return 1
    n = 0
    for p in r[1]:
        n += 4 if p[0] in ("F2", "E2") else 2
    return n


def _node_flops(r):
    """Arithmetic of one node: the products of its terms (c (v - r w) is two
    products and a difference), plus one addition fewer than it has terms."""
    if r[0] == "base":
        return 1  # pref * G_m
    n = 0
    for p in r[1]:
        if p[0] in ("QC", "WQ", "PA", "WP", "EX", "FX"):
            n += 1
        elif p[0] in ("F2", "E2"):
            n += 3
    return n + len(r[1]) - 1


def emit_vrr(em, la, lb, lc, ld, name, f_targets=None, policy="auto"):
    rec, order, e_t, f_t, cost = vrr_graph(la, lb, lc, ld, f_targets, policy)
    T = em.T
    L = la + lb + lc + ld
    ids = {n: k for k, n in enumerate(order)}
    # nodes that another node reads; a target read by none is summed straight
    # into its accumulator (acc + t1 + t2 ... contracts to multiply-adds)
    used = set()
    for n in order:
        r = rec[n]
        if r[0] != "base":
            for p in r[1]:
                for x in p:
                    if isinstance(x, tuple) and len(x) == 3 and isinstance(x[0], tuple):
                        used.add(x)
    acc_index = {}
    k = 0
    for e in e_t:
        for f in f_t:
            acc_index[(e, f)] = k
            k += 1
    nacc = k
    ax = "xyz"
    em.lines.append(f"  __device__ __forceinline__ static void {name}(const {T}* __restrict__ g,")
    em.lines.append(f"      {T} PAx, {T} PAy, {T} PAz, {T} WPx, {T} WPy, {T} WPz,")
    em.lines.append(f"      {T} QCx, {T} QCy, {T} QCz, {T} WQx, {T} WQy, {T} WQz,")
    em.lines.append(f"      {T} i2z, {T} roz, {T} i2e, {T} roe, {T} i2ze, {T}* __restrict__ acc) {{")
    for n in order:
        r = rec[n]
        e, f, m = n
        v = f"v{ids[n]}"
        if r[0] == "base":
            em.lines.append(f"    const {T} {v} = g[{m}];")
            if m == 0 and (e, f) in acc_index:
                em.lines.append(f"    acc[{acc_index[(e, f)]}] += {v};")
            continue
        terms = []
        for p in r[1]:
            tag = p[0]
            if tag in ("QC", "WQ", "PA", "WP"):
                terms.append(f"{tag}{ax[p[1]]} * v{ids[p[2]]}")
            elif tag == "F2":
                c = p[2]
                coef = "i2e" if c == 1 else f"({em.lit(c)} * i2e)"
                terms.append(f"{coef} * (v{ids[p[3]]} - roe * v{ids[p[4]]})")
            elif tag == "E2":
                c = p[2]
                coef = "i2z" if c == 1 else f"({em.lit(c)} * i2z)"
                terms.append(f"{coef} * (v{ids[p[3]]} - roz * v{ids[p[4]]})")
            elif tag in ("EX", "FX"):
                c = p[2]
                coef = "i2ze" if c == 1 else f"({em.lit(c)} * i2ze)"
                terms.append(f"{coef} * v{ids[p[3]]}")
        if m == 0 and (e, f) in acc_index and n not in used:
            k = acc_index[(e, f)]
            em.lines.append(f"    acc[{k}] = acc[{k}] + " + " + ".join(terms) + ";")
            continue
        em.lines.append(f"    const {T} {v} = " + " + ".join(terms) + ";")
        if m == 0 and (e, f) in acc_index:
            # accumulate a target as soon as it exists: its value dies here
            em.lines.append(f"    acc[{acc_index[(e, f)]}] += {v};")
    em.lines.append("  }")
    flops = sum(_node_flops(rec[n]) for n in order)
    return nacc, flops + nacc  # accumulation adds


# --------------------------------------------------------- HRR + sph ----
def hrr_plan(la, lb):
    """Nodes (e, b) needed for the targets (a, b), |a| = la, |b| = lb, with
    (e, b+1_i) = (e+1_i, b) + AB_i (e, b)."""
    rec = {}
    order = []

    def need(n):
        if n in rec:
            return
        e, b = n
        if sum(b) == 0:
            rec[n] = ("base",)
            order.append(n)
            return
        i = [k for k in range(3) if b[k] > 0][0]
        b1 = sub(b, i)
        p1, p2 = (add(e, i), b1), (e, b1)
        need(p1)
        need(p2)
        rec[n] = ("hrr", i, p1, p2)
        order.append(n)

    for a in cart(la):
        for b in cart(lb):
            need((a, b))
    return rec, order


def emit_post(em, la, lb, lc, ld, name="post"):
    """acc[ie*NF + jf] (ie over bra e components la..la+lb, jf over ket f
    components lc..lc+ld)  ->  out[((as*nbs+bs)*ncs+cs)*nds+ds]."""
    T = em.T
    E, F = la + lb, lc + ld
    e_list = [e for d in range(la, E + 1) for e in cart(d)]
    f_list = [f for d in range(lc, F + 1) for f in cart(d)]
    eidx = {e: k for k, e in enumerate(e_list)}
    fidx = {f: k for k, f in enumerate(f_list)}
    NF = len(f_list)
    nas, nbs, ncs, nds = 2 * la + 1, 2 * lb + 1, 2 * lc + 1, 2 * ld + 1
    ax = "xyz"
    em.lines.append(f"  __device__ __forceinline__ static void {name}(const {T}* __restrict__ acc,")
    em.lines.append(f"      {T} ABx, {T} ABy, {T} ABz, {T} CDx, {T} CDy, {T} CDz, {T}* __restrict__ out) {{")
    flops = 0
    brec, border = hrr_plan(la, lb)
    krec, korder = hrr_plan(lc, ld)
    # bra HRR + bra spherical for every f component
    for jf in range(NF):
        names = {}
        for k, n in enumerate(border):
            r = brec[n]
            nm = f"b{jf}_{k}"
            names[n] = nm
            if r[0] == "base":
                names[n] = f"acc[{eidx[n[0]] * NF + jf}]"
                continue
            _, i, p1, p2 = r
            em.lines.append(f"    const {T} {nm} = {names[p1]} + AB{ax[i]} * {names[p2]};")
            flops += 2
        for as_ in range(nas):
            for bs in range(nbs):
                terms = []
                for a, ca in SPH[la][as_].items():
                    for b, cb in SPH[lb][bs].items():
                        c = ca * cb
                        nm = names[(a, b)]
                        terms.append(nm if c == 1.0 else f"{em.lit(c)} * {nm}")
                        flops += 0 if c == 1.0 else 1
                flops += len(terms) - 1
                em.lines.append(f"    const {T} s{as_}_{bs}_{jf} = " + " + ".join(terms) + ";")
    # ket HRR + ket spherical for every bra spherical pair
    for as_ in range(nas):
        for bs in range(nbs):
            names = {}
            for k, n in enumerate(korder):
                r = krec[n]
                if r[0] == "base":
                    names[n] = f"s{as_}_{bs}_{fidx[n[0]]}"
                    continue
                nm = f"k{as_}_{bs}_{k}"
                names[n] = nm
                _, i, p1, p2 = r
                em.lines.append(f"    const {T} {nm} = {names[p1]} + CD{ax[i]} * {names[p2]};")
                flops += 2
            for cs in range(ncs):
                for ds in range(nds):
                    terms = []
                    for c_, cc in SPH[lc][cs].items():
                        for d_, cd in SPH[ld][ds].items():
                            c = cc * cd
                            nm = names[(c_, d_)]
                            terms.append(nm if c == 1.0 else f"{em.lit(c)} * {nm}")
                            flops += 0 if c == 1.0 else 1
                    flops += len(terms) - 1
                    o = ((as_ * nbs + bs) * ncs + cs) * nds + ds
                    em.lines.append(f"    out[{o}] = " + " + ".join(terms) + ";")
    em.lines.append("  }")
    return flops


def emit_digest_part(em, la, lb, lc, ld, name, f_part, mode="K"):
    """Streaming digestion of one slice of the contracted array.

    mode "K": exchange (below).  mode "J": the Coulomb digestion of the same
    shares, J'_ab += 2 d v P_cd and J'_cd += 2 d v P_ab (J = J' + J'^T).
    mode "R": exchange rows chosen per call (periodic builds): the four sums
    of mode "K" are added with weights wA, wB to rows of A and B and, P being
    symmetric, the same sums with weights wC, wD to rows of C and D
    (K_ca += wC v P_db = wC v P_bd, ...); P and K have their own leading
    dimensions and no K' + K'^T follows.

    acc holds [e|f] for every bra e (la..la+lb) and the ket components f in
    `f_part` (layout e-major).  The bra horizontal recurrence and spherical
    transform are applied per f; the ket recurrence and transform are linear,
    so applying them to the slice (other f taken as zero) gives this slice's
    share of every spherical value, which is digested at once:
      K'_ac += d v P_bd, K'_ad += d v P_bc, K'_bc += d v P_ad, K'_bd += d v P_ac.
    Shares of all slices add up in K' through the atomics."""
    # the contracted array may be FP32 (mixed mode); the horizontal
    # recurrence, spherical transform and digestion always run in FP64 (once
    # per contracted quartet, a small share of the work)
    T = "double"
    AT = em.T
    E, F = la + lb, lc + ld
    e_list = [e for d in range(la, E + 1) for e in cart(d)]
    eidx = {e: k for k, e in enumerate(e_list)}
    fidx = {f: k for k, f in enumerate(f_part)}
    NF = len(f_part)
    nas, nbs, ncs, nds = 2 * la + 1, 2 * lb + 1, 2 * lc + 1, 2 * ld + 1
    ax = "xyz"
    L = em.lines
    L.append(f"  __device__ __forceinline__ static void {name}(const {AT}* __restrict__ acc,")
    if mode == "E":
        # raw values: this slice's share of every spherical value is added to
        # out[(as nbs + bs) sab + (cs nds + ds) scd] (the caller's lane-private
        # output, strides chosen by the caller so exchanged classes land in the
        # original index order)
        L.append(f"      {T} ABx, {T} ABy, {T} ABz, {T} CDx, {T} CDy, {T} CDz, int64_t sab, int64_t scd,")
        L.append("      double* __restrict__ out) {")
    elif mode == "R":
        L.append(f"      {T} ABx, {T} ABy, {T} ABz, {T} CDx, {T} CDy, {T} CDz, int a0, int b0, int c0, int d0,")
        L.append("      double wA, double wB, double wC, double wD, const double* __restrict__ P, int64_t ldP,")
        L.append("      double* K, int64_t ldK) {")
    else:
        L.append(f"      {T} ABx, {T} ABy, {T} ABz, {T} CDx, {T} CDy, {T} CDz, int a0, int b0, int c0, int d0,")
        L.append(f"      double deg, const double* __restrict__ P, double* K, int64_t ld) {{")
    brec, border = hrr_plan(la, lb)
    krec, korder = hrr_plan(lc, ld)
    jtouched = set()
    if mode == "J":
        # K is the Coulomb matrix here; P_cd of the ket pair is read once
        L.append("    const double deg2 = 2.0 * deg;")
        for cs in range(ncs):
            for ds in range(nds):
                L.append(f"    const double pcd{cs}_{ds} = P[(int64_t)(c0 + {cs}) * ld + d0 + {ds}];")
                L.append(f"    double jcd{cs}_{ds} = 0.0;")
    # bra HRR + spherical for every f of the slice
    for jf, f in enumerate(f_part):
        names = {}
        for k, n in enumerate(border):
            r = brec[n]
            if r[0] == "base":
                names[n] = f"acc[{eidx[n[0]] * NF + jf}]"
                continue
            nm = f"b{jf}_{k}"
            names[n] = nm
            _, i, p1, p2 = r
            L.append(f"    const {T} {nm} = {names[p1]} + AB{ax[i]} * {names[p2]};")
        for as_ in range(nas):
            for bs in range(nbs):
                terms = []
                for a, ca in SPH[la][as_].items():
                    for b, cb in SPH[lb][bs].items():
                        c = ca * cb
                        nm = names[(a, b)]
                        terms.append(nm if c == 1.0 else f"{fmt(c)} * {nm}")
                L.append(f"    const {T} s{as_}_{bs}_{jf} = " + " + ".join(terms) + ";")
    # ket HRR + spherical with the missing f as structural zeros, then digestion
    ldp = "ldP" if mode == "R" else "ld"
    if mode in ("K", "R"):
        for bs in range(nbs):
            for ks in ("c", "d"):
                n = ncs if ks == "c" else nds
                for x in range(n):
                    L.append(f"    double kb{ks}{bs}_{x} = 0.0;")
    for as_ in range(nas):
        if mode in ("D", "E"):
            L.append("    {")
        else:
            L.append(f"    {{ const double* Pa = P + (int64_t)(a0 + {as_}) * {ldp};")
        if mode in ("K", "R"):
            L.append("      double kac[%d] = {0}; double kad[%d] = {0};" % (ncs, nds))
        for bs in range(nbs):
            if mode in ("D", "E"):
                L.append("      {")
            else:
                L.append(f"      {{ const double* Pb = P + (int64_t)(b0 + {bs}) * {ldp};")
            names = {}
            for k, n in enumerate(korder):
                r = krec[n]
                if r[0] == "base":
                    names[n] = f"s{as_}_{bs}_{fidx[n[0]]}" if n[0] in fidx else None
                    continue
                _, i, p1, p2 = r
                x1, x2 = names[p1], names[p2]
                if x1 is None and x2 is None:
                    names[n] = None
                    continue
                nm = f"k{as_}_{bs}_{k}"
                names[n] = nm
                if x2 is None:
                    L.append(f"        const {T} {nm} = {x1};")
                elif x1 is None:
                    L.append(f"        const {T} {nm} = CD{ax[i]} * {x2};")
                else:
                    L.append(f"        const {T} {nm} = {x1} + CD{ax[i]} * {x2};")
            vals = {}
            for cs in range(ncs):
                for ds in range(nds):
                    terms = []
                    for c_, cc in SPH[lc][cs].items():
                        for d_, cd in SPH[ld][ds].items():
                            c = cc * cd
                            nm = names[(c_, d_)]
                            if nm is None:
                                continue
                            terms.append(nm if c == 1.0 else f"{fmt(c)} * {nm}")
                    if terms:
                        v = f"v{as_}_{bs}_{cs}_{ds}"
                        L.append(f"        const double {v} = " + " + ".join(terms) + ";")
                        vals[(cs, ds)] = v
            if mode == "D":
                # Schwarz diagonal (ab|ab): K is the diagonal accumulator here
                if (as_, bs) in vals:
                    L.append(f"        K[{as_ * nbs + bs}] += {vals[(as_, bs)]};")
                L.append("      }")
                continue
            if mode == "E":
                for (cs, ds) in sorted(vals):
                    L.append(f"        out[{as_ * nbs + bs} * sab + {cs * nds + ds} * scd] += {vals[(cs, ds)]};")
                L.append("      }")
                continue
            if mode == "J":
                if vals:
                    L.append(f"        const double pab = Pa[b0 + {bs}];")
                    L.append("        const double jab = " + " + ".join(
                        f"{vals[k]} * pcd{k[0]}_{k[1]}" for k in sorted(vals)) + ";")
                    L.append(f"        atomicAdd(&K[(int64_t)(a0 + {as_}) * ld + b0 + {bs}], deg2 * jab);")
                    for (cs, ds) in sorted(vals):
                        L.append(f"        jcd{cs}_{ds} += {vals[(cs, ds)]} * pab;")
                        jtouched.add((cs, ds))
                L.append("      }")
                continue
            for cs in range(ncs):
                t1 = [f"{vals[(cs, ds)]} * Pb[d0 + {ds}]" for ds in range(nds) if (cs, ds) in vals]
                t2 = [f"{vals[(cs, ds)]} * Pa[d0 + {ds}]" for ds in range(nds) if (cs, ds) in vals]
                if t1:
                    L.append(f"        kac[{cs}] += " + " + ".join(t1) + ";")
                    L.append(f"        kbc{bs}_{cs} += " + " + ".join(t2) + ";")
            for ds in range(nds):
                t1 = [f"{vals[(cs, ds)]} * Pb[c0 + {cs}]" for cs in range(ncs) if (cs, ds) in vals]
                t2 = [f"{vals[(cs, ds)]} * Pa[c0 + {cs}]" for cs in range(ncs) if (cs, ds) in vals]
                if t1:
                    L.append(f"        kad[{ds}] += " + " + ".join(t1) + ";")
                    L.append(f"        kbd{bs}_{ds} += " + " + ".join(t2) + ";")
            L.append("      }")
        if mode in ("J", "D", "E"):
            L.append("    }")
            continue
        if mode == "R":
            L.append(f"      if (wA != 0.0) {{ double* Ka = K + (int64_t)(a0 + {as_}) * ldK;")
            L.append(f"        for (int x = 0; x < {ncs}; ++x) atomicAdd(&Ka[c0 + x], wA * kac[x]);")
            L.append(f"        for (int x = 0; x < {nds}; ++x) atomicAdd(&Ka[d0 + x], wA * kad[x]); }}")
            L.append(f"      if (wC != 0.0) for (int x = 0; x < {ncs}; ++x)")
            L.append(f"        atomicAdd(&K[(int64_t)(c0 + x) * ldK + a0 + {as_}], wC * kac[x]);")
            L.append(f"      if (wD != 0.0) for (int x = 0; x < {nds}; ++x)")
            L.append(f"        atomicAdd(&K[(int64_t)(d0 + x) * ldK + a0 + {as_}], wD * kad[x]);")
            L.append("    }")
            continue
        L.append(f"      double* Ka = K + (int64_t)(a0 + {as_}) * ld;")
        L.append(f"      for (int x = 0; x < {ncs}; ++x) atomicAdd(&Ka[c0 + x], deg * kac[x]);")
        L.append(f"      for (int x = 0; x < {nds}; ++x) atomicAdd(&Ka[d0 + x], deg * kad[x]);")
        L.append("    }")
    if mode in ("D", "E"):
        L.append("  }")
        return
    if mode == "J":
        for cs in range(ncs):
            for ds in range(nds):
                if (cs, ds) in jtouched:
                    L.append(f"    atomicAdd(&K[(int64_t)(c0 + {cs}) * ld + d0 + {ds}], deg2 * jcd{cs}_{ds});")
        L.append("  }")
        return
    if mode == "R":
        for bs in range(nbs):
            L.append(f"    if (wB != 0.0) {{ double* Kb = K + (int64_t)(b0 + {bs}) * ldK;")
            for cs in range(ncs):
                L.append(f"      atomicAdd(&Kb[c0 + {cs}], wB * kbc{bs}_{cs});")
            for ds in range(nds):
                L.append(f"      atomicAdd(&Kb[d0 + {ds}], wB * kbd{bs}_{ds});")
            L.append("    }")
            L.append("    if (wC != 0.0) {")
            for cs in range(ncs):
                L.append(f"      atomicAdd(&K[(int64_t)(c0 + {cs}) * ldK + b0 + {bs}], wC * kbc{bs}_{cs});")
            L.append("    }")
            L.append("    if (wD != 0.0) {")
            for ds in range(nds):
                L.append(f"      atomicAdd(&K[(int64_t)(d0 + {ds}) * ldK + b0 + {bs}], wD * kbd{bs}_{ds});")
            L.append("    }")
        L.append("  }")
        return
    for bs in range(nbs):
        L.append(f"    {{ double* Kb = K + (int64_t)(b0 + {bs}) * ld;")
        for cs in range(ncs):
            L.append(f"      atomicAdd(&Kb[c0 + {cs}], deg * kbc{bs}_{cs});")
        for ds in range(nds):
            L.append(f"      atomicAdd(&Kb[d0 + {ds}], deg * kbd{bs}_{ds});")
        L.append("    }")
    L.append("  }")


@functools.lru_cache(maxsize=None)
def _slice_cost(la, lb, lc, ld, part):
    r = vrr_graph(la, lb, lc, ld, f_targets=list(part))
    return r[4], len(r[1])


def _refine_split(la, lb, lc, ld, parts, f_list, iters=400):
    """Seeded local search over swaps and moves of components between slices:
    keep a partition whose summed recurrence cost is lower while its largest
    slice (cost within 2 %, live values) is no worse and no slice grows
    beyond the largest one (the registers a slice's array takes); used only
    if it saves more than 2 % of the summed cost."""
    pos = {f: k for k, f in enumerate(f_list)}

    def score(ps):
        c = [_slice_cost(la, lb, lc, ld, p) for p in ps]
        return sum(x[0] for x in c), max(x[0] for x in c), max(x[1] for x in c)

    best = [tuple(p) for p in parts]
    base = best_sc = score(best)
    maxsize = max(len(p) for p in parts)
    rnd = random.Random(1)
    G = len(parts)
    for _ in range(iters):
        ps = [list(p) for p in best]
        a, b = rnd.sample(range(G), 2)
        if rnd.random() < 0.7:
            i, j = rnd.randrange(len(ps[a])), rnd.randrange(len(ps[b]))
            ps[a][i], ps[b][j] = ps[b][j], ps[a][i]
        elif len(ps[a]) > 1 and len(ps[b]) < maxsize:
            ps[b].append(ps[a].pop(rnd.randrange(len(ps[a]))))
        else:
            continue
        ps = [tuple(sorted(p, key=pos.get)) for p in ps]
        sc = score(ps)
        if sc[0] < best_sc[0] and sc[1] <= base[1] * 1.02 and sc[2] <= base[2]:
            best, best_sc = ps, sc
    # a gain of a few per cent in the model is within what register
    # allocation moves either way (measured: (dp|dp) -1 % model, +3 % time)
    if best_sc[0] > 0.98 * base[0]:
        return [list(p) for p in parts]
    return [list(p) for p in best]


@functools.lru_cache(maxsize=None)
def _best_split(la, lb, lc, ld, G):
    f_list = [f for d in range(lc, lc + ld + 1) for f in cart(d)]
    orders = [f_list,
              sorted(f_list, key=lambda f: (f[2], f[1], f[0])),
              sorted(f_list, key=lambda f: (-f[0], -f[1], sum(f))),
              sorted(f_list, key=lambda f: (sum(f), f[2], f[1]))]
    best = None
    for od in orders:
        n = len(od)
        parts = [od[(g * n) // G:((g + 1) * n) // G] for g in range(G)]
        costs = [vrr_graph(la, lb, lc, ld, f_targets=p)[4] for p in parts]
        key = (max(costs), sum(costs))
        if best is None or key < best[0]:
            best = (key, parts)
    parts = best[1]
    if G >= 3:
        parts = _refine_split(la, lb, lc, ld, parts, f_list)
    return tuple(tuple(p) for p in parts)


def best_split(la, lb, lc, ld, G):
    """Partition the ket f components into G slices.  Candidate orders of the
    components are tried and the one with the smallest largest-slice
    recurrence cost is kept; for three or more slices a local search then
    lowers the summed cost of the slices."""
    return [list(p) for p in _best_split(la, lb, lc, ld, G)]


PAIR_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]

# Number of ket slices (waves) per quartet for the classes whose contracted
# array does not fit one lane's registers.  Measured on the 256-atom DZP
# shard: more slices recompute more of the shared recurrence; fewer spill
# registers to scratch, mostly 2-3x slower, though (dd|dd) in 10 slices
# (2.7 KB of scratch per lane) runs 10 % faster than in 12 and 3 % faster
# than in 9.
DEFAULT_SPLITS = {
    (2, 1, 1, 1): 2, (2, 1, 2, 0): 1, (2, 2, 1, 0): 1, (2, 2, 2, 0): 3,
    (2, 1, 2, 1): 3, (2, 2, 1, 1): 3, (2, 2, 2, 1): 5, (2, 2, 2, 2): 10,
}

# Override for tuning: HFX_SPLITS="2221:16,2222:32".
for _kv in filter(None, os.environ.get("HFX_SPLITS", "").split(",")):
    _k, _v = _kv.split(":")
    DEFAULT_SPLITS[tuple(int(c) for c in _k)] = int(_v)

# FP32 slices: the same as FP64.  FP32 halves the contracted array but not
# the rest of a slice's live values (its FP64 large-argument Boys branch, FP64
# digestion, addresses), and with fewer slices the FP32 kernels spilled
# 1.6-3.4 KB per lane (compiler resource reports); unpacked FP32 arithmetic
# runs at the FP64 rate on this chip, so FP32 gains no issue rate either.
DEFAULT_SPLITS_F32 = dict(DEFAULT_SPLITS)
for _kv in filter(None, os.environ.get("HFX_SPLITS_F32", "").split(",")):
    _k, _v = _kv.split(":")
    DEFAULT_SPLITS_F32[tuple(int(c) for c in _k)] = int(_v)

# Waves per workgroup of the FP64 quartet kernel, per class (classes not
# listed: 1; tuning: HFX_WPB="1000:4").  Four-wave workgroups for the nine
# lightest classes, which hold about four waves per SIMD where their
# registers would allow eight, made them 2-28 % slower.
WPB = {}
for _kv in filter(None, os.environ.get("HFX_WPB", "").split(",")):
    _k, _v = _kv.split(":")
    WPB[tuple(int(c) for c in _k)] = int(_v)

# Minimum waves per SIMD asked of the register allocator, per class (classes
# not listed: 1).  (ds|ds) gains from two waves; the other mid classes lose.
WAVES = {(2, 0, 2, 0): 2}
for _kv in filter(None, os.environ.get("HFX_WAVES", "").split(",")):
    _k, _v = _kv.split(":")
    WAVES[tuple(int(c) for c in _k)] = int(_v)


def write_jk_tu(outdir, tag, suffix, nm, kernel, launcher, swap="false"):
    """A translation unit of its own for the kernel that also digests the
    Coulomb matrix (kept apart so the exchange-only kernel is unchanged)."""
    tu = [
        "// Generated by gen_eri.py; do not edit.",
        '#include "hfx_device.hpp"',
        f'#include "eri_{tag}{suffix}.h"',
        "namespace hfx {",
        f"void {launcher}_{tag}(const QuartetArgs &a0, unsigned nblk, hipStream_t s) {{",
        f"  launch_segments(a0, (long long)nblk * {nm}::NSPLIT, 8ll * {nm}::XCH,  // 8 XCDs x chunk",
        "                  [&](const QuartetArgs &a, unsigned grid) {",
        f"                    hipLaunchKernelGGL(HIP_KERNEL_NAME({kernel}<{nm}, true{', true' if swap == 'true' else ''}>), dim3(grid), dim3(64 * {nm}::WPB), 0, s, a);",
        f"                  }}, {nm}::WPB);",
        "}",
        "}  // namespace hfx",
    ]
    write_if_changed(os.path.join(outdir, f"tu_{tag}{suffix}_jk.hip"), "\n".join(tu) + "\n")


def write_per_tu(outdir, tag, nm, la, lb, lc, ld):
    """Periodic builds: the canonical class kernel with the wave's pair as the
    recurrence's bra (its class the higher one), and -- for classes of two
    different pair classes -- with the lane's pair as the bra (the wave's
    pair of the lower class)."""
    lines = [
        "// Generated by gen_eri.py; do not edit.",
        '#include "hfx_device.hpp"',
        f'#include "eri_{tag}.h"',
        "namespace hfx {",
        f"void launch_eriper_{tag}(const QuartetArgs &a0, unsigned nblk, hipStream_t s) {{",
        f"  launch_segments(a0, (long long)nblk * {nm}::NSPLIT, 8ll * {nm}::XCH,",
        "                  [&](const QuartetArgs &a, unsigned grid) {",
        f"                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri<{nm}, false, false, true>), dim3(grid), dim3(64 * {nm}::WPB), 0, s, a);",
        f"                  }}, {nm}::WPB);",
        "}",
    ]
    if (la, lb) != (lc, ld):
        lines += [
            f"void launch_eriperS_{tag}(const QuartetArgs &a0, unsigned nblk, hipStream_t s) {{",
            f"  launch_segments(a0, (long long)nblk * {nm}::NSPLIT, 8ll * {nm}::XCH,",
            "                  [&](const QuartetArgs &a, unsigned grid) {",
            f"                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri<{nm}, false, true, true>), dim3(grid), dim3(64 * {nm}::WPB), 0, s, a);",
            f"                  }}, {nm}::WPB);",
            "}",
        ]
    else:
        lines += [f"void launch_eriperS_{tag}(const QuartetArgs &, unsigned, hipStream_t) {{}}"]
    lines.append("}  // namespace hfx")
    write_if_changed(os.path.join(outdir, f"tu_{tag}_per.hip"), "\n".join(lines) + "\n")


# Classes evaluated with the roles of the pairs exchanged, (cd|ab) in place of
# (ab|cd), so that the slices split the components of the original bra pair
# (for these classes the recurrence shared between slices is smaller that way),
# with the slice counts of the exchanged class.  The digestion images are then
# the transposes of the usual ones, which K = K' + K'^T absorbs.  FP64 direct
# and persistent launches.  Measured on the 256-atom shard against the
# unexchanged class: (dp|pp) -8 %, (dd|pp) -7 %, (dd|ds) -4 %; then, with the
# slice counts re-measured: (dp|pp) in 1 slice instead of 2 -16 %, (dd|pp) in
# 2 instead of 3 -12 %, (ds|pp) -9 % and (dd|ps) -6 % exchanged; (dd|dp),
# (dp|ds) and (dp|ps) exchanged are 2-13 % slower and stay as they are.
# HFX_TRANSPOSED="2111:2,2211:3" overrides (tuning); "none" turns it off.
TRANSPOSED = {(2, 1, 1, 1): 1, (2, 2, 1, 1): 2, (2, 2, 2, 0): 2, (2, 2, 1, 0): 1, (2, 0, 1, 1): 1}
_tr = os.environ.get("HFX_TRANSPOSED", "")
if _tr == "none":
    TRANSPOSED = {}
if _tr != "none":
    for _kv in filter(None, _tr.split(",")):
        _k, _v = _kv.split(":")
        TRANSPOSED[tuple(int(c) for c in _k)] = int(_v)


def class_tag(c):
    return "".join(str(x) for x in c)


def write_if_changed(path, text):
    """Write only when the content differs, so unchanged outputs keep their
    time stamps (incremental builds recompile only what changed)."""
    try:
        with open(path) as f:
            if f.read() == text:
                return
    except OSError:
        pass
    with open(path, "w") as f:
        f.write(text)


def emit_struct(em, la, lb, lc, ld, nm, G):
    """One class struct: the unsplit recurrence, the G ket-component slices
    (recurrence, exchange and Coulomb digestion, Schwarz diagonal of diagonal
    classes) and the unsplit post-processing.  Returns the model figures."""
    E, F = la + lb, lc + ld
    NE = sum(ncart(d) for d in range(la, E + 1))
    NF = sum(ncart(d) for d in range(lc, F + 1))
    em.lines.append(f"struct {nm} {{")
    em.lines.append(f"  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld}, L = {E + F};")
    em.lines.append(f"  static constexpr int NE = {NE}, NF = {NF}, NACC = {NE * NF};")
    nsph = (2 * la + 1) * (2 * lb + 1) * (2 * lc + 1) * (2 * ld + 1)
    em.lines.append(f"  static constexpr int NOUT = {nsph};")
    _, vflops = emit_vrr(em, la, lb, lc, ld, "vrr")
    G = min(G, NF)  # no empty slices
    em.lines.append(f"  static constexpr int NSPLIT = {G};")
    # keyed by the class as listed, so an exchanged struct takes its class's value
    em.lines.append(f"  static constexpr int WAVES = {WAVES.get((la, lb, lc, ld), WAVES.get((lc, ld, la, lb), 1))};")
    # waves (independent logical blocks) per workgroup of the FP64 quartet
    # kernel, and the XCD chunk in workgroups (8 tiles' slices)
    wpb = WPB.get((la, lb, lc, ld), WPB.get((lc, ld, la, lb), 1)) if em.T == "double" else 1
    em.lines.append(f"  static constexpr int WPB = {wpb};")
    em.lines.append(f"  static constexpr int XCH = {(8 * G + wpb - 1) // wpb};")
    split_cost = []
    groups = best_split(la, lb, lc, ld, G) if G > 1 else [[f for d in range(lc, F + 1) for f in cart(d)]]
    nacc_p = []
    for g, ft in enumerate(groups):
        n_, c = emit_vrr(em, la, lb, lc, ld, f"vrr_p{g}", f_targets=ft)
        nacc_p.append(n_)
        split_cost.append(c)
        emit_digest_part(em, la, lb, lc, ld, f"dig_p{g}", ft)
        emit_digest_part(em, la, lb, lc, ld, f"digJ_p{g}", ft, mode="J")
        if em.T == "double":
            emit_digest_part(em, la, lb, lc, ld, f"store_p{g}", ft, mode="E")
            emit_digest_part(em, la, lb, lc, ld, f"digR_p{g}", ft, mode="R")
        if (la, lb) == (lc, ld):
            emit_digest_part(em, la, lb, lc, ld, f"diag_p{g}", ft, mode="D")
            # largest diagonal value [e0|e0] of the contracted array (bra and
            # ket are the same pair): the scale of the horizontal
            # recurrence's inputs
            e_all = [e for d in range(la, la + lb + 1) for e in cart(d)]
            ei = {e: k for k, e in enumerate(e_all)}
            fi = {f: k for k, f in enumerate(ft)}
            em.lines.append(f"  __device__ __forceinline__ static void diagE_p{g}(const {em.T}* __restrict__ acc, "
                            "double* __restrict__ m) {")
            for f in ft:
                em.lines.append(f"    m[0] = fmax(m[0], (double)acc[{ei[f] * len(ft) + fi[f]}]);")
            em.lines.append("  }")
    em.lines.append(f"  static constexpr int NACCP[{G}] = {{{', '.join(str(x) for x in nacc_p)}}};")
    T_ = em.T
    em.lines.append("  template <int W> __device__ __forceinline__ static void vrr_p(const %s* __restrict__ g," % T_)
    em.lines.append("      %s PAx, %s PAy, %s PAz, %s WPx, %s WPy, %s WPz," % ((T_,) * 6))
    em.lines.append("      %s QCx, %s QCy, %s QCz, %s WQx, %s WQy, %s WQz," % ((T_,) * 6))
    em.lines.append("      %s i2z, %s roz, %s i2e, %s roe, %s i2ze, %s* __restrict__ acc) {" % ((T_,) * 6))
    for g_ in range(G):
        kw = "if" if g_ == 0 else "else if"
        em.lines.append(f"    {kw} constexpr (W == {g_}) vrr_p{g_}(g, PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz,"
                        " WQx, WQy, WQz, i2z, roz, i2e, roe, i2ze, acc);")
    em.lines.append("  }")
    em.lines.append("  template <int W> __device__ __forceinline__ static void dig(const %s* __restrict__ acc," % T_)
    em.lines.append("      double ABx, double ABy, double ABz, double CDx, double CDy, double CDz, int a0, int b0, int c0, int d0,")
    em.lines.append("      double deg, const double* __restrict__ P, double* K, int64_t ld) {")
    for g_ in range(G):
        kw = "if" if g_ == 0 else "else if"
        em.lines.append(f"    {kw} constexpr (W == {g_}) dig_p{g_}(acc, ABx, ABy, ABz, CDx, CDy, CDz, a0, b0, c0, d0,"
                        " deg, P, K, ld);")
    em.lines.append("  }")
    if (la, lb) == (lc, ld):
        # share of slice W in the diagonal values (ab|ab), for the Schwarz factors
        em.lines.append("  template <int W> __device__ __forceinline__ static void diag(const %s* __restrict__ acc," % T_)
        em.lines.append("      double ABx, double ABy, double ABz, double* __restrict__ d) {")
        for g_ in range(G):
            kw = "if" if g_ == 0 else "else if"
            em.lines.append(f"    {kw} constexpr (W == {g_}) diag_p{g_}(acc, ABx, ABy, ABz, ABx, ABy, ABz, 0, 0, 0, 0,"
                            " 1.0, nullptr, d, 0);")
        em.lines.append("  }")
        em.lines.append("  template <int W> __device__ __forceinline__ static void diagE(const %s* __restrict__ acc,"
                        " double* __restrict__ m) {" % T_)
        for g_ in range(G):
            kw = "if" if g_ == 0 else "else if"
            em.lines.append(f"    {kw} constexpr (W == {g_}) diagE_p{g_}(acc, m);")
        em.lines.append("  }")
    if T_ == "double":
        # exchange rows chosen per call (periodic builds)
        em.lines.append("  template <int W> __device__ __forceinline__ static void digR(const %s* __restrict__ acc," % T_)
        em.lines.append("      double ABx, double ABy, double ABz, double CDx, double CDy, double CDz, int a0, int b0, int c0, int d0,")
        em.lines.append("      double wA, double wB, double wC, double wD, const double* __restrict__ P, int64_t ldP, double* K,")
        em.lines.append("      int64_t ldK) {")
        for g_ in range(G):
            kw = "if" if g_ == 0 else "else if"
            em.lines.append(f"    {kw} constexpr (W == {g_}) digR_p{g_}(acc, ABx, ABy, ABz, CDx, CDy, CDz, a0, b0, c0, d0, wA,"
                            " wB, wC, wD, P, ldP, K, ldK);")
        em.lines.append("  }")
        # this slice's share of the raw spherical values (hfx_eval_quartets)
        em.lines.append("  template <int W> __device__ __forceinline__ static void store(const %s* __restrict__ acc," % T_)
        em.lines.append("      double ABx, double ABy, double ABz, double CDx, double CDy, double CDz, int64_t sab,")
        em.lines.append("      int64_t scd, double* __restrict__ out) {")
        for g_ in range(G):
            kw = "if" if g_ == 0 else "else if"
            em.lines.append(f"    {kw} constexpr (W == {g_}) store_p{g_}(acc, ABx, ABy, ABz, CDx, CDy, CDz, sab, scd, out);")
        em.lines.append("  }")
    em.lines.append("  template <int W> __device__ __forceinline__ static void digJ(const %s* __restrict__ acc," % T_)
    em.lines.append("      double ABx, double ABy, double ABz, double CDx, double CDy, double CDz, int a0, int b0, int c0, int d0,")
    em.lines.append("      double deg, const double* __restrict__ P, double* J, int64_t ld) {")
    for g_ in range(G):
        kw = "if" if g_ == 0 else "else if"
        em.lines.append(f"    {kw} constexpr (W == {g_}) digJ_p{g_}(acc, ABx, ABy, ABz, CDx, CDy, CDz, a0, b0, c0, d0,"
                        " deg, P, J, ld);")
    em.lines.append("  }")
    pflops = emit_post(em, la, lb, lc, ld)
    em.lines.append("};")
    return vflops, pflops, NE, NF, nsph, G, split_cost


def generate(outdir, T="double", splits=None):
    """Write one header and one translation unit per class into outdir and
    return the operation-count model."""
    if splits is None:
        splits = DEFAULT_SPLITS if T == "double" else DEFAULT_SPLITS_F32
    os.makedirs(outdir, exist_ok=True)
    suffix = "" if T == "double" else "_f32"
    model = {}
    for (la, lb, lc, ld) in classes():
        em = Emitter(T)
        tag = class_tag((la, lb, lc, ld))
        em.lines.append("// Generated by gen_eri.py; do not edit.")
        em.lines.append("#pragma once")
        E, F = la + lb, lc + ld
        NE = sum(ncart(d) for d in range(la, E + 1))
        NF = sum(ncart(d) for d in range(lc, F + 1))
        nm = f"Eri{tag}{suffix}"
        vflops, pflops, NE, NF, nsph, G, split_cost = emit_struct(
            em, la, lb, lc, ld, nm, splits.get((la, lb, lc, ld), 1))
        if (la, lb, lc, ld) in TRANSPOSED:
            # the same integrals with the pairs' roles exchanged, sliced over
            # the components of the original bra pair (see TRANSPOSED)
            tinfo = emit_struct(em, lc, ld, la, lb, nm + "T", TRANSPOSED[(la, lb, lc, ld)])
        else:
            tinfo = None
        write_if_changed(os.path.join(outdir, f"eri_{tag}{suffix}.h"), "\n".join(em.lines) + "\n")
        model[tag] = dict(vrr_flops=vflops, post_flops=pflops, nacc=NE * NF,
                          nout=nsph, split=G, split_vrr_flops=split_cost)
        if tinfo is not None:  # the kernel that runs: the exchanged struct
            model[tag].update(split_exchanged=tinfo[5], split_vrr_flops_exchanged=tinfo[6])
        diag = (la, lb) == (lc, ld)
        # launches of a class in TRANSPOSED use the exchanged struct
        tr = (la, lb, lc, ld) in TRANSPOSED
        dn, sw = (nm + "T", "true") if tr else (nm, "false")
        if T != "double":
            tu = [
                "// Generated by gen_eri.py; do not edit.",
                '#include "hfx_device.hpp"',
                f'#include "eri_{tag}{suffix}.h"',
                "namespace hfx {",
                f"void launch_eri32_{tag}(const QuartetArgs &a0, unsigned nblk, hipStream_t s) {{",
                f"  launch_segments(a0, (long long)nblk * {dn}::NSPLIT, 64ll * {dn}::NSPLIT,  // 8 XCDs x chunk",
                "                  [&](const QuartetArgs &a, unsigned grid) {",
                f"                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri32<{dn}, false, {sw}>), dim3(grid), dim3(64), 0, s, a);",
                "                  });",
                "}",
                f"void launch_persist32_{tag}(const BatchJob *j, int nj, long long vt, unsigned long long *h, int claim,",
                "                          unsigned grid, hipStream_t s) {",
                f"  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri32_persist<{dn}, {sw}>), dim3(grid), dim3(64), 0, s, j, nj, vt, h, claim);",
                "}",
                f"int nsplit32_{tag}() {{ return {dn}::NSPLIT; }}",
            ]
            tu.append("}  // namespace hfx")
            write_if_changed(os.path.join(outdir, f"tu_{tag}{suffix}.hip"), "\n".join(tu) + "\n")
            write_jk_tu(outdir, tag, suffix, dn, "k_eri32", "launch_erijk32", sw)
            continue
        tu = [
            "// Generated by gen_eri.py; do not edit.",
            '#include "hfx_device.hpp"',
            f'#include "eri_{tag}{suffix}.h"',
            "namespace hfx {",
            f"void launch_eri_{tag}(const QuartetArgs &a0, unsigned nblk, hipStream_t s) {{",
            f"  launch_segments(a0, (long long)nblk * {dn}::NSPLIT, 8ll * {dn}::XCH,  // 8 XCDs x chunk",
            "                  [&](const QuartetArgs &a, unsigned grid) {",
            f"                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri<{dn}, false, {sw}>), dim3(grid), dim3(64 * {dn}::WPB), 0, s, a);",
            f"                  }}, {dn}::WPB);",
            "}",
            f"void launch_persist_{tag}(const BatchJob *j, int nj, long long vt, unsigned long long *h, int claim,",
            "                        unsigned grid, hipStream_t s) {",
            f"  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eri_persist<{dn}, {sw}>), dim3(grid), dim3(64), 0, s, j, nj, vt, h, claim);",
            "}",
            f"int nsplit_{tag}() {{ return {dn}::NSPLIT; }}",
            f"void launch_eval_{tag}(const PairHdr *h, const PrimRec *p, const int32_t *bk, int n, int op,",
            "                    double om2, const double *tab, double *out, hipStream_t s) {",
            f"  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eval<{dn}, {sw}>), dim3((n + 63) / 64), dim3(64), 0, s, h, p, bk, n, op,",
            "                     om2, tab, out);",
            "}",
        ]
        if diag:
            tu += [
                f"void launch_schwarz_{class_tag((la, lb))}(const PairHdr *h, const PrimRec *p, const int32_t *ids, int n,",
                "                    int op, double om2, const double *tab, double *Q, double *E, hipStream_t s) {",
                f"  hipLaunchKernelGGL(k_schwarz<{nm}>, dim3((n + 63) / 64), dim3(64), 0, s, h, p, ids, n, op, om2, tab, Q, E);",
                "}",
                f"void launch_primbound_{class_tag((la, lb))}(const PairHdr *h, PrimRec *p, const int32_t *ids, int n,",
                "                    int op, double om2, const double *tab, hipStream_t s) {",
                f"  hipLaunchKernelGGL(k_primbound<{nm}>, dim3((n + 63) / 64), dim3(64), 0, s, h, p, ids, n, op, om2, tab);",
                "}",
            ]
        tu.append("}  // namespace hfx")
        write_if_changed(os.path.join(outdir, f"tu_{tag}{suffix}.hip"), "\n".join(tu) + "\n")
        write_jk_tu(outdir, tag, suffix, dn, "k_eri", "launch_erijk", sw)
        write_per_tu(outdir, tag, nm, la, lb, lc, ld)
    return model


def write_model(outdir, model):
    """FLOP model table (per primitive quartet: the vertical recurrence; per
    contracted quartet: horizontal recurrence, spherical transform and the
    four digestion contractions)."""
    tags = [class_tag(c) for c in classes()]
    vr = ", ".join(f"{model[t]['vrr_flops']}.0" for t in tags)
    po = ", ".join(f"{model[t]['post_flops'] + 8 * model[t]['nout'] + 4}.0" for t in tags)
    src = [
        "// Generated by gen_eri.py; do not edit.",
        "namespace hfx {",
        f"static const double k_model_vrr[21] = {{{vr}}};",
        f"static const double k_model_post[21] = {{{po}}};",
        "const double *model_vrr() { return k_model_vrr; }",
        "const double *model_post() { return k_model_post; }",
        "// Arithmetic of one primitive quartet outside the recurrence: geometry",
        "// (24), Boys Taylor + recursion (15 + 3L per evaluation), prefactor",
        "// scaling, and for the attenuated kernel the second Boys evaluation and",
        "// the theta powers.",
        "double model_prim_overhead(int op, int L) {",
        "  return 24.0 + (op ? 2 : 1) * (15.0 + 3.0 * L) + (op ? 3 : 1) * (L + 1.0) + (op ? 4.0 : 0.0);",
        "}",
        "}  // namespace hfx",
    ]
    write_if_changed(os.path.join(outdir, "model.hip"), "\n".join(src) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--outdir", required=True)
    ap.add_argument("--type", default="double")
    ap.add_argument("--model", default=None)
    a = ap.parse_args()
    model = generate(a.outdir, "double")
    generate(a.outdir, "float")
    write_model(a.outdir, model)
    if a.model:
        with open(a.model, "w") as f:
            json.dump(model, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
