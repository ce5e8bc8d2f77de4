#!/usr/bin/env python3
"""Benchmark of the screened exchange build on one MI355X.

Workload: the 256-atom DZP-like lattice system (1280 shells, 3328 spherical
functions; erfc(omega r)/r with omega = 0.11; Schwarz tau = 1e-10; plain
FP64).  A full K-build of it is ~10^13 primitive quartets -- far more than a
one-minute timed region -- so one step is one GPU's share of that build when
it is distributed over `--shards` devices (bra pairs of every class dealt
round-robin, `hfx_build_K_shard`): the kernels run at the workload's real
shape and class mix, and `projected_full_build_s` states shards x step time.

A step = one pass of the whole path on that share: the P symmetry check, the
Schwarz bounds and screening lists (cached in the pair handle after the first
call, as across SCF iterations), all 21 class kernels and the
symmetrisation.  Pair data and P are resident in HBM before timing starts.

Output: one JSON line (rank 0) with the metric, a roofline object for the
dominant class kernel (device time from HIP events on the launch stream) and
the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shards", type=int, default=64,
                    help="the step is one of this many bra-pair shards of the full build")
    ap.add_argument("--shard", type=int, default=0)
    ap.add_argument("--natom", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle timing leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--mixed-cut", type=float, default=1e-5, help="FP32 cut on the error scale E_IJ E_KL")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch leg")
    ap.add_argument("--no-jk", action="store_true", help="skip the Coulomb + exchange leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served leg")
    ap.add_argument("--no-density", action="store_true", help="skip the density-screened leg")
    ap.add_argument("--no-periodic", action="store_true", help="skip the periodic leg")
    ap.add_argument("--batch-natom", type=str, default="6,20",
                    help="atom-count range of the batched systems (scaled-down uneven-batch recipe)")
    ap.add_argument("--serve-natom", type=str, default="6,24",
                    help="atom-count range of served requests (scaled-down serving recipe)")
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--no-latency", action="store_true", help="skip the full K-build latency leg")
    ap.add_argument("--latency-natom", type=int, default=64,
                    help="atoms of the lattice (256-atom workload recipe) built whole in the latency leg")
    ap.add_argument("--latency-builds", type=int, default=10)
    ap.add_argument("--dzp1024", action="store_true",
                    help="only the 1024-atom mixed-precision workload: full K of the 128-atom subset in FP64 and "
                         "mixed, and one shard of the 1024-atom build")
    ap.add_argument("--dzp1024-shards", type=int, default=2048)
    ap.add_argument("--serve-mix", type=int, default=0, metavar="N",
                    help="only run a served mix of 16 small requests x 3 builds with N builds in flight "
                         "(for kernel traces)")
    ap.add_argument("--kernel-overlap", type=str, default=None, metavar="DIR",
                    help="only summarise a rocprofv3 kernel trace under DIR: time with quartet kernels of two "
                         "or more queues running at once")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 512 MiB device copy five times (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(sysm, tau, omega, budget_s):
    """The oracle on a seeded sample of screened quartets of the same
    workload, on all host cores: a random pool of shell pairs, their Schwarz
    factors from the oracle itself, every unique quartet of the pool that
    passes Q_IJ Q_KL >= tau, shuffled; the sample size is calibrated to the
    time budget."""
    import oracle

    rng = np.random.default_rng(12345)
    npair = sysm.nshell * (sysm.nshell + 1) // 2
    cores = len(os.sched_getaffinity(0))
    pool = np.unique(rng.integers(0, npair, size=min(npair, 2400)))
    qpool = oracle.schwarz_list(sysm, pool, omega=omega)
    ii, jj = np.tril_indices(len(pool))
    keep = qpool[ii] * qpool[jj] >= tau
    cand = np.stack([pool[ii[keep]], pool[jj[keep]]], axis=1)
    rng.shuffle(cand)
    # calibrate on growing samples until one takes 0.5 s, then time a sample
    # sized to the whole budget
    n = 512
    while True:
        t0 = time.perf_counter()
        oracle.digest_list(sysm, cand[:n], omega=omega, nthreads=cores)
        dt = time.perf_counter() - t0
        if dt >= 0.5 or n >= len(cand):
            break
        n = min(len(cand), n * 4)
    # three timed repeats share the budget; the median is reported
    n = min(len(cand), max(n, int(n * budget_s / 3 / max(dt, 1e-3))))
    reps = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.digest_list(sysm, cand[:n], omega=omega, nthreads=cores)
        reps.append(time.perf_counter() - t0)
    dt = float(np.median(reps))
    desc = (f"{n} screened unique shell quartets (Q_IJ Q_KL >= tau by the oracle's own Schwarz factors) "
            f"among a seeded random pool of {len(pool)} shell pairs of the same system; FP64 integrals and "
            f"digestion into K; median of 3 timings ({', '.join(f'{r:.2f}' for r in reps)} s)")
    return {"value": n / dt, "unit": "quartets/s", "cores": cores, "kind": "oracle", "sample": desc,
            "repeats_s": reps}


def batch_leg(a, hfx, hi, torch):
    """64 independent systems (uneven-batch recipe: uniform atom counts, l_max in
    {1, 2}, lattice shells and P) in one persistent launch per class through
    the device work queue, FP64 and mixed, against building them one by one."""
    lo, hi_ = (int(x) for x in a.batch_natom.split(","))
    systems = hi.uneven_batch(seed=3, nsys=64, natom_range=(lo, hi_))
    tau, omega = 1e-10, hi.OMEGA_HSE
    res = {"workload": f"64 systems, atoms uniform in [{lo},{hi_}] (uneven-batch recipe scaled down from [20,400]), "
                       f"l_max in {{1,2}}, erfc omega={omega}, tau={tau}"}
    for name, prec in (("fp64", hfx.PREC_FP64), ("mixed", hfx.PREC_MIXED)):
        o = hfx.opts(tau=tau, omega=omega, prec=prec, mixed_cut=a.mixed_cut)
        pairs = [hfx.pairs_from_system(s, o) for s in systems]
        Ps = [torch.from_numpy(s.P).cuda() for s in systems]
        Ks = [torch.empty_like(P) for P in Ps]
        # default launch parameters, no autotuning (bounds and lists built on the
        # first of the two calls)
        os.environ["HFX_TUNE"] = "0"
        for _ in range(2):
            t0 = time.perf_counter()
            hfx.build_K_batch(pairs, Ps, Ks, o)
            torch.cuda.synchronize()
            t_default = time.perf_counter() - t0
            print(f"# batch {name}: default parameters {t_default:.3f} s", file=sys.stderr, flush=True)
        del os.environ["HFX_TUNE"]
        t0 = time.perf_counter()
        hfx.build_K_batch(pairs, Ps, Ks, o)  # first tuned call: autotuning
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        print(f"# batch {name}: first tuned call {t_first:.3f} s", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        st = hfx.build_K_batch(pairs, Ps, Ks, o, stats=True)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        Kb = [K.cpu().numpy() for K in Ks]
        # the same systems one call at a time (lists already resident)
        t0 = time.perf_counter()
        for i, (p, P, K) in enumerate(zip(pairs, Ps, Ks)):
            hfx.build_K(p, P, K, o)
            if i % 16 == 15:
                torch.cuda.synchronize()
                print(f"# batch {name}: {i + 1} systems one by one", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        dmax = max(float(np.abs(K.cpu().numpy() - k).max()) for K, k in zip(Ks, Kb))
        res[name] = {"value": st["quartets"] / tb, "unit": "quartets/s", "batch_s": tb,
                     "sequential_s": ts, "speedup_vs_sequential": ts / tb, "first_call_s": t_first,
                     "default_params_s": t_default, "tuning_speedup": t_default / tb,
                     "quartets": st["quartets"], "max_abs_dK_batch_vs_solo": dmax}
        print(f"# batch {name}: {tb:.3f} s vs sequential {ts:.3f} s", file=sys.stderr, flush=True)
    return res


def serve_leg(a, hfx, hi, torch):
    """Served K-builds (serving recipe scaled down): requests with log-uniform
    atom counts, each 10 SCF-like iterations with P perturbed by 1e-3 relative
    noise, Poisson arrivals at 70 % of the measured closed-loop capacity,
    mixed precision, pair data resident, admission by an HBM budget."""
    lo, hi_ = (int(x) for x in a.serve_natom.split(","))
    reqs = hi.served_requests(seed=4, nreq=a.serve_requests, natom_range=(lo, hi_), iters=10)
    tau, omega = 1e-10, hi.OMEGA_HSE
    o = hfx.opts(tau=tau, omega=omega, prec=hfx.PREC_MIXED, mixed_cut=a.mixed_cut)
    systems = [hi.lattice_system(r["natom"], seed=r["seed"], name=f"served{r['id']}") for r in reqs]
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    Ks = [torch.empty_like(P) for P in Ps]
    budget = int(32 * 2**30)
    srv = None
    rng = np.random.default_rng(44)

    def run(arrivals):
        """arrivals[i] = release time of request i (s); each request runs its
        iterations back to back; returns per-build and per-request latencies."""
        t_start = time.perf_counter()
        state = [{"it": 0, "ticket": None, "t_req": None} for _ in reqs]
        build_lat, req_lat, quartets = [], [], 0
        left = len(reqs)
        while left:
            now = time.perf_counter() - t_start
            for i, stt in enumerate(state):
                if stt["it"] >= reqs[i]["iters"]:
                    continue
                if stt["ticket"] is None and now >= arrivals[i]:
                    if stt["t_req"] is None:
                        stt["t_req"] = time.perf_counter()
                    Pn = hi.perturbed_density(systems[i].P, rng)
                    Ps[i].copy_(torch.from_numpy(Pn))
                    torch.cuda.synchronize()
                    stt["ticket"] = srv.submit(pairs[i], Ps[i], Ks[i], o)
                elif stt["ticket"] is not None:
                    done, st = srv.poll(stt["ticket"])
                    if done:
                        build_lat.append(st["latency_s"])
                        quartets += st["quartets"]
                        stt["ticket"] = None
                        stt["it"] += 1
                        if stt["it"] == reqs[i]["iters"]:
                            req_lat.append(time.perf_counter() - stt["t_req"])
                            left -= 1
            time.sleep(0.0005)
        return time.perf_counter() - t_start, build_lat, req_lat, quartets

    # capacity: closed loop, everything released at t = 0; first with one
    # build in flight (no overlap), then with four (builds of different
    # requests overlap on the device)
    srv = hfx.Server(budget, max_inflight=1)
    wall1, _, _, nq1 = run([0.0] * len(reqs))
    del srv
    srv = hfx.Server(budget, max_inflight=4)
    wall, bl, rl, nq = run([0.0] * len(reqs))
    cap = len(reqs) / wall  # requests/s
    lam = 0.7 * cap
    arr = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
    arr -= arr[0]
    wall2, bl2, rl2, nq2 = run(list(arr))
    pct = lambda v, q: float(np.percentile(v, q))
    return {
        "workload": f"{len(reqs)} requests, atoms log-uniform in [{lo},{hi_}] (serving recipe scaled down from "
                    f"[50,2000]), 10 iterations each, P x (1 + 1e-3 E_t), mixed cut {a.mixed_cut}, "
                    f"HBM budget {budget >> 30} GiB, 4 in flight",
        "capacity_req_per_s": cap,
        "capacity_req_per_s_one_in_flight": len(reqs) / wall1,
        "closed_loop_speedup_4_vs_1_in_flight": wall1 / wall,
        "lambda_req_per_s": lam,
        "value": nq2 / wall2,
        "unit": "quartets/s",
        "build_p50_ms": 1e3 * pct(bl2, 50),
        "build_p99_ms": 1e3 * pct(bl2, 99),
        "request_p50_s": pct(rl2, 50),
        "request_p99_s": pct(rl2, 99),
        "closed_loop_quartets_per_s": nq / wall,
    }


def periodic_leg(a, hfx, hi, torch):
    """Periodic exchange of a crystal: 2 atoms per 5.5-bohr cubic cell, DZP-like
    shells (3-6 primitives, exponents in [0.1, 10]: the paper keeps fitted
    exponents above 0.1 for solids), 27 image cells (cells -1..1 per axis);
    K^G for the home cell's rows, lattice sums over the cluster, FP64, erfc."""
    cl = hi.periodic_cluster(natom_cell=2, cell_len=5.5, reach=(1, 1, 1), lmax=2, nprim_range=(3, 6),
                             alpha_range=(0.1, 10.0), seed=11)
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    p = hfx.pairs_from_system(cl, o)
    nhs = int(cl.meta["nhome_shell"])
    nh = int(np.sum(2 * cl.shell_l[:nhs] + 1))
    P = torch.from_numpy(cl.P).cuda()
    K = torch.empty((nh, cl.nbf), dtype=torch.float64, device="cuda")
    hfx.build_K_periodic(p, nhs, P, K, o)  # bounds and lists
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = hfx.build_K_periodic(p, nhs, P, K, o, stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# periodic leg: {dt:.3f} s", file=sys.stderr, flush=True)
    return {"workload": f"crystal of 2 atoms per 5.5-bohr cell, {cl.meta['ncell']} image cells ({cl.natom} atoms, "
                        f"{cl.nshell} shells, {cl.nbf} functions), home-cell rows of K^G, erfc omega={hi.OMEGA_HSE}, "
                        f"tau=1e-10, FP64",
            "value": st["quartets"] / dt, "unit": "quartets/s", "build_s": dt, "quartets": st["quartets"],
            "gflops": st["flops"] / st["device_s"] / 1e9}


def latency_leg(a, hfx, hi, torch):
    """Whole K-builds of one system of the benchmark recipe (FP64, erfc,
    tau = 1e-10), one after another on one stream with the inputs resident:
    per-build wall time from the call to the end of its stream work (the P
    check, the class kernels and the symmetrisation; bounds and lists are
    resident after the warm-up build, as across SCF iterations)."""
    s = hi.lattice_system(a.latency_natom, seed=1, name=f"lattice_dzp{a.latency_natom}")
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    hfx.build_K(pairs, P, K, o)
    torch.cuda.synchronize()
    lat, st = [], None
    for i in range(a.latency_builds):
        t0 = time.perf_counter()
        st = hfx.build_K(pairs, P, K, o)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    st = hfx.build_K(pairs, P, K, o, stats=True)
    torch.cuda.synchronize()
    print(f"# latency leg: {a.latency_builds} full builds of {a.latency_natom} atoms, "
          f"p50 {np.percentile(lat, 50):.3f} s", file=sys.stderr, flush=True)
    return {"workload": f"whole K-builds of a {s.natom}-atom lattice of the benchmark recipe ({s.nshell} shells, "
                        f"{s.nbf} functions, erfc omega={hi.OMEGA_HSE}, tau=1e-10, FP64)",
            "builds": a.latency_builds, "build_p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "build_p99_ms": 1e3 * float(np.percentile(lat, 99)), "quartets_per_build": st["quartets"],
            "quartets_per_s": st["quartets"] / float(np.median(lat))}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dominant_kernel.json")


def source_hash():
    """Hash of the sources the quartet kernels are generated and compiled from;
    stored HBM-traffic counters apply only while it is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in ("hfx_device.hpp", "gen_eri.py"):
        with open(os.path.join(ROOT, "paper_2009_03559_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_tag, shards):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None
    if the kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash() or t.get("kernel_tag") != kernel_tag or t.get("shards") != shards:
        return None
    return t.get("hbm_bytes_per_launch")


def serve_mix(n_inflight):
    """Served mix for kernel traces: 16 requests of 4-10 atoms (the
    lattice workload's shells), 3 SCF-like builds each, all released at once; bounds and lists
    resident before the mix starts."""
    import torch

    import hfx_inputs as hi
    import paper_2009_03559_amd as hfx

    torch.cuda.init()
    rng = np.random.default_rng(5)
    systems = [hi.lattice_system(int(n), seed=100 + i) for i, n in enumerate(rng.integers(4, 11, size=16))]
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    Ks = [torch.empty_like(P) for P in Ps]
    for p, P, K in zip(pairs, Ps, Ks):
        hfx.build_K(p, P, K, o)
    torch.cuda.synchronize()
    srv = hfx.Server(1 << 34, max_inflight=n_inflight)
    t0 = time.perf_counter()
    left = {i: 3 for i in range(len(systems))}
    ticket = {i: srv.submit(pairs[i], Ps[i], Ks[i], o) for i in left}
    while ticket:
        for i in list(ticket):
            done, _ = srv.poll(ticket[i])
            if done:
                left[i] -= 1
                if left[i]:
                    ticket[i] = srv.submit(pairs[i], Ps[i], Ks[i], o)
                else:
                    del ticket[i]
        time.sleep(0.0005)
    print(json.dumps({"served_mix": f"{len(systems)} requests x 3 builds", "in_flight": n_inflight,
                      "wall_s": time.perf_counter() - t0}), flush=True)


def kernel_overlap(d):
    """Quartet-kernel dispatches of a rocprofv3 kernel trace (CSV under d):
    busy time (any running) and time with kernels of two or more queues
    running at once."""
    import csv
    import glob

    f = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    ev = []
    with open(f) as fh:
        for r in csv.DictReader(fh):
            if "k_eri" in r.get("Kernel_Name", ""):
                ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Queue_Id", "0")))
    pts = sorted([(s_, 1, q) for s_, e_, q in ev] + [(e_, -1, q) for s_, e_, q in ev])
    active, busy, over, t_prev = {}, 0, 0, None
    for t, dlt, q in pts:
        if t_prev is not None:
            nq = sum(1 for v in active.values() if v > 0)
            busy += (t - t_prev) if nq >= 1 else 0
            over += (t - t_prev) if nq >= 2 else 0
        active[q] = active.get(q, 0) + dlt
        t_prev = t
    print(json.dumps({"dispatches": len(ev), "queues": len({q for _, _, q in ev}), "busy_ms": busy / 1e6,
                      "overlap_ms": over / 1e6, "overlap_fraction": over / max(busy, 1)}), flush=True)


def copy_calibration():
    import torch
    n = (512 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8, "launches": 5}))


def screened_count(s, Q, tau):
    """Screened unique quartets of system s, counted with numpy from the
    Schwarz factors alone (a check on the kernels' own count)."""
    n = s.nshell
    I = np.repeat(np.arange(n), np.arange(1, n + 1))
    J = np.concatenate([np.arange(i + 1) for i in range(n)])
    la = np.maximum(s.shell_l[I], s.shell_l[J])
    lb = np.minimum(s.shell_l[I], s.shell_l[J])
    cls = la * (la + 1) // 2 + lb
    total = 0
    for cb in range(6):
        qb = Q[cls == cb]
        qb = qb[qb > 0]
        for ck in range(cb + 1):
            qk = np.sort(Q[cls == ck])
            cnt = int((len(qk) - np.searchsorted(qk, tau / qb, side="left")).sum())
            if cb == ck:
                cnt = (cnt + int((qb * qb >= tau).sum())) // 2
            total += cnt
    return total


def dzp1024_leg(a):
    """Mixed precision on the 256-atom lattice recipe at 1024 atoms (13312 functions).
    The 128 atoms nearest the centroid: full K in FP64 (the parity-checked
    path) and in mixed precision, max-abs and tr(PK) differences, speedup.
    The 1024-atom system: one bra-pair shard in FP64 and mixed."""
    import torch

    import hfx_inputs as hi
    import paper_2009_03559_amd as hfx

    torch.cuda.init()
    tau, omega = 1e-10, hi.OMEGA_HSE
    big = hi.dzp1024_lattice()
    sub = hi.central_subset(big, 128)
    out = {"metric": "1024-atom lattice, mixed precision", "workload": f"256-atom lattice recipe at 1024 atoms ({big.nbf} functions); "
           f"128-atom subset nearest the centroid ({sub.nbf} functions)", "mixed_cut": a.mixed_cut}
    res = {}
    pairs = hfx.pairs_from_system(sub)
    P = torch.from_numpy(sub.P).cuda()
    want = screened_count(sub, hfx.schwarz_bounds(pairs, hfx.opts(tau=tau, omega=omega)), tau)
    for name, prec in (("fp64", hfx.PREC_FP64), ("mixed", hfx.PREC_MIXED)):
        o = hfx.opts(tau=tau, omega=omega, prec=prec, mixed_cut=a.mixed_cut)
        K = torch.empty_like(P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = hfx.build_K(pairs, P, K, o, stats=True)
        torch.cuda.synchronize()
        res[name] = (K.cpu().numpy(), time.perf_counter() - t0, st)
        print(f"# subset {name}: {res[name][1]:.2f} s, {st['quartets']} quartets ({want} screened)",
              file=sys.stderr, flush=True)
        if st["quartets"] != want:
            raise SystemExit(f"subset {name}: evaluated {st['quartets']} quartets, screening keeps {want}")
    K64, t64, s64 = res["fp64"]
    Km, tm, sm = res["mixed"]
    out["subset128"] = {"quartets": s64["quartets"], "quartets_screened_numpy": want, "fp64_s": t64, "mixed_s": tm, "speedup": t64 / tm,
                        "fp32_quartet_fraction": sm["quartets_fp32"] / max(1, sm["quartets"]),
                        "max_abs_dK_mixed_vs_fp64_gpu": float(np.abs(Km - K64).max()),
                        "trPK_err_mixed_vs_fp64_gpu": float(abs(np.sum(sub.P * Km) - np.sum(sub.P * K64))),
                        "fp64_quartets_per_s": s64["quartets"] / t64, "mixed_quartets_per_s": sm["quartets"] / tm}
    del pairs, P
    pb = hfx.pairs_from_system(big)
    Pb = torch.from_numpy(big.P).cuda()
    Kb = torch.empty_like(Pb)
    shard = {}
    hfx.schwarz_bounds(pb, hfx.opts(tau=tau, omega=omega))
    for name, prec in (("fp64", hfx.PREC_FP64), ("mixed", hfx.PREC_MIXED)):
        o = hfx.opts(tau=tau, omega=omega, prec=prec, mixed_cut=a.mixed_cut)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = hfx.build_K_shard(pb, Pb, Kb, o, 0, a.dzp1024_shards, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        shard[name] = {"s": dt, "quartets": st["quartets"], "quartets_per_s": st["quartets"] / dt,
                       "projected_full_build_s": st["device_s"] * a.dzp1024_shards}
        print(f"# 1024-atom shard {name}: {dt:.2f} s", file=sys.stderr, flush=True)
    shard["speedup"] = shard["fp64"]["s"] / shard["mixed"]["s"]
    out["shard_of_1024"] = dict(shard, shards=a.dzp1024_shards)
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.copy_calib:
        copy_calibration()
        return
    if a.serve_mix:
        serve_mix(a.serve_mix)
        return
    if a.kernel_overlap:
        kernel_overlap(a.kernel_overlap)
        return
    if a.dzp1024:
        dzp1024_leg(a)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported in this build "
              "(the multi-GPU split is hfx_build_K_shard + one all-reduce of K)", file=sys.stderr)
        sys.exit(2)
    import torch

    import hfx_inputs as hi
    import paper_2009_03559_amd as hfx

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    tau, omega = 1e-10, hi.OMEGA_HSE
    sysm = hi.dzp256_lattice() if a.natom == 256 else hi.lattice_system(a.natom, seed=1, name=f"lattice_dzp{a.natom}")
    o = hfx.opts(tau=tau, omega=omega)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    pairs = hfx.pairs_from_system(sysm, o)
    P = torch.from_numpy(sysm.P).to(dev)
    K = torch.empty_like(P)
    # bounds and lists are built once and stay resident (SCF-like reuse)
    hfx.schwarz_bounds(pairs, o)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"# workload {sysm.meta['name']}: {sysm.natom} atoms, {sysm.nshell} shells, {sysm.nbf} functions; "
          f"shard {a.shard}/{a.shards}", file=sys.stderr, flush=True)
    for w in range(a.warmup):
        hfx.build_K_shard(pairs, P, K, o, a.shard, a.shards)
        torch.cuda.synchronize()
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    times, stats = [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(a.steps):
        t0 = time.perf_counter()
        st = hfx.build_K_shard(pairs, P, K, o, a.shard, a.shards, stats=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(st)
        print(f"# step {k}: {times[-1]:.3f} s, {st['quartets']} quartets", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    Kh = K.cpu().numpy()
    assert np.isfinite(Kh).all() and np.abs(Kh - Kh.T).max() == 0.0
    st = stats[-1]
    q_per_step = st["quartets"]
    ms = 1e3 * total / a.steps
    value = q_per_step * a.steps / total
    # roofline of the dominant class kernel (largest device time)
    ci = int(np.argmax(st["class_device_s"]))
    cls_t = np.mean([s["class_device_s"][ci] for s in stats])
    ach = st["class_flops"][ci] / cls_t / 1e12
    dev_s = np.mean([s["device_s"] for s in stats])
    out = {
        "metric": "HFX K-build screened ERI quartets/s",
        "value": value,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{sysm.meta['name']}: {sysm.natom}-atom DZP-like lattice (2s2p1d, 3-6 primitives), "
                        f"{sysm.nshell} shells, {sysm.nbf} functions, erfc omega={omega}, tau={tau}; "
                        f"step = shard {a.shard} of {a.shards} round-robin bra-pair shards of the full K-build",
            "shards": a.shards,
            "precision": "fp64",
        },
        "gflops": st["flops"] / dev_s / 1e9,
        "frac_fp64_vector_peak": st["flops"] / dev_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
        "shard_step_p50_ms": float(np.percentile(times, 50) * 1e3),
        "shard_step_p99_ms": float(np.percentile(times, 99) * 1e3),
        "quartets_per_step": q_per_step,
        "prim_quartets_per_step": st["prim_quartets"],
        "projected_full_build_s": dev_s * a.shards,
        "setup_s": t_setup,
        "class_quartets": dict(zip(hfx.CLASS_NAMES, st["class_quartets"])),
        "class_ms": dict(zip(hfx.CLASS_NAMES, [round(1e3 * x, 3) for x in st["class_device_s"]])),
        "roofline": {
            "bound": "alu",
            "kernel": f"k_eri<Eri{hfx.CLASS_TAGS[ci]}> {hfx.CLASS_NAMES[ci]}",
            "kernel_avg_ms": 1e3 * cls_t,
            "achieved": ach,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": ach / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic_for(hfx.CLASS_TAGS[ci], a.shards),
        },
    }
    if not a.no_mixed:
        # mixed precision on the same shard: quartets with bound < cut in FP32
        om = hfx.opts(tau=tau, omega=omega, prec=hfx.PREC_MIXED, mixed_cut=a.mixed_cut)
        Km = torch.empty_like(P)
        hfx.build_K_shard(pairs, P, Km, om, a.shard, a.shards)  # warm-up (FP32 record copies)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stm = hfx.build_K_shard(pairs, P, Km, om, a.shard, a.shards, stats=True)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        print(f"# mixed step: {tm:.3f} s", file=sys.stderr, flush=True)
        # mixed builds order their lists by (primitive count, FP32 error-scale
        # bin), so their round-robin shard holds other bra pairs than the
        # FP64 shard: the reference is the same build with every quartet in
        # FP64 (cut 0, same lists, same shard)
        o0 = hfx.opts(tau=tau, omega=omega, prec=hfx.PREC_MIXED, mixed_cut=0.0)
        K0 = torch.empty_like(P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hfx.build_K_shard(pairs, P, K0, o0, a.shard, a.shards)
        torch.cuda.synchronize()
        t0m = time.perf_counter() - t0
        Kmh, K0h = Km.cpu().numpy(), K0.cpu().numpy()
        Ph = sysm.P
        out["mixed"] = {
            "value": stm["quartets"] / tm,
            "unit": "quartets/s",
            "ms_per_step": 1e3 * tm,
            "speedup_vs_fp64": ms / (1e3 * tm),
            "speedup_vs_fp64_same_shard": t0m / tm,
            "mixed_cut": a.mixed_cut,
            "fp32_quartet_fraction": stm["quartets_fp32"] / max(1, stm["quartets"]),
            "max_abs_dK_vs_fp64_gpu": float(np.abs(Kmh - K0h).max()),
            "trPK_err_vs_fp64_gpu": float(abs(np.sum(Ph * Kmh) - np.sum(Ph * K0h))),
        }
    if not a.no_density:
        # the same shard with the density-weighted test added to the Schwarz
        # test (P of the workload is zero beyond 12 bohr and decays as
        # exp(-r/3))
        od = hfx.opts(tau=tau, omega=omega, density=True)
        Kd = torch.empty_like(P)
        hfx.build_K_shard(pairs, P, Kd, od, a.shard, a.shards)  # warm-up: |P| block maxima workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        std = hfx.build_K_shard(pairs, P, Kd, od, a.shard, a.shards, stats=True)
        torch.cuda.synchronize()
        td = time.perf_counter() - t0
        print(f"# density-screened step: {td:.3f} s", file=sys.stderr, flush=True)
        out["density_screened"] = {
            "value": std["quartets"] / td,
            "unit": "quartets/s",
            "ms_per_step": 1e3 * td,
            "quartets": std["quartets"],
            "quartet_fraction_kept": std["quartets"] / max(1, q_per_step),
            "speedup_vs_schwarz_only": ms / (1e3 * td),
            "max_abs_dK_vs_schwarz_only": float(np.abs(Kd.cpu().numpy() - Kh).max()),
        }
    if not a.no_jk:
        # Coulomb J digested from the same quartets (FP64): cost over K alone
        Jj, Kj = torch.empty_like(P), torch.empty_like(P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stj = hfx.build_JK_shard(pairs, P, Jj, Kj, o, a.shard, a.shards, stats=True)
        torch.cuda.synchronize()
        tj = time.perf_counter() - t0
        print(f"# J+K step: {tj:.3f} s", file=sys.stderr, flush=True)
        Jh = Jj.cpu().numpy()
        out["coulomb_and_exchange"] = {
            "value": stj["quartets"] / tj,
            "unit": "quartets/s",
            "ms_per_step": 1e3 * tj,
            "time_vs_exchange_only": (1e3 * tj) / ms,
            "max_abs_dK_vs_exchange_only": float(np.abs(Kj.cpu().numpy() - Kh).max()),
            "J_symmetric": bool(np.abs(Jh - Jh.T).max() == 0.0),
        }
    if not a.no_latency:
        out["latency"] = latency_leg(a, hfx, hi, torch)
    if not a.no_periodic:
        out["periodic"] = periodic_leg(a, hfx, hi, torch)
    if not a.no_batch:
        out["batched"] = batch_leg(a, hfx, hi, torch)
    if not a.no_serve:
        out["served"] = serve_leg(a, hfx, hi, torch)
        print("# served leg done", file=sys.stderr, flush=True)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sysm, tau, omega, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
