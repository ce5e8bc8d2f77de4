// Batched and served exchange builds.
//
// Batch: every system's lists are built as for hfx_build_K; then, per
// angular-momentum class, one persistent launch drains a device work queue
// that holds the class's tiles of all systems (largest jobs first), popped
// through an atomic head.  This is the dynamic distribution the paper's
// conclusion (Sec. 5) proposes in place of its static pair/quartet splits,
// applied across systems.  The quartet-block size (ket quartets per tile),
// the claim size and the persistent grid are chosen per class by an
// autotuner that times candidates on a strided sample of the batch's own
// tiles and caches the winner per device (in memory and in a text file).
//
// Server: a request loop.  Submissions are queued; worker threads, each with
// its own stream, take the oldest request that fits the HBM budget and whose
// pair handle is not busy, so requests that arrive while others run are
// admitted as slots and memory free up, and their kernels overlap on the
// device (continuous batching).  Pair data stays resident in its handle
// across the SCF iterations of a request.  A build allocates and frees no
// device memory once its handle holds its bounds and lists (a hipFree would
// wait for the kernels of every stream and serialise the workers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "hfx.h"
#include "hfx_device.hpp"
#include "hfx_internal.hpp"

namespace hfx {

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess)                                                          \
            return fail(HFX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));  \
    } while (0)

#define HFX_FOR_CLASSES(X) \
    X(0000) X(1000) X(1010) X(1100) X(1110) X(1111) X(2000) X(2010) X(2011) X(2020) X(2100) \
    X(2110) X(2111) X(2120) X(2121) X(2200) X(2210) X(2211) X(2220) X(2221) X(2222)
#define DECL(T)                                                                                          \
    void launch_persist_##T(const BatchJob *, int, long long, unsigned long long *, int, unsigned,      \
                            hipStream_t);                                                               \
    void launch_persist32_##T(const BatchJob *, int, long long, unsigned long long *, int, unsigned,    \
                              hipStream_t);                                                             \
    int nsplit_##T();                                                                                   \
    int nsplit32_##T();
HFX_FOR_CLASSES(DECL)
#undef DECL

typedef void (*persist_fn)(const BatchJob *, int, long long, unsigned long long *, int, unsigned, hipStream_t);
typedef int (*nsplit_fn)();
static const persist_fn k_persist_tab[2][21] = {
    {
#define E(T) launch_persist_##T,
        HFX_FOR_CLASSES(E)
#undef E
    },
    {
#define E(T) launch_persist32_##T,
        HFX_FOR_CLASSES(E)
#undef E
    }};
static const nsplit_fn k_nsplit_tab[2][21] = {
    {
#define E(T) nsplit_##T,
        HFX_FOR_CLASSES(E)
#undef E
    },
    {
#define E(T) nsplit32_##T,
        HFX_FOR_CLASSES(E)
#undef E
    }};

// ------------------------------------------------------------ autotune ----
struct Tune {
    int tq = 0;          // ket quartets per tile (0 = whole range)
    int claim = 1;       // virtual blocks per atomic pop
    int grid_per_cu = 8; // persistent workgroups per CU
};

static std::mutex g_tune_mu;
static std::map<std::string, Tune> g_tune;
static bool g_tune_loaded = false;

static std::string tune_path() {
    const char *e = std::getenv("HFX_TUNE_CACHE");
    if (e && *e) return e;
    const char *h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/hfx_autotune.txt";
}

static std::string dev_name() {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    return std::string(pr.gcnArchName) + "-cu" + std::to_string(pr.multiProcessorCount);
}

static void load_tune() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::ifstream f(tune_path());
    std::string key;
    Tune t;
    while (f >> key >> t.tq >> t.claim >> t.grid_per_cu) g_tune[key] = t;
}

static void save_tune() {
    std::string path = tune_path();
    std::string dir = path.substr(0, path.find_last_of('/'));
    std::string cmd;
    (void)cmd;
    std::ofstream f(path);
    if (!f) return;  // the cache is optional
    for (auto &kv : g_tune) f << kv.first << " " << kv.second.tq << " " << kv.second.claim << " " << kv.second.grid_per_cu << "\n";
}

// --------------------------------------------------------------- batch ----
struct ClassJobs {
    std::vector<BatchJob> jobs;
    long long vtotal = 0;
};

static void make_jobs(ClassJobs &cj, int ci, int nsys, hfx_pairs const *p, const double *const *P,
                      double *const *K, const int64_t *ld, const hfx_opts *o, bool f32,
                      unsigned long long *const *cnt, int tq, int nsplit, int bra_stride) {
    int cb = 0;
    while ((cb + 1) * (cb + 2) / 2 <= ci) ++cb;
    const int ck = ci - cb * (cb + 1) / 2;
    const int op = kernel_op(o);
    const bool mixed = (o->prec == HFX_PREC_MIXED);
    std::vector<std::pair<double, int>> order;
    for (int s = 0; s < nsys; ++s) {
        const ClassList &B = class_lists(p[s], mixed)[cb], &Kl = class_lists(p[s], mixed)[ck];
        if (!B.n || !Kl.n) continue;
        if (f32 && !(mixed && o->mixed_cut > 0.0)) continue;
        order.push_back({-(double)B.n * (double)Kl.n, s});  // largest first
    }
    std::sort(order.begin(), order.end());
    cj.jobs.clear();
    cj.vtotal = 0;
    for (auto &os : order) {
        const int s = os.second;
        const ClassList &B = class_lists(p[s], mixed)[cb], &Kl = class_lists(p[s], mixed)[ck];
        BatchJob j;
        std::memset(&j, 0, sizeof(j));
        QuartetArgs &a = j.a;
        a.hdr = p[s]->d_hdr;
        a.prim = p[s]->d_prim;
        a.prim32 = p[s]->d_prim32;
        a.bra_ids = B.d_ids;
        a.bra_Q = B.d_Q;
        a.bra_grp = B.d_grp;
        a.n_bra = B.n;
        a.bra_first = 0;
        a.bra_stride = 1;
        a.nsub = 1;
        a.tq = 1 << 30;
        a.ket_ids = Kl.d_ids;
        a.ket_Q = Kl.d_Q;
        a.ket_goff = Kl.d_goff;
        a.ket_gnp = Kl.d_gnp;
        a.n_kgrp = Kl.ngrp;
        a.same = (cb == ck);
        a.op = op;
        a.om2 = op ? o->omega * o->omega : 0.0;
        a.om = op ? o->omega : 0.0;
        a.prim_tau = o->prim_tau;
        a.boys = p[s]->d_boys;
        a.boys32 = p[s]->d_boys32;
        a.P = P[s];
        a.K = K[s];
        a.ld = ld[s];
        // FP64 side (all of it unless mixed) and FP32 side of the per-block
        // split on the FP32 error scale (see ket_cut)
        a.tau = o->tau;
        a.tau_hi = HUGE_VAL;
        a.part = mixed ? (f32 ? 2 : 1) : 0;
        a.mixed_cut = o->mixed_cut;
        a.bra_A = B.d_A;
        a.ket_gA = Kl.d_gA;
        a.dens = density_mode(o, false);
        a.nsh = p[s]->nshell;
        a.pmax = p[s]->d_pmax;
        a.count = cnt ? cnt[s] + 4 * ci + (f32 ? 2 : 0) : nullptr;
        int gmax = 1;
        for (size_t g = 0; g + 1 < Kl.goff.size(); ++g) gmax = std::max(gmax, Kl.goff[g + 1] - Kl.goff[g]);
        j.tq = tq > 0 ? tq : gmax;
        j.nsub = (gmax + j.tq - 1) / j.tq;
        // bra slots 0, stride, 2 stride, ... (stride > 1: a sample for autotuning)
        a.bra_first = 0;
        a.bra_stride = bra_stride;
        const long long nbra = (B.n + bra_stride - 1) / bra_stride;
        j.vbase = cj.vtotal;
        cj.vtotal += nbra * (long long)Kl.ngrp * j.nsub * nsplit;
        cj.jobs.push_back(j);
    }
}

struct BatchRun {
    std::vector<BatchJob *> dev_jobs;
    ~BatchRun() {
        for (auto *d : dev_jobs) hipFree(d);
    }
};

static hfx_status launch_class(int ci, bool f32, ClassJobs &cj, const Tune &t, unsigned long long *head,
                               hipStream_t st, BatchRun &run) {
    if (cj.jobs.empty() || cj.vtotal == 0) return HFX_OK;
    BatchJob *d = nullptr;
    HIPCHK(hipMalloc(&d, cj.jobs.size() * sizeof(BatchJob)));
    run.dev_jobs.push_back(d);
    HIPCHK(hipMemcpyAsync(d, cj.jobs.data(), cj.jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, st));
    launch_fill_u64(head, 1, st);
    int dev = 0, ncu = 256;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::max(1, ncu * t.grid_per_cu);
    k_persist_tab[f32 ? 1 : 0][ci](d, (int)cj.jobs.size(), cj.vtotal, head, t.claim, grid, st);
    HIPCHK(hipGetLastError());
    return HFX_OK;
}

static hfx_status autotune_class(int ci, bool f32, int nsys, hfx_pairs const *p, const double *const *P,
                                 double *const *Kscratch, const int64_t *ld, const hfx_opts *o,
                                 unsigned long long *head, hipStream_t st, Tune *best_out) {
    const int nsplit = k_nsplit_tab[f32 ? 1 : 0][ci]();
    // four candidates: a wider search (three tile sizes x two claim sizes x
    // three grids, 18 in all) gained 1-2 % over the defaults at most and made
    // the first batched call several times longer
    const int tqs[] = {0, 256};
    const int claims[] = {1};
    const int grids[] = {4, 8};
    double best = 1e300;
    Tune best_t;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int tq : tqs)
        for (int cl : claims)
            for (int gr : grids) {
                Tune t;
                t.tq = tq;
                t.claim = cl;
                t.grid_per_cu = gr;
                ClassJobs cj;
                make_jobs(cj, ci, nsys, p, P, Kscratch, ld, o, f32, nullptr, tq, nsplit, 16);
                if (cj.jobs.empty()) {
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    *best_out = Tune();
                    return HFX_OK;
                }
                BatchRun run;
                HIPCHK(hipEventRecord(e0, st));
                hfx_status s = launch_class(ci, f32, cj, t, head, st, run);
                if (s != HFX_OK) return s;
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_t = t;
                }
            }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *best_out = best_t;
    return HFX_OK;
}

hfx_status batch_impl(int32_t nsys, const hfx_pairs *p, const double *const *P, double *const *K,
                      const int64_t *ld, const hfx_opts *o, void *stream, hfx_stats *st_out) {
    auto t0 = std::chrono::steady_clock::now();
    if (nsys < 0 || (nsys > 0 && (!p || !P || !K || !ld))) return fail(HFX_EINVAL, "bad batch arrays");
    hfx_status s = check_opts(o);
    if (s != HFX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < nsys; ++i) {
        if (!p[i] || !P[i] || !K[i]) return fail(HFX_EINVAL, "NULL entry in batch");
        for (int j = 0; j < i; ++j)
            if (p[j] == p[i]) return fail(HFX_EINVAL, "a pair handle appears twice in one batch");
        const int64_t n = p[i]->nbf;
        if (ld[i] < n) return fail(HFX_EINVAL, "ld < n_bf");
        s = check_P(P[i], n, ld[i], st, p[i]->d_part);
        if (s != HFX_OK) return s;
        s = compute_bounds(p[i], o, st);
        if (s != HFX_OK) return s;
        s = build_lists(p[i], o->tau, o->prec == HFX_PREC_MIXED, st);
        if (s != HFX_OK) return s;
        if (o->flags & HFX_FLAG_DENSITY_SCREEN) s = shell_pmax(p[i], P[i], ld[i], true, st);
        if (s != HFX_OK) return s;
        if (o->prec == HFX_PREC_MIXED) {
            s = ensure_prim32(p[i], st);
            if (s != HFX_OK) return s;
        }
        launch_fill_u64(p[i]->d_count, NCOUNT, st);
    }
    unsigned long long *head = nullptr;
    HIPCHK(hipMalloc(&head, 2 * sizeof(unsigned long long)));
    std::unique_ptr<unsigned long long, void (*)(unsigned long long *)> head_guard(
        head, [](unsigned long long *x) { hipFree(x); });
    // autotune the classes not yet known for this device (into scratch K)
    const std::string dn = dev_name();
    std::vector<Tune> tune(2 * HFX_NCLASS);
    // HFX_TUNE=0: the default parameters for every class, nothing timed
    const char *tenv = std::getenv("HFX_TUNE");
    const bool no_tune = tenv && std::strcmp(tenv, "0") == 0;
    if (!no_tune) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune();
        bool changed = false;
        double *scratch = nullptr;
        for (int f = 0; f < 2; ++f)
            for (int ci = 0; ci < HFX_NCLASS; ++ci) {
                if (f == 1 && o->prec != HFX_PREC_MIXED) continue;
                const std::string key = dn + ":" + std::to_string(ci) + (f ? ":f32" : ":f64");
                auto it = g_tune.find(key);
                if (it != g_tune.end()) {
                    tune[f * HFX_NCLASS + ci] = it->second;
                    continue;
                }
                if (!scratch) {
                    int64_t mx = 0;
                    for (int i = 0; i < nsys; ++i) mx = std::max(mx, p[i]->nbf * ld[i]);
                    HIPCHK(hipMalloc(&scratch, std::max<int64_t>(mx, 1) * sizeof(double)));
                }
                std::vector<double *> ks(nsys, scratch);
                Tune t;
                s = autotune_class(ci, f == 1, nsys, p, P, ks.data(), ld, o, head, st, &t);
                if (s != HFX_OK) {
                    hipFree(scratch);
                    return s;
                }
                bool any = false;
                for (int i = 0; i < nsys; ++i) {
                    int cb = 0;
                    while ((cb + 1) * (cb + 2) / 2 <= ci) ++cb;
                    const int ck = ci - cb * (cb + 1) / 2;
                    const ClassList *ls = class_lists(p[i], o->prec == HFX_PREC_MIXED);
                    any |= ls[cb].n && ls[ck].n;
                }
                tune[f * HFX_NCLASS + ci] = t;
                if (any) {
                    g_tune[key] = t;
                    changed = true;
                }
            }
        if (scratch) {
            HIPCHK(hipStreamSynchronize(st));
            hipFree(scratch);
        }
        if (changed) save_tune();
    }
    for (int i = 0; i < nsys; ++i) launch_fill_K(K[i], p[i]->nbf, ld[i], st);
    std::vector<unsigned long long *> cnt(nsys);
    for (int i = 0; i < nsys; ++i) cnt[i] = p[i]->d_count;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st_out) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, st));
    }
    BatchRun run;
    for (int f = 0; f < 2; ++f)
        for (int ci = 0; ci < HFX_NCLASS; ++ci) {
            if (f == 1 && !(o->prec == HFX_PREC_MIXED && o->mixed_cut > 0.0)) continue;
            const Tune &t = tune[f * HFX_NCLASS + ci];
            ClassJobs cj;
            make_jobs(cj, ci, nsys, p, P, K, ld, o, f == 1, cnt.data(), t.tq, k_nsplit_tab[f][ci](), 1);
            s = launch_class(ci, f == 1, cj, t, head + (f & 1), st, run);
            if (s != HFX_OK) return s;
        }
    if (st_out) HIPCHK(hipEventRecord(e1, st));
    for (int i = 0; i < nsys; ++i) launch_symmetrize(K[i], p[i]->nbf, ld[i], st);
    HIPCHK(hipGetLastError());
    if (st_out) {
        HIPCHK(hipStreamSynchronize(st));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        std::memset(st_out, 0, sizeof(*st_out));
        st_out->device_s = ms * 1e-3;
        const double *mv = model_vrr(), *mp = model_post();
        for (int i = 0; i < nsys; ++i) {
            std::vector<unsigned long long> h(4 * HFX_NCLASS);
            HIPCHK(hipMemcpy(h.data(), cnt[i], h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
            for (int c = 0; c < HFX_NCLASS; ++c) {
                int cb = 0;
                while ((cb + 1) * (cb + 2) / 2 <= c) ++cb;
                const int ck = c - cb * (cb + 1) / 2;
                const int L = PAIR_L[cb][0] + PAIR_L[cb][1] + PAIR_L[ck][0] + PAIR_L[ck][1];
                const double nq = (double)(h[4 * c] + h[4 * c + 2]), npq = (double)(h[4 * c + 1] + h[4 * c + 3]);
                const double fl = (mv[c] + model_prim_overhead(kernel_op(o), L)) * npq + mp[c] * nq;
                st_out->class_quartets[c] += (int64_t)nq;
                st_out->class_flops[c] += fl;
                st_out->quartets += (int64_t)nq;
                st_out->quartets_fp32 += (int64_t)h[4 * c + 2];
                st_out->prim_quartets += (int64_t)npq;
                st_out->flops += fl;
            }
        }
        st_out->latency_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } else {
        HIPCHK(hipStreamSynchronize(st));  // job tables are freed on return
    }
    return HFX_OK;
}

}  // namespace hfx

using namespace hfx;

namespace {
// Systems with at least this many basis functions fill the device on their
// own and run on the direct kernels; the rest share the persistent launches.
// Measured on 64 lattice systems, batch time against one by one: all in the
// queue, 6-20 atoms (78-260 functions) 1.5x faster, 20-40 atoms (260-520)
// 0.87x; from 300 functions direct 1.55x / 0.93x, from 200 1.38x / 0.99x,
// from 150 1.19x / 1.00x.
int64_t direct_nbf() {
    if (const char *e = std::getenv("HFX_BATCH_DIRECT_NBF")) return std::atoll(e);
    return 250;
}

void add_stats(hfx_stats &a, const hfx_stats &b) {
    a.device_s += b.device_s;
    a.quartets += b.quartets;
    a.quartets_fp32 += b.quartets_fp32;
    a.prim_quartets += b.prim_quartets;
    a.flops += b.flops;
    for (int c = 0; c < HFX_NCLASS; ++c) {
        a.class_quartets[c] += b.class_quartets[c];
        a.class_device_s[c] += b.class_device_s[c];
        a.class_flops[c] += b.class_flops[c];
    }
}
}  // namespace

extern "C" hfx_status hfx_build_K_batch(int32_t nsys, const hfx_pairs *p, const double *const *P,
                                        double *const *K, const int64_t *ld, const hfx_opts *o, void *stream,
                                        hfx_stats *st) {
    const auto t0 = std::chrono::steady_clock::now();
    if (nsys < 0 || (nsys > 0 && (!p || !P || !K || !ld))) return fail(HFX_EINVAL, "bad batch arrays");
    for (int i = 0; i < nsys; ++i) {
        if (!p[i] || !P[i] || !K[i]) return fail(HFX_EINVAL, "NULL entry in batch");
        for (int j = 0; j < i; ++j)
            if (p[j] == p[i]) return fail(HFX_EINVAL, "a pair handle appears twice in one batch");
    }
    const int64_t thr = direct_nbf();
    std::vector<hfx_pairs> sp;
    std::vector<const double *> sP;
    std::vector<double *> sK;
    std::vector<int64_t> sld;
    std::vector<int> big;
    for (int i = 0; i < nsys; ++i) {
        if (thr > 0 && p[i]->nbf >= thr) {
            big.push_back(i);
        } else {
            sp.push_back(p[i]);
            sP.push_back(P[i]);
            sK.push_back(K[i]);
            sld.push_back(ld[i]);
        }
    }
    if (big.empty()) return batch_impl(nsys, p, P, K, ld, o, stream, st);
    hfx_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    if (!sp.empty()) {
        hfx_stats s1;
        const hfx_status s = batch_impl((int32_t)sp.size(), sp.data(), sP.data(), sK.data(), sld.data(), o, stream,
                                        st ? &s1 : nullptr);
        if (s != HFX_OK) return s;
        if (st) add_stats(acc, s1);
    }
    for (int i : big) {
        hfx_stats s1;
        const hfx_status s = build_K_impl(p[i], P[i], K[i], ld[i], o, 0, 1, stream, st ? &s1 : nullptr);
        if (s != HFX_OK) return s;
        if (st) add_stats(acc, s1);
    }
    if (st) {
        acc.latency_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *st = acc;
    }
    return HFX_OK;
}

// -------------------------------------------------------------- server ----
struct hfx_server_s {
    struct Req {
        hfx_pairs p;
        const double *P;
        double *K;
        int64_t ld;
        hfx_opts o;
        int64_t bytes;
        std::chrono::steady_clock::time_point t_sub;
        bool done = false, running = false;
        hfx_status status = HFX_OK;
        std::string err;
        hfx_stats st;
    };
    int64_t budget = 0;
    int max_inflight = 1;
    int dev = 0;
    size_t max_queue = 4096;
    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, Req> reqs;
    std::deque<uint64_t> pending;
    std::set<hfx_pairs> busy;
    int64_t inflight_bytes = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;

    void worker() {
        hipSetDevice(dev);
        hipStream_t st = nullptr;
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        for (;;) {
            uint64_t id = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stop) break;
                    // oldest admissible request: fits the budget, handle not busy
                    auto it = pending.begin();
                    for (; it != pending.end(); ++it) {
                        Req &r = reqs[*it];
                        if (busy.count(r.p)) continue;
                        if (inflight_bytes + r.bytes > budget) continue;
                        break;
                    }
                    if (it != pending.end()) {
                        id = *it;
                        pending.erase(it);
                        Req &r = reqs[id];
                        r.running = true;
                        busy.insert(r.p);
                        inflight_bytes += r.bytes;
                        break;
                    }
                    cv.wait(lk);
                }
                if (!id) break;
            }
            Req *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                r = &reqs[id];
            }
            hfx_stats st_local;
            hfx_status s = build_K_impl(r->p, r->P, r->K, r->ld, &r->o, 0, 1, st, &st_local);
            std::string msg = s == HFX_OK ? std::string() : std::string(hfx_last_error());
            {
                std::lock_guard<std::mutex> lk(mu);
                r->status = s;
                r->err = msg;
                r->st = st_local;
                r->st.latency_s =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_sub).count();
                r->done = true;
                r->running = false;
                busy.erase(r->p);
                inflight_bytes -= r->bytes;
            }
            cv.notify_all();
        }
        if (st) hipStreamDestroy(st);
    }
};

extern "C" hfx_status hfx_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, hfx_server *out) {
    if (!out) return fail(HFX_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || max_inflight < 1 || max_inflight > 64)
        return fail(HFX_EINVAL, "budget must be > 0 and max_inflight in [1, 64]");
    std::unique_ptr<hfx_server_s> s(new hfx_server_s());
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    // capacity of the queue of waiting requests (submit returns HFX_EBUSY when
    // it is full); HFX_SERVER_QUEUE overrides the default of 4096
    if (const char *e = std::getenv("HFX_SERVER_QUEUE"))
        if (*e) s->max_queue = (size_t)std::max(1ll, std::atoll(e));
    if (hipGetDevice(&s->dev) != hipSuccess) return fail(HFX_EDEVICE, "hipGetDevice failed");
    for (int i = 0; i < max_inflight; ++i) s->workers.emplace_back(&hfx_server_s::worker, s.get());
    *out = s.release();
    return HFX_OK;
}

extern "C" hfx_status hfx_submit(hfx_server s, hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                                 const hfx_opts *o, uint64_t *ticket) {
    if (!s || !p || !P_dev || !K_dev || !ticket) return fail(HFX_EINVAL, "NULL argument");
    hfx_status st = check_opts(o);
    if (st != HFX_OK) return st;
    if (ld < p->nbf) return fail(HFX_EINVAL, "ld < n_bf");
    // device memory the request holds while it runs: its resident pair data
    // (plus FP32 copies in mixed mode) and its P and K
    int64_t bytes = p->dev_bytes + 2 * p->nbf * ld * (int64_t)sizeof(double);
    if (o->prec == HFX_PREC_MIXED && !p->d_prim32) bytes += p->nrec * (int64_t)sizeof(PrimRec32);
    std::lock_guard<std::mutex> lk(s->mu);
    if (bytes > s->budget) return fail(HFX_ENOMEM, "request larger than the server's HBM budget");
    if (s->pending.size() >= s->max_queue) return fail(HFX_EBUSY, "server queue full");
    const uint64_t id = s->next_id++;
    hfx_server_s::Req &r = s->reqs[id];
    r.p = p;
    r.P = P_dev;
    r.K = K_dev;
    r.ld = ld;
    r.o = *o;
    r.bytes = bytes;
    r.t_sub = std::chrono::steady_clock::now();
    s->pending.push_back(id);
    *ticket = id;
    s->cv.notify_all();
    return HFX_OK;
}

extern "C" hfx_status hfx_poll(hfx_server s, uint64_t ticket, int32_t *done, hfx_stats *st) {
    if (!s || !done) return fail(HFX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(HFX_ENOTFOUND, "unknown ticket");
    if (!it->second.done) {
        *done = 0;
        return HFX_OK;
    }
    *done = 1;
    if (st) *st = it->second.st;
    hfx_status r = it->second.status;
    std::string msg = it->second.err;
    s->reqs.erase(it);
    if (r != HFX_OK) return fail(r, msg);
    return HFX_OK;
}

extern "C" void hfx_server_destroy(hfx_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto &t : s->workers) t.join();
    delete s;
}
