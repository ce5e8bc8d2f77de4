// Host-code sanitizer driver: runs every entry point of the C ABI on the
// systems of make_input.py and checks the results against the oracle's K
// stored there.  Built together with a copy of the library whose host code
// carries AddressSanitizer and UndefinedBehaviorSanitizer (the executable
// links the sanitizer runtime itself, so nothing is preloaded); any finding
// ends the process with a report.  Exit status 0 means every check passed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hfx.h"

namespace {

int failures = 0;

void check(bool ok, const char *what, double val = 0.0) {
    std::printf("%-52s %s %.3e\n", what, ok ? "ok  " : "FAIL", val);
    std::fflush(stdout);
    if (!ok) ++failures;
}

void need(hfx_status s, const char *what) {
    if (s != HFX_OK) {
        std::printf("%s: status %d (%s)\n", what, (int)s, hfx_last_error());
        std::exit(2);
    }
}

void need_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        std::printf("%s: %s\n", what, hipGetErrorString(e));
        std::exit(2);
    }
}

struct System {
    int32_t natom, nshell, nprim, nbf, nhome, nrow;
    std::vector<double> xyz, exps, coefs, P, Kref;
    std::vector<hfx_shell> shells;
};

template <class T>
void rd(FILE *f, T *p, size_t n) {
    if (std::fread(p, sizeof(T), n, f) != n) {
        std::printf("short input file\n");
        std::exit(2);
    }
}

std::vector<System> load(const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        std::printf("cannot open %s\n", path);
        std::exit(2);
    }
    int32_t n = 0;
    rd(f, &n, 1);
    std::vector<System> out(n);
    for (auto &s : out) {
        int32_t h[6];
        rd(f, h, 6);
        s.natom = h[0], s.nshell = h[1], s.nprim = h[2], s.nbf = h[3], s.nhome = h[4], s.nrow = h[5];
        s.xyz.resize(3 * (size_t)s.natom);
        rd(f, s.xyz.data(), s.xyz.size());
        std::vector<int32_t> sh(4 * (size_t)s.nshell);
        rd(f, sh.data(), sh.size());
        s.shells.resize(s.nshell);
        for (int i = 0; i < s.nshell; ++i) s.shells[i] = {sh[4 * i], sh[4 * i + 1], sh[4 * i + 2], sh[4 * i + 3]};
        s.exps.resize(s.nprim);
        s.coefs.resize(s.nprim);
        rd(f, s.exps.data(), s.nprim);
        rd(f, s.coefs.data(), s.nprim);
        s.P.resize((size_t)s.nbf * s.nbf);
        rd(f, s.P.data(), s.P.size());
        s.Kref.resize((size_t)s.nrow * s.nbf);
        rd(f, s.Kref.data(), s.Kref.size());
    }
    std::fclose(f);
    return out;
}

struct Dev {
    double *p = nullptr;
    size_t n = 0;
    explicit Dev(size_t n_) : n(n_) { need_hip(hipMalloc(&p, n * sizeof(double)), "hipMalloc"); }
    Dev(const std::vector<double> &h) : Dev(h.size()) {
        need_hip(hipMemcpy(p, h.data(), n * sizeof(double), hipMemcpyHostToDevice), "H2D");
    }
    ~Dev() { (void)hipFree(p); }
    std::vector<double> get() const {
        std::vector<double> h(n);
        need_hip(hipMemcpy(h.data(), p, n * sizeof(double), hipMemcpyDeviceToHost), "D2H");
        return h;
    }
};

double maxdiff(const std::vector<double> &a, const std::vector<double> &b, size_t n) {
    double m = 0.0;
    for (size_t i = 0; i < n; ++i) m = std::fmax(m, std::fabs(a[i] - b[i]));
    return m;
}

hfx_opts opts(int32_t prec = HFX_PREC_FP64, int32_t flags = 0) {
    hfx_opts o{};
    o.tau = 1e-10;
    o.op = HFX_OP_ERFC;
    o.omega = 0.11;
    o.prec = prec;
    o.mixed_cut = 1e-5;
    o.prim_tau = 0.0;
    o.flags = flags;
    return o;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 2) {
        std::printf("usage: %s input.bin\n", argv[0]);
        return 2;
    }
    std::vector<System> sys = load(argv[1]);
    std::vector<hfx_pairs> mol_pairs;
    std::vector<Dev *> mol_P, mol_K;
    std::vector<int64_t> mol_ld;
    const hfx_opts o = opts();
    for (size_t si = 0; si < sys.size(); ++si) {
        const System &s = sys[si];
        char tag[64];
        hfx_pairs p = nullptr;
        need(hfx_build_shell_pairs(s.xyz.data(), s.natom, s.shells.data(), s.nshell, s.exps.data(),
                                   s.coefs.data(), &o, nullptr, &p),
             "hfx_build_shell_pairs");
        const int64_t n = s.nbf, npair = hfx_pairs_npair(p);
        check(hfx_pairs_nbf(p) == n && npair == (int64_t)s.nshell * (s.nshell + 1) / 2, "pair counts");
        std::vector<double> q(npair);
        need(hfx_schwarz_bounds(p, &o, q.data(), nullptr), "hfx_schwarz_bounds");
        Dev P(s.P), K(n * n);
        if (s.nhome) {
            Dev Kh((size_t)s.nrow * n);
            need(hfx_build_K_periodic(p, s.nhome, P.p, n, Kh.p, n, &o, nullptr, nullptr), "periodic");
            std::snprintf(tag, sizeof tag, "system %zu periodic K vs oracle", si);
            const double e = maxdiff(Kh.get(), s.Kref, Kh.n);
            check(e <= 1e-10, tag, e);
            check(hfx_build_K_periodic(p, 0, P.p, n, Kh.p, n, &o, nullptr, nullptr) == HFX_EINVAL,
                  "periodic rejects nhome 0");
            hfx_pairs_destroy(p);
            continue;
        }
        hfx_stats st{};
        need(hfx_build_K(p, P.p, K.p, n, &o, nullptr, &st), "hfx_build_K");
        const std::vector<double> K64 = K.get();
        std::snprintf(tag, sizeof tag, "system %zu K vs oracle", si);
        double e = maxdiff(K64, s.Kref, K64.size());
        check(e <= 1e-10, tag, e);
        {
            Dev J(n * n), K2(n * n);
            need(hfx_build_JK(p, P.p, J.p, K2.p, n, &o, nullptr, nullptr), "hfx_build_JK");
            e = maxdiff(K2.get(), K64, K64.size());
            check(e <= 1e-12, "  K of the joint J+K build", e);
        }
        {
            std::vector<double> acc(n * n, 0.0);
            Dev Ks(n * n);
            for (int sh = 0; sh < 3; ++sh) {
                need(hfx_build_K_shard(p, P.p, Ks.p, n, &o, sh, 3, nullptr, nullptr), "shard");
                const std::vector<double> h = Ks.get();
                for (size_t i = 0; i < h.size(); ++i) acc[i] += h[i];
            }
            e = maxdiff(acc, K64, K64.size());
            check(e <= 1e-12, "  three shards add up to K", e);
            Dev Js(n * n);
            need(hfx_build_JK_shard(p, P.p, Js.p, Ks.p, n, &o, 1, 3, nullptr, nullptr), "JK shard");
        }
        {
            const hfx_opts om = opts(HFX_PREC_MIXED);
            Dev Km(n * n);
            need(hfx_build_K(p, P.p, Km.p, n, &om, nullptr, nullptr), "mixed");
            e = maxdiff(Km.get(), s.Kref, K64.size());
            check(e <= 1e-6, "  mixed K vs oracle", e);
            const hfx_opts od = opts(HFX_PREC_FP64, HFX_FLAG_DENSITY_SCREEN);
            need(hfx_build_K(p, P.p, Km.p, n, &od, nullptr, nullptr), "density");
            e = maxdiff(Km.get(), s.Kref, K64.size());
            check(e <= 1e-8, "  density-screened K vs oracle", e);
            need(hfx_build_K_noalloc(p, P.p, Km.p, n, &o, nullptr, nullptr), "noalloc");
            e = maxdiff(Km.get(), K64, K64.size());
            check(e <= 1e-12, "  allocation-free K", e);
        }
        {
            const int32_t nq = 3;
            std::vector<int32_t> quart = {0, 0, 0, 0, 1, 0, 1, 0, s.nshell - 1, 0, s.nshell - 1, 1};
            std::vector<double> out(nq * 625);
            const hfx_status r = hfx_eval_quartets(p, &o, nq, quart.data(), out.data(), nullptr);
            check(r == HFX_OK, "  hfx_eval_quartets");
        }
        check(hfx_build_K(p, nullptr, K.p, n, &o, nullptr, nullptr) == HFX_EINVAL, "  null P rejected");
        check(hfx_build_K(p, P.p, K.p, n - 1, &o, nullptr, nullptr) == HFX_EINVAL, "  short ld rejected");
        mol_pairs.push_back(p);
        mol_P.push_back(new Dev(s.P));
        mol_K.push_back(new Dev(n * n));
        mol_ld.push_back(n);
    }
    // batched launch over the molecular systems, then the server
    const int32_t nm = (int32_t)mol_pairs.size();
    std::vector<const double *> Pp(nm);
    std::vector<double *> Kp(nm);
    for (int i = 0; i < nm; ++i) Pp[i] = mol_P[i]->p, Kp[i] = mol_K[i]->p;
    need(hfx_build_K_batch(nm, mol_pairs.data(), Pp.data(), Kp.data(), mol_ld.data(), &o, nullptr, nullptr),
         "batch");
    int mi = 0;
    for (size_t si = 0; si < sys.size(); ++si) {
        if (sys[si].nhome) continue;
        const double e = maxdiff(mol_K[mi]->get(), sys[si].Kref, sys[si].Kref.size());
        check(e <= 1e-10, "batched K vs oracle", e);
        ++mi;
    }
    hfx_server srv = nullptr;
    need(hfx_server_create(int64_t(1) << 32, 2, &srv), "server");
    std::vector<uint64_t> tickets(nm);
    for (int i = 0; i < nm; ++i)
        need(hfx_submit(srv, mol_pairs[i], mol_P[i]->p, mol_K[i]->p, mol_ld[i], &o, &tickets[i]), "submit");
    for (int i = 0; i < nm; ++i) {
        int32_t done = 0;
        hfx_stats st{};
        while (!done) need(hfx_poll(srv, tickets[i], &done, &st), "poll");
    }
    int32_t d = 0;
    check(hfx_poll(srv, 987654321ull, &d, nullptr) == HFX_ENOTFOUND, "unknown ticket rejected");
    mi = 0;
    for (size_t si = 0; si < sys.size(); ++si) {
        if (sys[si].nhome) continue;
        const double e = maxdiff(mol_K[mi]->get(), sys[si].Kref, sys[si].Kref.size());
        check(e <= 1e-10, "served K vs oracle", e);
        ++mi;
    }
    hfx_server_destroy(srv);
    for (int i = 0; i < nm; ++i) {
        hfx_pairs_destroy(mol_pairs[i]);
        delete mol_P[i];
        delete mol_K[i];
    }
    std::printf("%s: %d failures\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
}
