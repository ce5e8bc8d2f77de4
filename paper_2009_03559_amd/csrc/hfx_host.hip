// libhfx host side: basis setup, pair enumeration, Schwarz bounds, screened
// class-sorted quartet lists and the launch sequence of the exchange build.
//
// Paper mapping (Sec. 3): contracted shells; pair lists preselected with the
// Schwarz factors; per-quartet Schwarz screening; 8-fold symmetry (unique
// quartets plus degeneracy factors, digestion of four images and K = K' + K'^T);
// Cartesian->spherical transform.  The static MPI shell-pair / shell-quartet
// distributions of Sec. 3.1 are replaced by one GPU grid over
// (bra pair, ket group) whose ket range is cut by binary search on the
// Q-sorted list: the screened quartet set is never materialised.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "hfx.h"
#include "hfx_device.hpp"
#include "hfx_internal.hpp"

namespace hfx {

thread_local std::string g_err;

hfx_status fail(hfx_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess)                                                          \
            return fail(HFX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));  \
    } while (0)

// ---------------------------------------------------------------- Boys ----
// F_m(x) on the grid x_i = i/32, m = 0..14, in long double: the top order by
// its power series  F_M(x) = e^-x sum_k (2x)^k / ((2M+1)(2M+3)...(2M+2k+1)),
// the lower orders by the stable downward recursion.  Stored as
// T_L[i][k] = F_(L+k)(x_i) / k! for k = 0..6 and T_L[i][7] = e^-x_i.
static std::vector<double> make_boys_table() {
    const int M = BOYS_LMAX + BOYS_NTAY - 2;
    std::vector<double> tab((size_t)BOYS_TAB_SIZE);
    std::vector<long double> F(M + 1);
    for (int i = 0; i < BOYS_NROW; ++i) {
        long double x = (long double)i / 32.0L;
        long double term = 1.0L / (2 * M + 1), sum = term;
        for (int k = 1; k < 4000; ++k) {
            term *= 2.0L * x / (2 * M + 2 * k + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        long double ex = expl(-x);
        F[M] = ex * sum;
        for (int m = M - 1; m >= 0; --m) F[m] = (2.0L * x * F[m + 1] + ex) / (2 * m + 1);
        for (int L = 0; L <= BOYS_LMAX; ++L) {
            long double fact = 1.0L;
            for (int k = 0; k < BOYS_NTAY - 1; ++k) {
                if (k > 0) fact *= k;
                tab[((size_t)L * BOYS_NROW + i) * BOYS_NTAY + k] = (double)(F[L + k] / fact);
            }
            tab[((size_t)L * BOYS_NROW + i) * BOYS_NTAY + BOYS_NTAY - 1] = (double)ex;
        }
    }
    return tab;
}

static std::mutex g_boys_mu;
static std::vector<double *> g_boys_dev;  // per device
static std::vector<float *> g_boys32_dev;  // per device: the same table rounded to FP32

static hfx_status boys_table(const double **out, const float **out32) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_boys_mu);
    if ((int)g_boys_dev.size() <= dev) {
        g_boys_dev.resize(dev + 1, nullptr);
        g_boys32_dev.resize(dev + 1, nullptr);
    }
    if (!g_boys_dev[dev]) {
        std::vector<double> t = make_boys_table();
        std::vector<float> t32(t.begin(), t.end());
        double *d = nullptr;
        float *d32 = nullptr;
        HIPCHK(hipMalloc(&d, t.size() * sizeof(double)));
        HIPCHK(hipMemcpy(d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMalloc(&d32, t32.size() * sizeof(float)));
        HIPCHK(hipMemcpy(d32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
        g_boys_dev[dev] = d;
        g_boys32_dev[dev] = d32;
    }
    *out = g_boys_dev[dev];
    *out32 = g_boys32_dev[dev];
    return HFX_OK;
}

// ------------------------------------------------------------ kernels ----
// Primitive-pair records of every pair.
struct ShellDev {
    double x, y, z;
    int32_t nprim, off;
};

__global__ void k_pairdata(const PairHdr *__restrict__ hdr, const int32_t *__restrict__ shA,
                           const int32_t *__restrict__ shB, const ShellDev *__restrict__ sh,
                           const double *__restrict__ ex, const double *__restrict__ cn, int64_t npair,
                           PrimRec *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair) return;
    const PairHdr h = hdr[t];
    const ShellDev A = sh[shA[t]], B = sh[shB[t]];
    const double ab2 = h.ABx * h.ABx + h.ABy * h.ABy + h.ABz * h.ABz;
    const double c0 = 5.914967172795613;  // sqrt(2) pi^(5/4)
    int r = h.off;
    for (int i = 0; i < A.nprim; ++i) {
        const double a = ex[A.off + i], ca = cn[A.off + i];
        for (int j = 0; j < B.nprim; ++j) {
            const double b = ex[B.off + j], cb = cn[B.off + j];
            const double z = a + b, iz = 1.0 / z;
            PrimRec p;
            p.z = z;
            p.i2z = 0.5 * iz;
            p.Px = (a * A.x + b * B.x) * iz;
            p.Py = (a * A.y + b * B.y) * iz;
            p.Pz = (a * A.z + b * B.z) * iz;
            p.PAx = p.Px - A.x;
            p.PAy = p.Py - A.y;
            p.PAz = p.Pz - A.z;
            p.K = c0 * ca * cb * exp(-a * b * iz * ab2) * iz;
            p.B = 0.0;
            out[r++] = p;
        }
    }
}

__global__ void k_to_f32(const PrimRec *__restrict__ in, int64_t n, PrimRec32 *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const PrimRec r = in[t];
    PrimRec32 o;
    o.Px = r.Px;
    o.Py = r.Py;
    o.Pz = r.Pz;
    o.z = (float)r.z;
    o.i2z = (float)r.i2z;
    o.PAx = (float)r.PAx;
    o.PAy = (float)r.PAy;
    o.PAz = (float)r.PAz;
    o.K = (float)r.K;
    o.B = (float)r.B;
    o.pad = 0.0f;
    out[t] = o;
}

__global__ void k_fill(double *K, int64_t n, int64_t ld) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    K[(t / n) * ld + t % n] = 0.0;
}

__global__ void k_fill_rect(double *K, int64_t rows, int64_t cols, int64_t ld) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    K[(t / cols) * ld + t % cols] = 0.0;
}

__global__ void k_fill_u64(unsigned long long *c, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) c[t] = 0ull;
}

void launch_fill_K(double *K, int64_t n, int64_t ld, hipStream_t st);
void launch_fill_u64(unsigned long long *c, int n, hipStream_t st);
void launch_symmetrize(double *K, int64_t n, int64_t ld, hipStream_t st);

void launch_fill_K(double *K, int64_t n, int64_t ld, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, K, n, ld);
}
void launch_fill_u64(unsigned long long *c, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, c, n);
}

// K = K' + K'^T in place; one thread per (i, j) with j >= i.
__global__ void k_symmetrize(double *K, int64_t n, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.y * 16 + threadIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 16 + threadIdx.x;
    if (i >= n || j >= n || j < i) return;
    const double s = K[i * ld + j] + K[j * ld + i];
    K[i * ld + j] = s;
    K[j * ld + i] = s;
}

void launch_symmetrize(double *K, int64_t n, int64_t ld, hipStream_t st) {
    const unsigned g = (unsigned)((n + 15) / 16);
    hipLaunchKernelGGL(k_symmetrize, dim3(g, g), dim3(16, 16), 0, st, K, n, ld);
}

// Largest |P_xy| of every shell block (X, Y): one thread per block.
__global__ void k_pmax(const double *__restrict__ P, int64_t ld, const int32_t *__restrict__ bfo, int nsh,
                       double *__restrict__ M) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nsh * nsh) return;
    const int X = (int)(t / nsh), Y = (int)(t % nsh);
    double m = 0.0;
    for (int x = bfo[X]; x < bfo[X + 1]; ++x)
        for (int y = bfo[Y]; y < bfo[Y + 1]; ++y) m = fmax(m, fabs(P[(int64_t)x * ld + y]));
    M[t] = m;
}

// Per-block max |P_ij - P_ji| and max |P_ij|.
__global__ void k_asym(const double *P, int64_t n, int64_t ld, double *part) {
    __shared__ double s0[256], s1[256];
    double m0 = 0.0, m1 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n * n; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / n, j = t % n;
        const double a = P[i * ld + j];
        m0 = fmax(m0, fabs(a - P[j * ld + i]));
        m1 = fmax(m1, fabs(a));
    }
    s0[threadIdx.x] = m0;
    s1[threadIdx.x] = m1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + w]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// ----------------------------------------------------- class dispatch ----
#define HFX_FOR_CLASSES(X) \
    X(0000) X(1000) X(1010) X(1100) X(1110) X(1111) X(2000) X(2010) X(2011) X(2020) X(2100) \
    X(2110) X(2111) X(2120) X(2121) X(2200) X(2210) X(2211) X(2220) X(2221) X(2222)
#define DECL(T)                                                                                  \
    void launch_eri_##T(const QuartetArgs &, unsigned, hipStream_t);                            \
    void launch_eval_##T(const PairHdr *, const PrimRec *, const int32_t *, int, int, double,   \
                         const double *, double *, hipStream_t);
HFX_FOR_CLASSES(DECL)
#undef DECL
#define DECLPER(T)                                                          \
    void launch_eriper_##T(const QuartetArgs &, unsigned, hipStream_t);    \
    void launch_eriperS_##T(const QuartetArgs &, unsigned, hipStream_t);
HFX_FOR_CLASSES(DECLPER)
#undef DECLPER
#define DECL32(T)                                                           \
    void launch_eri32_##T(const QuartetArgs &, unsigned, hipStream_t);     \
    void launch_erijk_##T(const QuartetArgs &, unsigned, hipStream_t);     \
    void launch_erijk32_##T(const QuartetArgs &, unsigned, hipStream_t);
HFX_FOR_CLASSES(DECL32)
#undef DECL32
void launch_schwarz_00(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
void launch_schwarz_10(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
void launch_schwarz_11(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
void launch_schwarz_20(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
void launch_schwarz_21(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
void launch_schwarz_22(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *, double *, double *, hipStream_t);
#define PB(T) void launch_primbound_##T(const PairHdr *, PrimRec *, const int32_t *, int, int, double, const double *, hipStream_t);
PB(00) PB(10) PB(11) PB(20) PB(21) PB(22)
#undef PB
typedef void (*primbound_fn)(const PairHdr *, PrimRec *, const int32_t *, int, int, double, const double *, hipStream_t);
static const primbound_fn k_primbound_tab[6] = {launch_primbound_00, launch_primbound_10, launch_primbound_11,
                                                launch_primbound_20, launch_primbound_21, launch_primbound_22};

typedef void (*eri_fn)(const QuartetArgs &, unsigned, hipStream_t);
typedef void (*eval_fn)(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *,
                        double *, hipStream_t);
typedef void (*schwarz_fn)(const PairHdr *, const PrimRec *, const int32_t *, int, int, double, const double *,
                           double *, double *, hipStream_t);

// class index cb(cb+1)/2 + ck, pair classes ss ps pp ds dp dd
static const eri_fn k_eri_tab[21] = {
#define E(T) launch_eri_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
static const eri_fn k_eri32_tab[21] = {
#define E(T) launch_eri32_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
// the same kernels digesting the Coulomb matrix as well
static const eri_fn k_erijk_tab[21] = {
#define E(T) launch_erijk_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
static const eri_fn k_erijk32_tab[21] = {
#define E(T) launch_erijk32_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
// periodic builds: canonical class, wave's pair as the recurrence's bra
// (class of the wave's pair >= the lane's) or lane's pair as the bra
static const eri_fn k_eriper_tab[21] = {
#define E(T) launch_eriper_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
static const eri_fn k_eriperS_tab[21] = {
#define E(T) launch_eriperS_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
static const eval_fn k_eval_tab[21] = {
#define E(T) launch_eval_##T,
    HFX_FOR_CLASSES(E)
#undef E
};
static const schwarz_fn k_schwarz_tab[6] = {launch_schwarz_00, launch_schwarz_10, launch_schwarz_11,
                                            launch_schwarz_20, launch_schwarz_21, launch_schwarz_22};

const int PAIR_L[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

// -------------------------------------------------------------- pairs ----
static void nrm_coefs(const std::vector<hfx_shell> &sh, const double *exps, const double *coefs,
                      std::vector<double> &cn) {
    // Coefficients multiply primitives normalised like x^l exp(-a r^2):
    //   N(a, l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!),
    // then the contraction is scaled to unit self-overlap, using the overlap
    // of two such primitives of the same l on one centre,
    //   [2 sqrt(a b)/(a+b)]^(l + 3/2).
    static const double df[3] = {1.0, 1.0, 3.0};
    for (const hfx_shell &s : sh) {
        for (int i = 0; i < s.nprim; ++i) {
            const double a = exps[s.prim_off + i];
            cn[s.prim_off + i] = coefs[s.prim_off + i] * std::pow(2.0 * a / M_PI, 0.75) *
                                 std::pow(4.0 * a, 0.5 * s.l) / std::sqrt(df[s.l]);
        }
        double ss = 0.0;
        for (int i = 0; i < s.nprim; ++i)
            for (int j = 0; j < s.nprim; ++j) {
                const double a = exps[s.prim_off + i], b = exps[s.prim_off + j];
                ss += coefs[s.prim_off + i] * coefs[s.prim_off + j] *
                      std::pow(2.0 * std::sqrt(a * b) / (a + b), s.l + 1.5);
            }
        const double f = 1.0 / std::sqrt(ss);
        for (int i = 0; i < s.nprim; ++i) cn[s.prim_off + i] *= f;
    }
}

hfx_status check_opts(const hfx_opts *o) {
    if (!o) return fail(HFX_EINVAL, "opts is NULL");
    if (!(o->tau >= 0.0) || !std::isfinite(o->tau)) return fail(HFX_EINVAL, "tau must be finite and >= 0");
    if (o->op != HFX_OP_COULOMB && o->op != HFX_OP_ERFC) return fail(HFX_EINVAL, "unknown operator");
    if (!(o->omega >= 0.0) || !std::isfinite(o->omega)) return fail(HFX_EINVAL, "omega must be finite and >= 0");
    if (o->prec != HFX_PREC_FP64 && o->prec != HFX_PREC_MIXED) return fail(HFX_EINVAL, "unknown precision mode");
    if (o->prec == HFX_PREC_MIXED && !(o->mixed_cut >= 0.0)) return fail(HFX_EINVAL, "mixed_cut must be >= 0");
    if (!(o->prim_tau >= 0.0) || !std::isfinite(o->prim_tau)) return fail(HFX_EINVAL, "prim_tau must be finite and >= 0");
    if (o->flags & ~HFX_FLAG_DENSITY_SCREEN) return fail(HFX_EINVAL, "unknown flag");
    return HFX_OK;
}

int kernel_op(const hfx_opts *o) { return (o->op == HFX_OP_ERFC && o->omega > 0.0) ? 1 : 0; }

// Ket quartets per block of the direct (non-persistent) launches, by total L:
// cheap classes take longer ranges.  HFX_TQ overrides it (tuning).
int quartet_block(int L) {
    static int env = -1;
    if (env < 0) {
        const char *e = std::getenv("HFX_TQ");
        env = (e && *e) ? std::max(64, std::atoi(e)) : 0;
    }
    if (env > 0) return env;
    (void)L;
    return 64;  // measured best for every class on the 256-atom shard
}

// Blocks per direct launch: 2^24 blocks of 64 lanes is 2^30 work-items, a
// quarter of the dispatch packet's 32-bit limit.  HFX_MAX_BLOCKS lowers it
// (the tests use that to run the segmented path on small systems).
long long max_blocks_per_launch() {
    const char *e = std::getenv("HFX_MAX_BLOCKS");
    return (e && *e) ? std::min(1ll << 24, std::max(1ll, std::atoll(e))) : (1ll << 24);
}

}  // namespace hfx

using namespace hfx;

extern "C" const char *hfx_last_error(void) { return g_err.c_str(); }

extern "C" hfx_status hfx_build_shell_pairs(const double *xyz, int32_t natom, const hfx_shell *shells,
                                            int32_t nshell, const double *exps, const double *coefs,
                                            const hfx_opts *o, void *stream, hfx_pairs *out) {
    if (!out) return fail(HFX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!xyz || !shells || !exps || !coefs) return fail(HFX_EINVAL, "NULL input array");
    if (natom < 1 || nshell < 1) return fail(HFX_EINVAL, "natom and nshell must be >= 1");
    if (o) {
        hfx_status s = check_opts(o);
        if (s != HFX_OK) return s;
    }
    for (int i = 0; i < 3 * natom; ++i)
        if (!std::isfinite(xyz[i])) return fail(HFX_EINVAL, "non-finite coordinate");
    int64_t nprim_tot = 0;
    for (int s = 0; s < nshell; ++s) {
        const hfx_shell &h = shells[s];
        if (h.atom < 0 || h.atom >= natom) return fail(HFX_EINVAL, "shell atom index out of range");
        if (h.l < 0) return fail(HFX_EINVAL, "negative l");
        if (h.l > HFX_MAX_L) return fail(HFX_EUNSUPPORTED, "l > 2 is not supported");
        if (h.nprim < 1) return fail(HFX_EINVAL, "nprim < 1");
        if (h.nprim > HFX_MAX_PRIM) return fail(HFX_EUNSUPPORTED, "nprim > HFX_MAX_PRIM");
        if (h.prim_off < 0) return fail(HFX_EINVAL, "negative prim_off");
        nprim_tot = std::max<int64_t>(nprim_tot, (int64_t)h.prim_off + h.nprim);
    }
    for (int s = 0; s < nshell; ++s)
        for (int i = 0; i < shells[s].nprim; ++i) {
            const double a = exps[shells[s].prim_off + i], c = coefs[shells[s].prim_off + i];
            if (!(a > 0.0) || !std::isfinite(a)) return fail(HFX_EINVAL, "exponent must be finite and > 0");
            if (!std::isfinite(c)) return fail(HFX_EINVAL, "non-finite contraction coefficient");
        }
    std::unique_ptr<hfx_pairs_s> P(new hfx_pairs_s());
    P->natom = natom;
    P->nshell = nshell;
    P->stream = (hipStream_t)stream;
    P->sh.assign(shells, shells + nshell);
    P->xyz.assign(xyz, xyz + 3 * natom);
    P->exps.assign(exps, exps + nprim_tot);
    P->cn.assign(nprim_tot, 0.0);
    nrm_coefs(P->sh, exps, coefs, P->cn);
    P->bfo.resize(nshell + 1);
    P->bfo[0] = 0;
    for (int s = 0; s < nshell; ++s) P->bfo[s + 1] = P->bfo[s] + 2 * shells[s].l + 1;
    P->nbf = P->bfo[nshell];
    // n_bf^2 element kernels (fill, symmetrisation) index one work-item per
    // element: the dispatch counts work-items in 32 bits
    if (P->nbf > HFX_MAX_NBF) return fail(HFX_EUNSUPPORTED, "more than 65535 basis functions");
    const int64_t npair = (int64_t)nshell * (nshell + 1) / 2;
    P->npair = npair;
    std::vector<PairHdr> hdr(npair);
    std::vector<int32_t> shA(npair), shB(npair);
    P->pcls.resize(npair);
    int64_t rec = 0;
    for (int I = 0; I < nshell; ++I)
        for (int J = 0; J <= I; ++J) {
            const int64_t id = (int64_t)I * (I + 1) / 2 + J;
            const bool sw = shells[J].l > shells[I].l;
            const int a = sw ? J : I, b = sw ? I : J;
            PairHdr h;
            h.off = (int32_t)rec;
            h.n = shells[a].nprim * shells[b].nprim;
            h.bfA = P->bfo[a];
            h.bfB = P->bfo[b];
            h.shA = a;
            h.shB = b;
            const double *A = xyz + 3 * shells[a].atom, *B = xyz + 3 * shells[b].atom;
            h.ABx = A[0] - B[0];
            h.ABy = A[1] - B[1];
            h.ABz = A[2] - B[2];
            h.diag = (I == J);
            h.id = (int32_t)id;
            hdr[id] = h;
            shA[id] = a;
            shB[id] = b;
            const int la = shells[a].l, lb = shells[b].l;
            P->pcls[id] = (int8_t)(la * (la + 1) / 2 + lb);
            rec += h.n;
        }
    if (rec > INT32_MAX || npair > INT32_MAX) return fail(HFX_EUNSUPPORTED, "too many primitive pairs");
    P->nrec = rec;
    P->hdr_host = hdr;
    for (int64_t id = 0; id < npair; ++id) P->class_ids[P->pcls[id]].push_back((int32_t)id);
    std::vector<ShellDev> shd(nshell);
    for (int s = 0; s < nshell; ++s) {
        shd[s].x = xyz[3 * shells[s].atom];
        shd[s].y = xyz[3 * shells[s].atom + 1];
        shd[s].z = xyz[3 * shells[s].atom + 2];
        shd[s].nprim = shells[s].nprim;
        shd[s].off = shells[s].prim_off;
    }
    hipStream_t st = (hipStream_t)stream;
    // temporaries are stream-ordered (hipFreeAsync does not wait for work of
    // other streams, unlike hipFree, so a pair build never stalls builds that
    // run concurrently on other streams)
    int32_t *d_shA = nullptr, *d_shB = nullptr;
    ShellDev *d_sh = nullptr;
    double *d_ex = nullptr, *d_cn = nullptr;
    auto cleanup = [&]() {
        if (d_shA) hipFreeAsync(d_shA, st);
        if (d_shB) hipFreeAsync(d_shB, st);
        if (d_sh) hipFreeAsync(d_sh, st);
        if (d_ex) hipFreeAsync(d_ex, st);
        if (d_cn) hipFreeAsync(d_cn, st);
    };
#define ALLOC(ptr, bytes)                                                        \
    do {                                                                         \
        if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {                 \
            cleanup();                                                           \
            return fail(HFX_ENOMEM, "device allocation of pair data failed");    \
        }                                                                        \
    } while (0)
#define ALLOC_TMP(ptr, bytes)                                                              \
    do {                                                                                   \
        if (hipMallocAsync((void **)&(ptr), (bytes), st) != hipSuccess) {                  \
            cleanup();                                                                     \
            return fail(HFX_ENOMEM, "device allocation of pair-build temporaries failed");  \
        }                                                                                  \
    } while (0)
    ALLOC(P->d_hdr, npair * sizeof(PairHdr));
    ALLOC(P->d_prim, std::max<int64_t>(rec, 1) * sizeof(PrimRec));
    ALLOC(P->d_Q, npair * sizeof(double));
    ALLOC(P->d_E, npair * sizeof(double));
    ALLOC(P->d_part, 2 * PCHECK_BLOCKS * sizeof(double));
    ALLOC(P->d_count, NCOUNT * sizeof(unsigned long long));
    ALLOC(P->d_class_ids, npair * sizeof(int32_t));
    ALLOC(P->d_bfo, (nshell + 1) * sizeof(int32_t));
    ALLOC_TMP(d_shA, npair * sizeof(int32_t));
    ALLOC_TMP(d_shB, npair * sizeof(int32_t));
    ALLOC_TMP(d_sh, nshell * sizeof(ShellDev));
    ALLOC_TMP(d_ex, std::max<int64_t>(nprim_tot, 1) * sizeof(double));
    ALLOC_TMP(d_cn, std::max<int64_t>(nprim_tot, 1) * sizeof(double));
#undef ALLOC
#undef ALLOC_TMP
    for (auto &ev : P->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            cleanup();
            return fail(HFX_EDEVICE, "hipEventCreate failed");
        }
    P->dev_bytes = npair * (sizeof(PairHdr) + 2 * sizeof(double)) + rec * sizeof(PrimRec);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(P->d_hdr, hdr.data(), npair * sizeof(PairHdr), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_shA, shA.data(), npair * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_shB, shB.data(), npair * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_sh, shd.data(), nshell * sizeof(ShellDev), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ex, P->exps.data(), nprim_tot * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_cn, P->cn.data(), nprim_tot * sizeof(double), hipMemcpyHostToDevice, st);
    {
        // pair ids of every pair class, concatenated in class order (uploaded once)
        std::vector<int32_t> ids;
        ids.reserve(npair);
        for (int c = 0; c < 6; ++c) ids.insert(ids.end(), P->class_ids[c].begin(), P->class_ids[c].end());
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->d_class_ids, ids.data(), npair * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->d_bfo, P->bfo.data(), (nshell + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vector dies here
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pairdata, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, st, P->d_hdr, d_shA,
                           d_shB, d_sh, d_ex, d_cn, npair, P->d_prim);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("pair data: ") + hipGetErrorString(e));
    const double *tab = nullptr;
    const float *tab32 = nullptr;
    hfx_status s = boys_table(&tab, &tab32);
    if (s != HFX_OK) return s;
    P->d_boys = tab;
    P->d_boys32 = tab32;
    *out = P.release();
    return HFX_OK;
}

hfx_pairs_s::~hfx_pairs_s() {
    hipFree(d_hdr);
    hipFree(d_prim);
    hipFree(d_Q);
    hipFree(d_E);
    hipFree(d_prim32);
    drop_lists();
    hipFree(d_count);
    hipFree(d_part);
    hipFree(d_class_ids);
    hipFree(d_bfo);
    hipFree(d_pmax);
    for (auto &e : ev)
        if (e) hipEventDestroy(e);
}

void hfx_pairs_s::drop_lists() {
    for (ClassList *set : {lists, mlists, hlists})
        for (int i = 0; i < 6; ++i) {
            ClassList &c = set[i];
            hipFree(c.d_ids);
            hipFree(c.d_Q);
            hipFree(c.d_grp);
            hipFree(c.d_goff);
            hipFree(c.d_gnp);
            hipFree(c.d_A);
            hipFree(c.d_gA);
            c = ClassList();
        }
    lists_valid = false;
    mlists_valid = false;
    hlists_valid = false;
}

extern "C" void hfx_pairs_destroy(hfx_pairs p) { delete p; }
extern "C" int64_t hfx_pairs_nbf(hfx_pairs p) { return p ? p->nbf : -1; }
extern "C" int64_t hfx_pairs_npair(hfx_pairs p) { return p ? p->npair : -1; }
extern "C" int64_t hfx_pairs_device_bytes(hfx_pairs p) { return p ? p->dev_bytes : -1; }

namespace hfx {

hfx_status compute_bounds(hfx_pairs p, const hfx_opts *o, hipStream_t st) {
    const int op = kernel_op(o);
    const double om2 = op ? o->omega * o->omega : 0.0;
    if (p->have_Q && p->q_op == op && p->q_om2 == om2) return HFX_OK;
    p->drop_lists();
    size_t off = 0;
    for (int c = 0; c < 6; ++c) {
        const auto &ids = p->class_ids[c];
        if (ids.empty()) continue;
        k_schwarz_tab[c](p->d_hdr, p->d_prim, p->d_class_ids + off, (int)ids.size(), op, om2, p->d_boys, p->d_Q,
                         p->d_E, st);
        k_primbound_tab[c](p->d_hdr, p->d_prim, p->d_class_ids + off, (int)ids.size(), op, om2, p->d_boys, st);
        off += ids.size();
    }
    hipError_t e = hipGetLastError();
    p->Q.resize(p->npair);
    p->E.resize(p->npair);
    if (e == hipSuccess) e = hipMemcpyAsync(p->Q.data(), p->d_Q, p->npair * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(p->E.data(), p->d_E, p->npair * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("bounds: ") + hipGetErrorString(e));
    p->have_Q = true;
    p->q_op = op;
    p->q_om2 = om2;
    p->prim32_valid = false;
    return HFX_OK;
}

// FP32 copies of the (sorted) primitive records, made on first mixed build.
hfx_status ensure_prim32(hfx_pairs p, hipStream_t st) {
    if (p->prim32_valid) return HFX_OK;
    if (!p->d_prim32) {
        if (hipMalloc(&p->d_prim32, std::max<int64_t>(p->nrec, 1) * sizeof(PrimRec32)) != hipSuccess)
            return fail(HFX_ENOMEM, "device allocation of FP32 records failed");
        p->dev_bytes += p->nrec * sizeof(PrimRec32);
    }
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((p->nrec + 255) / 256)), dim3(256), 0, st, p->d_prim, p->nrec,
                       p->d_prim32);
    HIPCHK(hipGetLastError());
    p->prim32_valid = true;
    return HFX_OK;
}

// Kept pairs of every class sorted by (primitive-pair count, -Q, id); groups =
// runs of equal primitive-pair count, so every lane of a block loops the same
// number of ket primitive pairs.  Mixed-precision lists are grouped by
// (primitive-pair count, bin of A = E/Q) so that a group's largest A, which
// sets its FP32/FP64 split, is close to that of each of its pairs.
static int amp_bin(double A) { return A <= 4.0 ? 0 : A <= 32.0 ? 1 : A <= 256.0 ? 2 : 3; }

static double amp_of(hfx_pairs p, int32_t id) {
    const double q = p->Q[id];
    return q > 0.0 ? std::max(1.0, p->E[id] / q) : 1.0;
}

const ClassList *class_lists(hfx_pairs p, bool mixed) { return mixed ? p->mlists : p->lists; }

hfx_status build_lists(hfx_pairs p, double tau, bool mixed, hipStream_t st) {
    if (!mixed && p->lists_valid && p->list_tau == tau) return HFX_OK;
    if (mixed && p->mlists_valid && p->mlist_tau == tau) return HFX_OK;
    ClassList *set = mixed ? p->mlists : p->lists;
    for (int c = 0; c < 6; ++c) {
        ClassList &L = set[c];
        hipFree(L.d_ids);
        hipFree(L.d_Q);
        hipFree(L.d_grp);
        hipFree(L.d_goff);
        hipFree(L.d_gnp);
        hipFree(L.d_A);
        hipFree(L.d_gA);
        L = ClassList();
    }
    double qmax = 0.0;
    for (double q : p->Q) qmax = std::max(qmax, q);
    p->qmax = qmax;
    for (int c = 0; c < 6; ++c) {
        std::vector<int32_t> ids;
        for (int32_t id : p->class_ids[c])
            if (p->Q[id] * qmax >= tau) ids.push_back(id);
        auto key = [&](int32_t x) { return p->hdr_host[x].n * 4 + (mixed ? amp_bin(amp_of(p, x)) : 0); };
        std::sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
            const int kx = key(x), ky = key(y);
            if (kx != ky) return kx < ky;
            if (p->Q[x] != p->Q[y]) return p->Q[x] > p->Q[y];
            return x < y;
        });
        ClassList &L = set[c];
        L.n = (int)ids.size();
        if (!L.n) continue;
        std::vector<double> q(L.n), A, gA;
        std::vector<int32_t> grp(L.n);
        std::vector<int> gkey;
        L.goff.clear();
        L.gnp.clear();
        for (int i = 0; i < L.n; ++i) {
            q[i] = p->Q[ids[i]];
            const int k = key(ids[i]);
            if (gkey.empty() || gkey.back() != k) {
                gkey.push_back(k);
                L.gnp.push_back(p->hdr_host[ids[i]].n);
                L.goff.push_back(i);
                if (mixed) gA.push_back(1.0);
            }
            grp[i] = (int)L.gnp.size() - 1;
            if (mixed) {
                A.push_back(amp_of(p, ids[i]));
                gA.back() = std::max(gA.back(), A.back());
            }
        }
        L.goff.push_back(L.n);
        L.ngrp = (int)L.gnp.size();
        HIPCHK(hipMalloc(&L.d_ids, L.n * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_Q, L.n * sizeof(double)));
        HIPCHK(hipMalloc(&L.d_grp, L.n * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_goff, L.goff.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_gnp, L.gnp.size() * sizeof(int32_t)));
        HIPCHK(hipMemcpyAsync(L.d_ids, ids.data(), L.n * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_Q, q.data(), L.n * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_grp, grp.data(), L.n * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_goff, L.goff.data(), L.goff.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_gnp, L.gnp.data(), L.gnp.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        if (mixed) {
            HIPCHK(hipMalloc(&L.d_A, L.n * sizeof(double)));
            HIPCHK(hipMalloc(&L.d_gA, gA.size() * sizeof(double)));
            HIPCHK(hipMemcpyAsync(L.d_A, A.data(), L.n * sizeof(double), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(L.d_gA, gA.data(), gA.size() * sizeof(double), hipMemcpyHostToDevice, st));
        }
        // the host vectors must outlive the copies
        HIPCHK(hipStreamSynchronize(st));
        L.h_ids = std::move(ids);
        L.h_Q = std::move(q);
        L.h_grp = std::move(grp);
    }
    HIPCHK(hipStreamSynchronize(st));
    if (mixed) {
        p->mlists_valid = true;
        p->mlist_tau = tau;
    } else {
        p->lists_valid = true;
        p->list_tau = tau;
    }
    return HFX_OK;
}

// part: device, 2 * PCHECK_BLOCKS doubles (every block writes its two
// entries, so nothing needs clearing).
hfx_status check_P(const double *P, int64_t n, int64_t ld, hipStream_t st, double *part) {
    const int nb = (int)std::min<int64_t>(PCHECK_BLOCKS, (n * n + 255) / 256);
    hipLaunchKernelGGL(k_asym, dim3(nb), dim3(256), 0, st, P, n, ld, part);
    double h[2 * PCHECK_BLOCKS];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, part, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("P check: ") + hipGetErrorString(e));
    double asym = 0.0, mx = 0.0;
    for (int b = 0; b < nb; ++b) {
        asym = std::max(asym, h[2 * b]);
        mx = std::max(mx, h[2 * b + 1]);
    }
    if (!(asym <= 1e-12 * mx)) return fail(HFX_EASYM, "P is not symmetric within 1e-12 max|P|");
    return HFX_OK;
}

// Shell-block maxima of |P| for density screening (per build: P changes
// between calls).  The nshell^2 array is allocated on the handle's first
// density-screened build; may_allocate = false refuses to make it.
hfx_status shell_pmax(hfx_pairs p, const double *P, int64_t ld, bool may_allocate, hipStream_t st) {
    const int64_t n2 = (int64_t)p->nshell * p->nshell;
    if (!p->d_pmax) {
        if (!may_allocate)
            return fail(HFX_EINVAL, "density-screening workspace is not resident in the handle "
                                    "(run hfx_build_K once with the same options first)");
        if (hipMalloc(&p->d_pmax, n2 * sizeof(double)) != hipSuccess)
            return fail(HFX_ENOMEM, "device allocation of the |P| block maxima failed");
        p->dev_bytes += n2 * sizeof(double);
    }
    hipLaunchKernelGGL(k_pmax, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, P, ld, p->d_bfo, p->nshell,
                       p->d_pmax);
    HIPCHK(hipGetLastError());
    return HFX_OK;
}

int density_mode(const hfx_opts *o, bool coulomb) {
    return (o->flags & HFX_FLAG_DENSITY_SCREEN) ? (coulomb ? 2 : 1) : 0;
}

// Ket candidates per block under density screening: longer than the plain
// blocks so that the survivors fill whole 64-lane tiles.  HFX_TQ_DENS
// overrides it (tuning).
static int quartet_block_dens() {
    static int env = -1;
    if (env < 0) {
        const char *e = std::getenv("HFX_TQ_DENS");
        env = (e && *e) ? std::max(64, std::atoi(e)) : 0;
    }
    return env > 0 ? env : 512;
}

const double *model_vrr();
const double *model_post();
double model_prim_overhead(int op, int L);

// Launch the quartet kernels of every class pair; K must already be zero.
hfx_status launch_classes(hfx_pairs p, const double *P, double *K, double *J, int64_t ld, const hfx_opts *o,
                          hipStream_t st, unsigned long long *count, int shard, int nshards,
                          hipEvent_t *ev) {
    const int op = kernel_op(o);
    const bool mixed = (o->prec == HFX_PREC_MIXED);
    const double inf = HUGE_VAL;
    const ClassList *lists = class_lists(p, mixed);
    for (int cb = 0; cb < 6; ++cb)
        for (int ck = 0; ck <= cb; ++ck) {
            const ClassList &B = lists[cb], &Kl = lists[ck];
            const int ci = cb * (cb + 1) / 2 + ck;
            if (ev) HIPCHK(hipEventRecord(ev[ci], st));
            if (!B.n || !Kl.n || shard >= B.n) continue;
            QuartetArgs a{};
            a.hdr = p->d_hdr;
            a.prim = p->d_prim;
            a.prim32 = p->d_prim32;
            a.bra_ids = B.d_ids;
            a.bra_Q = B.d_Q;
            a.bra_grp = B.d_grp;
            a.n_bra = B.n;
            a.bra_first = shard;
            a.bra_stride = nshards;
            a.ket_ids = Kl.d_ids;
            a.ket_Q = Kl.d_Q;
            a.ket_goff = Kl.d_goff;
            a.ket_gnp = Kl.d_gnp;
            a.n_kgrp = Kl.ngrp;
            a.same = (cb == ck);
            a.op = op;
            a.om2 = op ? o->omega * o->omega : 0.0;
            a.prim_tau = o->prim_tau;
            a.boys = p->d_boys;
            a.boys32 = p->d_boys32;
            a.P = P;
            a.K = K;
            a.J = J;
            a.ld = ld;
            // ket ranges are cut into sub-ranges of tq quartets so that no block
            // runs much longer than the others (quartet-block size per class)
            const int L = PAIR_L[cb][0] + PAIR_L[cb][1] + PAIR_L[ck][0] + PAIR_L[ck][1];
            int gmax = 1;
            for (size_t gi = 0; gi + 1 < Kl.goff.size(); ++gi) gmax = std::max(gmax, Kl.goff[gi + 1] - Kl.goff[gi]);
            a.dens = density_mode(o, J != nullptr);
            a.nsh = p->nshell;
            a.pmax = p->d_pmax;
            a.tq = a.dens ? quartet_block_dens() : quartet_block(L);
            a.nsub = (gmax + a.tq - 1) / a.tq;
            const int64_t nblk = (int64_t)((B.n - shard + nshards - 1) / nshards) * Kl.ngrp * a.nsub;
            if (nblk > (int64_t)UINT32_MAX) return fail(HFX_EUNSUPPORTED, "grid too large");
            a.om = op ? o->omega : 0.0;
            // FP64: Q_p Q_q >= tau, and in mixed mode E_p E_q >= cut as well
            // (split per block in ket_cut)
            a.tau = o->tau;
            a.tau_hi = inf;
            a.part = mixed ? 1 : 0;
            a.mixed_cut = o->mixed_cut;
            a.bra_A = B.d_A;
            a.ket_gA = Kl.d_gA;
            a.count = count ? count + 4 * ci : nullptr;
            (J ? k_erijk_tab : k_eri_tab)[ci](a, (unsigned)nblk, st);
            HIPCHK(hipGetLastError());
            if (mixed && o->mixed_cut > 0.0) {
                // FP32: Q_p Q_q >= tau and E_p E_q < cut
                a.part = 2;
                a.count = count ? count + 4 * ci + 2 : nullptr;
                (J ? k_erijk32_tab : k_eri32_tab)[ci](a, (unsigned)nblk, st);
                HIPCHK(hipGetLastError());
            }
        }
    if (ev) HIPCHK(hipEventRecord(ev[HFX_NCLASS], st));
    return HFX_OK;
}

}  // namespace hfx

extern "C" hfx_status hfx_schwarz_bounds(hfx_pairs p, const hfx_opts *o, double *q_host, void *stream) {
    if (!p) return fail(HFX_EINVAL, "pairs is NULL");
    hfx_status s = check_opts(o);
    if (s != HFX_OK) return s;
    s = compute_bounds(p, o, (hipStream_t)stream);
    if (s != HFX_OK) return s;
    if (q_host) std::memcpy(q_host, p->Q.data(), p->npair * sizeof(double));
    return HFX_OK;
}

static bool overlaps(const double *x, const double *y, int64_t n, int64_t ld) {
    return x < y + (n - 1) * ld + n && y < x + (n - 1) * ld + n;
}

hfx_status hfx::build_K_impl(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                             const hfx_opts *o, int shard, int nshards, void *stream, hfx_stats *st_out,
                             double *J_dev, const Workspace *ws_in) {
    auto t0 = std::chrono::steady_clock::now();
    if (!p) return fail(HFX_EINVAL, "pairs is NULL");
    if (!P_dev || !K_dev) return fail(HFX_EINVAL, "P or K is NULL");
    if (nshards < 1 || shard < 0 || shard >= nshards) return fail(HFX_EINVAL, "shard not in [0, nshards)");
    hfx_status s = check_opts(o);
    if (s != HFX_OK) return s;
    const int64_t n = p->nbf;
    if (ld < n) return fail(HFX_EINVAL, "ld < n_bf");
    if (overlaps(K_dev, P_dev, n, ld)) return fail(HFX_EINVAL, "K aliases P");
    if (J_dev && (overlaps(J_dev, P_dev, n, ld) || overlaps(J_dev, K_dev, n, ld)))
        return fail(HFX_EINVAL, "J aliases P or K");
    hipStream_t st = (hipStream_t)stream;
    const Workspace ws = ws_in ? *ws_in : Workspace{p->d_part, p->d_count};
    if (ws_in) {
        // nothing may be allocated: the handle must hold what these options need
        const int op = kernel_op(o);
        const double om2 = op ? o->omega * o->omega : 0.0;
        if (!(p->have_Q && p->q_op == op && p->q_om2 == om2))
            return fail(HFX_EINVAL, "Schwarz bounds for this kernel are not resident in the handle "
                                    "(run hfx_build_K once with the same options first)");
        const bool mx = o->prec == HFX_PREC_MIXED;
        if (!(mx ? (p->mlists_valid && p->mlist_tau == o->tau) : (p->lists_valid && p->list_tau == o->tau)))
            return fail(HFX_EINVAL, "screening lists for this tau are not resident in the handle "
                                    "(run hfx_build_K once with the same options first)");
        if (o->prec == HFX_PREC_MIXED && !p->prim32_valid)
            return fail(HFX_EINVAL, "FP32 records are not resident in the handle "
                                    "(run hfx_build_K once in mixed precision first)");
    }
    s = check_P(P_dev, n, ld, st, ws.part);
    if (s != HFX_OK) return s;
    if (o->flags & HFX_FLAG_DENSITY_SCREEN) {
        s = shell_pmax(p, P_dev, ld, ws_in == nullptr, st);
        if (s != HFX_OK) return s;
    }
    if (!ws_in) {
        s = compute_bounds(p, o, st);
        if (s != HFX_OK) return s;
        s = build_lists(p, o->tau, o->prec == HFX_PREC_MIXED, st);
        if (s != HFX_OK) return s;
        if (o->prec == HFX_PREC_MIXED) {
            s = ensure_prim32(p, st);
            if (s != HFX_OK) return s;
        }
    }
    unsigned long long *cnt = st_out ? ws.count : nullptr;
    if (cnt) hipLaunchKernelGGL(k_fill_u64, dim3(2), dim3(64), 0, st, cnt, NCOUNT);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, K_dev, n, ld);
    if (J_dev) hipLaunchKernelGGL(k_fill, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, J_dev, n, ld);
    HIPCHK(hipGetLastError());
    hipEvent_t *ev = p->ev;  // created with the handle (one build per handle at a time)
    s = launch_classes(p, P_dev, K_dev, J_dev, ld, o, st, cnt, shard, nshards, st_out ? ev : nullptr);
    if (s != HFX_OK) return s;
    const unsigned g = (unsigned)((n + 15) / 16);
    hipLaunchKernelGGL(k_symmetrize, dim3(g, g), dim3(16, 16), 0, st, K_dev, n, ld);
    if (J_dev) hipLaunchKernelGGL(k_symmetrize, dim3(g, g), dim3(16, 16), 0, st, J_dev, n, ld);
    HIPCHK(hipGetLastError());
    if (st_out) {
        unsigned long long h[NCOUNT];
        HIPCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::memset(st_out, 0, sizeof(*st_out));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[HFX_NCLASS]));
        st_out->device_s = ms * 1e-3;
        const double *mv = model_vrr(), *mp = model_post();
        for (int c = 0; c < HFX_NCLASS; ++c) {
            int cb = 0;
            while ((cb + 1) * (cb + 2) / 2 <= c) ++cb;
            const int ck = c - cb * (cb + 1) / 2;
            const int L = PAIR_L[cb][0] + PAIR_L[cb][1] + PAIR_L[ck][0] + PAIR_L[ck][1];
            float cm = 0.f;
            HIPCHK(hipEventElapsedTime(&cm, ev[c], ev[c + 1]));
            st_out->class_device_s[c] = cm * 1e-3;
            const double nq = (double)(h[4 * c] + h[4 * c + 2]), npq = (double)(h[4 * c + 1] + h[4 * c + 3]);
            st_out->class_quartets[c] = (int64_t)(h[4 * c] + h[4 * c + 2]);
            // the Coulomb digestion adds two multiply-adds per spherical value
            const double pj = J_dev ? 4.0 * (2 * PAIR_L[cb][0] + 1) * (2 * PAIR_L[cb][1] + 1) *
                                          (2 * PAIR_L[ck][0] + 1) * (2 * PAIR_L[ck][1] + 1)
                                    : 0.0;
            st_out->class_flops[c] = (mv[c] + model_prim_overhead(kernel_op(o), L)) * npq + (mp[c] + pj) * nq;
            st_out->quartets += st_out->class_quartets[c];
            st_out->quartets_fp32 += (int64_t)h[4 * c + 2];
            st_out->prim_quartets += (int64_t)npq;
            st_out->flops += st_out->class_flops[c];
        }
        st_out->latency_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return HFX_OK;
}

extern "C" hfx_status hfx_build_K(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                                  const hfx_opts *o, void *stream, hfx_stats *st_out) {
    return build_K_impl(p, P_dev, K_dev, ld, o, 0, 1, stream, st_out);
}

extern "C" hfx_status hfx_build_JK(hfx_pairs p, const double *P_dev, double *J_dev, double *K_dev, int64_t ld,
                                   const hfx_opts *o, void *stream, hfx_stats *st_out) {
    if (!J_dev) return fail(HFX_EINVAL, "J is NULL");
    return build_K_impl(p, P_dev, K_dev, ld, o, 0, 1, stream, st_out, J_dev);
}

extern "C" hfx_status hfx_build_JK_shard(hfx_pairs p, const double *P_dev, double *J_dev, double *K_dev,
                                         int64_t ld, const hfx_opts *o, int32_t shard, int32_t nshards,
                                         void *stream, hfx_stats *st_out) {
    if (!J_dev) return fail(HFX_EINVAL, "J is NULL");
    return build_K_impl(p, P_dev, K_dev, ld, o, shard, nshards, stream, st_out, J_dev);
}

extern "C" hfx_status hfx_build_K_shard(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                                        const hfx_opts *o, int32_t shard, int32_t nshards, void *stream,
                                        hfx_stats *st_out) {
    return build_K_impl(p, P_dev, K_dev, ld, o, shard, nshards, stream, st_out);
}

extern "C" hfx_status hfx_eval_quartets(hfx_pairs p, const hfx_opts *o, int64_t n, const int32_t *q,
                                        double *out, void *stream) {
    if (!p || !q || !out || n < 0) return fail(HFX_EINVAL, "bad arguments");
    hfx_status s = check_opts(o);
    if (s != HFX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int op = kernel_op(o);
    const double om2 = op ? o->omega * o->omega : 0.0;
    // bucket the quartets by class; canonical pair = (max, min) shell index
    struct Item { int64_t idx; int32_t bra, ket; bool swp_bk; };
    std::vector<std::vector<Item>> by(HFX_NCLASS);
    std::vector<int64_t> outoff(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        int I = q[4 * i], J = q[4 * i + 1], Kk = q[4 * i + 2], L = q[4 * i + 3];
        for (int x : {I, J, Kk, L})
            if (x < 0 || x >= p->nshell) return fail(HFX_EINVAL, "shell index out of range");
        const int64_t pb = (int64_t)std::max(I, J) * (std::max(I, J) + 1) / 2 + std::min(I, J);
        const int64_t pk = (int64_t)std::max(Kk, L) * (std::max(Kk, L) + 1) / 2 + std::min(Kk, L);
        int cb = p->pcls[pb], ck = p->pcls[pk];
        Item it{i, (int32_t)pb, (int32_t)pk, false};
        if (cb < ck) {
            std::swap(it.bra, it.ket);
            std::swap(cb, ck);
            it.swp_bk = true;
        }
        by[cb * (cb + 1) / 2 + ck].push_back(it);
        outoff[i + 1] = outoff[i] + (2 * p->sh[I].l + 1) * (2 * p->sh[J].l + 1) * (2 * p->sh[Kk].l + 1) *
                                        (2 * p->sh[L].l + 1);
    }
    for (int c = 0; c < HFX_NCLASS; ++c) {
        if (by[c].empty()) continue;
        int cb = 0;
        while ((cb + 1) * (cb + 2) / 2 <= c) ++cb;
        const int ck = c - cb * (cb + 1) / 2;
        const int na = 2 * PAIR_L[cb][0] + 1, nb = 2 * PAIR_L[cb][1] + 1, nc = 2 * PAIR_L[ck][0] + 1,
                  nd = 2 * PAIR_L[ck][1] + 1;
        const int nout = na * nb * nc * nd;
        const int m = (int)by[c].size();
        std::vector<int32_t> bk(2 * m);
        for (int i = 0; i < m; ++i) {
            bk[2 * i] = by[c][i].bra;
            bk[2 * i + 1] = by[c][i].ket;
        }
        int32_t *d_bk = nullptr;
        double *d_out = nullptr;
        HIPCHK(hipMallocAsync((void **)&d_bk, bk.size() * sizeof(int32_t), st));
        if (hipMallocAsync((void **)&d_out, (size_t)m * nout * sizeof(double), st) != hipSuccess) {
            hipFreeAsync(d_bk, st);
            return fail(HFX_ENOMEM, "eval: device allocation failed");
        }
        HIPCHK(hipMemcpyAsync(d_bk, bk.data(), bk.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        k_eval_tab[c](p->d_hdr, p->d_prim, d_bk, m, op, om2, p->d_boys, d_out, st);
        std::vector<double> h((size_t)m * nout);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
        hipFreeAsync(d_bk, st);
        hipFreeAsync(d_out, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("eval: ") + hipGetErrorString(e));
        // canonical block [A][B][C][D] -> caller order [I][J][K][L]
        for (int i = 0; i < m; ++i) {
            const Item &it = by[c][i];
            const int64_t qi = it.idx;
            int I = q[4 * qi], J = q[4 * qi + 1], Kk = q[4 * qi + 2], L = q[4 * qi + 3];
            if (it.swp_bk) {
                std::swap(I, Kk);
                std::swap(J, L);
            }
            // canonical shells of bra: A = higher l (ties: larger index)
            const PairHdr &hb = p->hdr_host[it.bra], &hk = p->hdr_host[it.ket];
            const bool sab = (p->bfo[I] != hb.bfA);
            const bool scd = (p->bfo[Kk] != hk.bfA);
            const int nI = 2 * p->sh[I].l + 1, nJ = 2 * p->sh[J].l + 1, nK = 2 * p->sh[Kk].l + 1,
                      nL = 2 * p->sh[L].l + 1;
            double *dst = out + outoff[qi];
            for (int a = 0; a < nI; ++a)
                for (int b = 0; b < nJ; ++b)
                    for (int cc = 0; cc < nK; ++cc)
                        for (int d = 0; d < nL; ++d) {
                            const int A = sab ? b : a, B = sab ? a : b, C = scd ? d : cc, D = scd ? cc : d;
                            const double v = h[(size_t)i * nout + ((A * nb + B) * nc + C) * nd + D];
                            if (!it.swp_bk)
                                dst[((a * nJ + b) * nK + cc) * nL + d] = v;
                            else  // caller's (I J) is our ket: output index order is (K L I J) of ours
                                dst[((cc * nL + d) * nI + a) * nJ + b] = v;
                        }
        }
    }
    return HFX_OK;
}

// ------------------------------------------------------------- periodic ----
namespace hfx {

// Kept pairs with at least one shell in the home cell (shell index < nhome),
// per pair class, in the layout of the other lists (groups of equal
// primitive-pair count, Q descending): the bra side of periodic builds.
static hfx_status build_home_lists(hfx_pairs p, double tau, int nhome, hipStream_t st) {
    if (p->hlists_valid && p->hlist_tau == tau && p->hlist_nhome == nhome) return HFX_OK;
    for (int c = 0; c < 6; ++c) {
        ClassList &L = p->hlists[c];
        hipFree(L.d_ids);
        hipFree(L.d_Q);
        hipFree(L.d_grp);
        hipFree(L.d_goff);
        hipFree(L.d_gnp);
        L = ClassList();
    }
    double qmax = 0.0;
    for (double q : p->Q) qmax = std::max(qmax, q);
    for (int c = 0; c < 6; ++c) {
        std::vector<int32_t> ids;
        for (int32_t id : p->class_ids[c]) {
            const PairHdr &h = p->hdr_host[id];
            if ((h.shA < nhome || h.shB < nhome) && p->Q[id] * qmax >= tau) ids.push_back(id);
        }
        std::sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
            const int nx = p->hdr_host[x].n, ny = p->hdr_host[y].n;
            if (nx != ny) return nx < ny;
            if (p->Q[x] != p->Q[y]) return p->Q[x] > p->Q[y];
            return x < y;
        });
        ClassList &L = p->hlists[c];
        L.n = (int)ids.size();
        if (!L.n) continue;
        std::vector<double> q(L.n);
        std::vector<int32_t> grp(L.n);
        for (int i = 0; i < L.n; ++i) {
            q[i] = p->Q[ids[i]];
            const int np = p->hdr_host[ids[i]].n;
            if (L.gnp.empty() || L.gnp.back() != np) {
                L.gnp.push_back(np);
                L.goff.push_back(i);
            }
            grp[i] = (int)L.gnp.size() - 1;
        }
        L.goff.push_back(L.n);
        L.ngrp = (int)L.gnp.size();
        HIPCHK(hipMalloc(&L.d_ids, L.n * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_Q, L.n * sizeof(double)));
        HIPCHK(hipMalloc(&L.d_grp, L.n * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_goff, L.goff.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc(&L.d_gnp, L.gnp.size() * sizeof(int32_t)));
        HIPCHK(hipMemcpyAsync(L.d_ids, ids.data(), L.n * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_Q, q.data(), L.n * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_grp, grp.data(), L.n * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_goff, L.goff.data(), L.goff.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.d_gnp, L.gnp.data(), L.gnp.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // the host vectors die here
        L.h_ids = std::move(ids);
        L.h_Q = std::move(q);
        L.h_grp = std::move(grp);
    }
    p->hlists_valid = true;
    p->hlist_tau = tau;
    p->hlist_nhome = nhome;
    return HFX_OK;
}

}  // namespace hfx

extern "C" hfx_status hfx_build_K_periodic(hfx_pairs p, int32_t nhome_shell, const double *P_dev, int64_t ldP,
                                           double *K_dev, int64_t ldK, const hfx_opts *o, void *stream,
                                           hfx_stats *st_out) {
    auto t0 = std::chrono::steady_clock::now();
    if (!p) return fail(HFX_EINVAL, "pairs is NULL");
    if (!P_dev || !K_dev) return fail(HFX_EINVAL, "P or K is NULL");
    hfx_status s = check_opts(o);
    if (s != HFX_OK) return s;
    if (o->prec != HFX_PREC_FP64) return fail(HFX_EUNSUPPORTED, "periodic builds are FP64 only");
    if (o->flags) return fail(HFX_EUNSUPPORTED, "periodic builds take no flags");
    if (nhome_shell < 1 || nhome_shell > p->nshell) return fail(HFX_EINVAL, "nhome_shell not in [1, nshell]");
    const int64_t n = p->nbf, nh = p->bfo[nhome_shell];
    if (ldP < n || ldK < n) return fail(HFX_EINVAL, "ldP or ldK < n_bf");
    if (K_dev < P_dev + (n - 1) * ldP + n && P_dev < K_dev + (nh - 1) * ldK + n)
        return fail(HFX_EINVAL, "K aliases P");
    hipStream_t st = (hipStream_t)stream;
    s = check_P(P_dev, n, ldP, st, p->d_part);
    if (s != HFX_OK) return s;
    s = compute_bounds(p, o, st);
    if (s != HFX_OK) return s;
    s = build_lists(p, o->tau, false, st);
    if (s != HFX_OK) return s;
    s = build_home_lists(p, o->tau, nhome_shell, st);
    if (s != HFX_OK) return s;
    unsigned long long *cnt = st_out ? p->d_count : nullptr;
    if (cnt) hipLaunchKernelGGL(k_fill_u64, dim3(2), dim3(64), 0, st, cnt, NCOUNT);
    hipLaunchKernelGGL(k_fill_rect, dim3((unsigned)((nh * n + 255) / 256)), dim3(256), 0, st, K_dev, nh, n, ldK);
    HIPCHK(hipGetLastError());
    if (st_out) HIPCHK(hipEventRecord(p->ev[0], st));
    const int op = kernel_op(o);
    for (int cb = 0; cb < 6; ++cb)
        for (int ck = 0; ck < 6; ++ck) {
            const ClassList &B = p->hlists[cb], &Kl = p->lists[ck];
            if (!B.n || !Kl.n) continue;
            const int hi = std::max(cb, ck), lo = std::min(cb, ck), ci = hi * (hi + 1) / 2 + lo;
            QuartetArgs a{};
            a.hdr = p->d_hdr;
            a.prim = p->d_prim;
            a.bra_ids = B.d_ids;
            a.bra_Q = B.d_Q;
            a.bra_grp = B.d_grp;
            a.n_bra = B.n;
            a.bra_first = 0;
            a.bra_stride = 1;
            a.ket_ids = Kl.d_ids;
            a.ket_Q = Kl.d_Q;
            a.ket_goff = Kl.d_goff;
            a.ket_gnp = Kl.d_gnp;
            a.n_kgrp = Kl.ngrp;
            a.same = 0;
            a.op = op;
            a.om2 = op ? o->omega * o->omega : 0.0;
            a.om = op ? o->omega : 0.0;
            a.prim_tau = o->prim_tau;
            a.boys = p->d_boys;
            a.P = P_dev;
            a.K = K_dev;
            a.ld = ldP;
            a.ldK = ldK;
            a.nhome = nhome_shell;
            a.tau = o->tau;
            a.tau_hi = HUGE_VAL;
            a.count = cnt ? cnt + 4 * ci : nullptr;
            int gmax = 1;
            for (size_t gi = 0; gi + 1 < Kl.goff.size(); ++gi) gmax = std::max(gmax, Kl.goff[gi + 1] - Kl.goff[gi]);
            const int L = PAIR_L[cb][0] + PAIR_L[cb][1] + PAIR_L[ck][0] + PAIR_L[ck][1];
            a.tq = quartet_block(L);
            a.nsub = (gmax + a.tq - 1) / a.tq;
            const int64_t nblk = (int64_t)B.n * Kl.ngrp * a.nsub;
            if (nblk > (int64_t)UINT32_MAX) return fail(HFX_EUNSUPPORTED, "grid too large");
            // the class kernel of (hi|lo): the wave's pair is its bra when
            // its class is the higher one, else the lane's pair is
            (cb >= ck ? k_eriper_tab : k_eriperS_tab)[ci](a, (unsigned)nblk, st);
            HIPCHK(hipGetLastError());
        }
    if (st_out) HIPCHK(hipEventRecord(p->ev[1], st));
    if (st_out) {
        unsigned long long h[NCOUNT];
        HIPCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::memset(st_out, 0, sizeof(*st_out));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
        st_out->device_s = ms * 1e-3;
        const double *mv = model_vrr(), *mp = model_post();
        for (int c = 0; c < HFX_NCLASS; ++c) {
            int cb = 0;
            while ((cb + 1) * (cb + 2) / 2 <= c) ++cb;
            const int ck = c - cb * (cb + 1) / 2;
            const int L = PAIR_L[cb][0] + PAIR_L[cb][1] + PAIR_L[ck][0] + PAIR_L[ck][1];
            const double nq = (double)h[4 * c], npq = (double)h[4 * c + 1];
            st_out->class_quartets[c] = (int64_t)h[4 * c];
            st_out->class_flops[c] = (mv[c] + model_prim_overhead(kernel_op(o), L)) * npq + mp[c] * nq;
            st_out->quartets += st_out->class_quartets[c];
            st_out->prim_quartets += (int64_t)npq;
            st_out->flops += st_out->class_flops[c];
        }
        st_out->latency_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return HFX_OK;
}
