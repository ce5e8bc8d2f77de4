// Device-side building blocks of the screened exchange build (gfx950).
//
// Data layout in HBM
//   PairHdr  one per shell pair (I >= J, A = the shell of higher l): offset
//            and count of its primitive-pair records, function offsets of A
//            and B, A-B, and whether I == J.
//   PrimRec  one per primitive pair (a, b): zeta = a + b, 1/(2 zeta), the
//            Gaussian product centre P, P - A and the scaled prefactor
//            sqrt(2) pi^(5/4) c_a c_b exp(-a b |AB|^2 / zeta) / zeta, so that
//            the [00|00] prefactor 2 pi^(5/2)/(zeta eta sqrt(zeta+eta)) K_AB
//            K_CD is the product of two records over sqrt(zeta + eta); and the
//            primitive pair's own Schwarz factor B, so that every primitive
//            quartet contributes at most B_ab B_cd to any integral.  The
//            records of a pair are sorted by B, largest first.
//   Boys     table T_L[i][k] = F_(L+k)(i h) / k! for k < 7 and T_L[i][7] =
//            exp(-i h), h = 1/32, i <= 1152: one 64-byte row per grid point
//            and L.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfx {

struct PairHdr {
    int32_t off;   // first PrimRec
    int32_t n;     // number of PrimRecs
    int32_t bfA;   // first spherical function of shell A
    int32_t bfB;   // first spherical function of shell B
    int32_t shA;   // shell index of A
    int32_t shB;   // shell index of B
    double ABx, ABy, ABz;
    int32_t diag;  // I == J
    int32_t id;    // global pair id
};

struct PrimRec {
    double z, i2z, Px, Py, Pz, PAx, PAy, PAz, K;
    double B;  // Schwarz factor of this primitive pair alone (records of a pair sorted by B, descending)
};

// FP32 copy of a record, used for quartets evaluated in FP32 (mixed mode).
// The product centre P stays FP64: P - Q is formed in FP64 and then rounded,
// so its error is relative to |P - Q|, not to the distance of P from the
// coordinate origin.
struct PrimRec32 {
    double Px, Py, Pz;
    float z, i2z, PAx, PAy, PAz, K, B, pad;
};

// Read-only views in the constant address space (scalar loads when uniform).
typedef __attribute__((address_space(4))) const PrimRec CPrimRec;
typedef __attribute__((address_space(4))) const PrimRec32 CPrimRec32;

__device__ __forceinline__ PrimRec load_rec(CPrimRec *r) {
    PrimRec x;
    x.z = r->z; x.i2z = r->i2z; x.Px = r->Px; x.Py = r->Py; x.Pz = r->Pz;
    x.PAx = r->PAx; x.PAy = r->PAy; x.PAz = r->PAz; x.K = r->K; x.B = r->B;
    return x;
}
__device__ __forceinline__ PrimRec32 load_rec(CPrimRec32 *r) {
    PrimRec32 x;
    x.Px = r->Px; x.Py = r->Py; x.Pz = r->Pz; x.z = r->z; x.i2z = r->i2z;
    x.PAx = r->PAx; x.PAy = r->PAy; x.PAz = r->PAz; x.K = r->K; x.B = r->B; x.pad = 0.0f;
    return x;
}

constexpr int MAX_WPB = 4;              // most waves per workgroup of a quartet kernel
constexpr int BOYS_NROW = 1153;         // grid points 0 .. 36 step 1/32
constexpr double BOYS_H = 1.0 / 32.0;
constexpr double BOYS_INVH = 32.0;
constexpr double BOYS_TMAX = 36.0;
constexpr int BOYS_NTAY = 8;            // doubles per row: 7 Taylor terms and exp(-x_i)
constexpr int BOYS_LMAX = 8;            // highest L = 4 * lmax
constexpr int BOYS_TAB_SIZE = (BOYS_LMAX + 1) * BOYS_NROW * BOYS_NTAY;

// F_m(x), m = 0..L.  x < 36: Taylor expansion of F_L around the nearest grid
// point x_i (|u| = |x_i - x| <= 1/64, seven terms: truncation below 5e-17
// relative), e^-x = e^-x_i e^u with e^u to sixth order (same bound), then the
// downward recursion F_m = (2x F_(m+1) + e^-x) / (2m+1).  x >= 36: F_0 =
// sqrt(pi/(4x)) (erf(sqrt x) equals 1 to 2e-17 there), then the upward
// recursion F_(m+1) = ((2m+1) F_m - e^-x) / (2x), stable for x > L; there e^-x
// weighs at most 6e-9 of (2m+1) F_m (m <= 8), so the FP32 exponential (relative
// error ~2e-7) changes F_m by ~1e-15 relative at most.
template <int L>
__device__ __forceinline__ void boys(double x, const double *__restrict__ tab, double *F) {
    if (x < BOYS_TMAX) {
        const int i = __double2int_rn(x * BOYS_INVH);
        const double u = i * BOYS_H - x;
        const double *r = tab + ((size_t)L * BOYS_NROW + i) * BOYS_NTAY;
        const double4 lo = *reinterpret_cast<const double4 *>(r);
        const double4 hi = *reinterpret_cast<const double4 *>(r + 4);
        double f = hi.z;
        f = fma(f, u, hi.y);
        f = fma(f, u, hi.x);
        f = fma(f, u, lo.w);
        f = fma(f, u, lo.z);
        f = fma(f, u, lo.y);
        f = fma(f, u, lo.x);
        F[L] = f;
        double e = fma(u, 1.0 / 720.0, 1.0 / 120.0);
        e = fma(e, u, 1.0 / 24.0);
        e = fma(e, u, 1.0 / 6.0);
        e = fma(e, u, 0.5);
        e = fma(e, u, 1.0);
        e = fma(e, u, 1.0);
        const double ex = hi.w * e;
        const double x2 = 2.0 * x;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) F[m] = fma(x2, F[m + 1], ex) * (1.0 / (2 * m + 1));
    } else {
        const double ex = (double)__expf(-(float)x);
        const double rs = rsqrt(x);
        F[0] = 0.88622692545275801365 * rs;  // sqrt(pi)/2
        const double h = 0.5 * rs * rs;       // 1/(2x)
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -ex) * h;
    }
}

// The same F_m(x) in two steps, so that a caller can issue the table loads of
// several arguments before it waits for any (the erfc kernel evaluates two per
// primitive quartet).  boys_fetch reads the row nearest x, clamped to the
// table so that the load stays in bounds for any x; boys_eval takes the
// Taylor value from that row for every lane, then replaces it by the
// large-argument form where x >= 36.  For x < 36 the arithmetic is that of
// boys().
template <int L>
__device__ __forceinline__ void boys_fetch(double x, const double *__restrict__ tab, double4 &lo, double4 &hi) {
    const double xc = fmin(fmax(x, 0.0), BOYS_TMAX);
    const int i = __double2int_rn(xc * BOYS_INVH);
    const double *r = tab + ((size_t)L * BOYS_NROW + i) * BOYS_NTAY;
    lo = *reinterpret_cast<const double4 *>(r);
    hi = *reinterpret_cast<const double4 *>(r + 4);
}

template <int L>
__device__ __forceinline__ void boys_eval(double x, const double4 &lo, const double4 &hi, double *F) {
    const double xc = fmin(fmax(x, 0.0), BOYS_TMAX);
    const int i = __double2int_rn(xc * BOYS_INVH);
    const double u = i * BOYS_H - xc;
    double f = hi.z;
    f = fma(f, u, hi.y);
    f = fma(f, u, hi.x);
    f = fma(f, u, lo.w);
    f = fma(f, u, lo.z);
    f = fma(f, u, lo.y);
    f = fma(f, u, lo.x);
    F[L] = f;
    double e = fma(u, 1.0 / 720.0, 1.0 / 120.0);
    e = fma(e, u, 1.0 / 24.0);
    e = fma(e, u, 1.0 / 6.0);
    e = fma(e, u, 0.5);
    e = fma(e, u, 1.0);
    e = fma(e, u, 1.0);
    const double ex = hi.w * e;
    const double x2 = 2.0 * xc;
#pragma unroll
    for (int m = L - 1; m >= 0; --m) F[m] = fma(x2, F[m + 1], ex) * (1.0 / (2 * m + 1));
    if (!(x < BOYS_TMAX)) {
        const double exl = (double)__expf(-(float)x);
        const double rs = rsqrt(x);
        F[0] = 0.88622692545275801365 * rs;  // sqrt(pi)/2
        const double h = 0.5 * rs * rs;       // 1/(2x)
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -exl) * h;
    }
}

// FP32 Boys: x < 36 from the FP32 table (Taylor to fourth order around the
// nearest grid point, |u| <= 1/64, truncation below 1e-11 relative) and the
// downward recursion in FP32; x >= 36 in FP64 (F_0 then upward), rounded.
template <int L>
__device__ __forceinline__ void boys32(float x, const float *__restrict__ tab, float *F) {
    if (x < (float)BOYS_TMAX) {
        const float ex = __expf(-x);
        const int i = __float2int_rn(x * (float)BOYS_INVH);
        const float u = (float)i * (float)BOYS_H - x;
        const float *r = tab + ((size_t)L * BOYS_NROW + i) * BOYS_NTAY;
        const float4 lo = *reinterpret_cast<const float4 *>(r);
        const float e4 = r[4];
        float f = e4;
        f = fmaf(f, u, lo.w);
        f = fmaf(f, u, lo.z);
        f = fmaf(f, u, lo.y);
        f = fmaf(f, u, lo.x);
        F[L] = f;
        const float x2 = 2.0f * x;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) F[m] = fmaf(x2, F[m + 1], ex) * (1.0f / (2 * m + 1));
    } else {
        double Fd[L + 1];
        boys<L>((double)x, nullptr, Fd);  // large-x branch only: no table access
#pragma unroll
        for (int m = 0; m <= L; ++m) F[m] = (float)Fd[m];
    }
}

// One primitive quartet of class C: geometry, kernel function G_m, VRR into acc.
// op: 0 = 1/r, 1 = erfc(omega r)/r, where G_m = F_m(T) - theta^(2m+1) F_m(theta^2 T),
// theta^2 = omega^2/(omega^2+rho): the Gaussian transform of the kernel restricted
// to [omega, inf) maps to the Boys variable interval [theta, 1].
template <class C>
__device__ __forceinline__ void prim_quartet(const PrimRec &b, double kz, double ki2z, double kPx,
                                             double kPy, double kPz, double kQCx, double kQCy,
                                             double kQCz, double kK, int op, double om2,
                                             const double *__restrict__ tab, double *acc, double om) {
    const double ze = b.z + kz;
    const double rs = rsqrt(ze);
    const double ize = rs * rs;
    const double rho = b.z * kz * ize;
    const double PQx = b.Px - kPx, PQy = b.Py - kPy, PQz = b.Pz - kPz;
    const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    const double pref = b.K * kK * rs;
    double g[C::L + 1];
    boys<C::L>(T, tab, g);
    if (op) {
        const double th = om * rsqrt(om2 + rho);  // theta
        const double th2 = th * th;
        double g2[C::L + 1];
        boys<C::L>(th2 * T, tab, g2);
        double f = th * pref;
#pragma unroll
        for (int m = 0; m <= C::L; ++m) {
            g[m] = fma(-f, g2[m], pref * g[m]);
            f *= th2;
        }
    } else {
#pragma unroll
        for (int m = 0; m <= C::L; ++m) g[m] *= pref;
    }
    const double re = kz * ize, rz = b.z * ize;  // rho/zeta, rho/eta
    C::vrr(g, b.PAx, b.PAy, b.PAz, -re * PQx, -re * PQy, -re * PQz, kQCx, kQCy, kQCz,
           rz * PQx, rz * PQy, rz * PQz, b.i2z, re, ki2z, rz, 0.5 * ize, acc);
}

template <class C, int W>
__device__ __forceinline__ void prim_quartet_p(const PrimRec &b, double kz, double ki2z, double kPx,
                                             double kPy, double kPz, double kQCx, double kQCy,
                                             double kQCz, double kK, int op, double om2,
                                             const double *__restrict__ tab, double *acc, double om) {
    const double ze = b.z + kz;
    const double rs = rsqrt(ze);
    const double ize = rs * rs;
    const double rho = b.z * kz * ize;
    const double PQx = b.Px - kPx, PQy = b.Py - kPy, PQz = b.Pz - kPz;
    const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    const double pref = b.K * kK * rs;
    double g[C::L + 1];
    if (op) {
        const double th = om * rsqrt(om2 + rho);  // theta
        const double th2 = th * th;
        double g2[C::L + 1];
        if constexpr (C::L >= 4) {
            // both table rows in flight before either is needed: these
            // classes run one or few waves per SIMD, which exposes waits
            double4 lo1, hi1, lo2, hi2;
            boys_fetch<C::L>(T, tab, lo1, hi1);
            boys_fetch<C::L>(th2 * T, tab, lo2, hi2);
            boys_eval<C::L>(T, lo1, hi1, g);
            boys_eval<C::L>(th2 * T, lo2, hi2, g2);
        } else {
            boys<C::L>(T, tab, g);
            boys<C::L>(th2 * T, tab, g2);
        }
        double f = th * pref;
#pragma unroll
        for (int m = 0; m <= C::L; ++m) {
            g[m] = fma(-f, g2[m], pref * g[m]);
            f *= th2;
        }
    } else {
        boys<C::L>(T, tab, g);
#pragma unroll
        for (int m = 0; m <= C::L; ++m) g[m] *= pref;
    }
    const double re = kz * ize, rz = b.z * ize;  // rho/zeta, rho/eta
    C::template vrr_p<W>(g, b.PAx, b.PAy, b.PAz, -re * PQx, -re * PQy, -re * PQz, kQCx, kQCy, kQCz,
           rz * PQx, rz * PQy, rz * PQz, b.i2z, re, ki2z, rz, 0.5 * ize, acc);
}

// FP32 primitive quartet (slice W of class C in FP32).
template <class C, int W>
__device__ __forceinline__ void prim_quartet32(const PrimRec32 &b, const PrimRec32 &k, int op, float om,
                                               float om2, const float *__restrict__ tab, float *acc) {
    const float ze = b.z + k.z;
    const float rs = rsqrtf(ze);
    const float ize = rs * rs;
    const float rho = b.z * k.z * ize;
    const float PQx = (float)(b.Px - k.Px), PQy = (float)(b.Py - k.Py), PQz = (float)(b.Pz - k.Pz);
    const float T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    const float pref = b.K * k.K * rs;
    float g[C::L + 1];
    boys32<C::L>(T, tab, g);
    if (op) {
        const float th = om * rsqrtf(om2 + rho);
        const float th2 = th * th;
        float g2[C::L + 1];
        boys32<C::L>(th2 * T, tab, g2);
        float f = th * pref;
#pragma unroll
        for (int m = 0; m <= C::L; ++m) {
            g[m] = fmaf(-f, g2[m], pref * g[m]);
            f *= th2;
        }
    } else {
#pragma unroll
        for (int m = 0; m <= C::L; ++m) g[m] *= pref;
    }
    const float re = k.z * ize, rz = b.z * ize;
    C::template vrr_p<W>(g, b.PAx, b.PAy, b.PAz, -re * PQx, -re * PQy, -re * PQz, k.PAx, k.PAy, k.PAz,
                         rz * PQx, rz * PQy, rz * PQz, b.i2z, re, k.i2z, rz, 0.5f * ize, acc);
}

// Launch parameters of one class pair (bra class cb >= ket class ck).
struct QuartetArgs {
    const PairHdr *hdr;
    const PrimRec *prim;
    const int32_t *bra_ids;   // bra class: pair ids sorted by (group, -Q)
    const double *bra_Q;
    const int32_t *bra_grp;   // group index of each bra slot
    int32_t n_bra;
    int32_t bra_first;        // slots bra_first, bra_first + bra_stride, ... (sharding)
    int32_t bra_stride;
    int32_t nsub;             // ket sub-ranges per (bra slot, ket group) block row
    int32_t tq;               // ket quartets per sub-range
    int32_t nblk;             // logical blocks of this launch (grid padded to whole XCD spans)
    long long blk_base;       // first logical block of this launch (long grids run in segments)
    double om;                // omega
    const int32_t *ket_ids;   // ket class, same order
    const double *ket_Q;
    const int32_t *ket_goff;  // n_kgrp + 1 group offsets into the ket list
    const int32_t *ket_gnp;   // primitive-pair count of each ket group
    int32_t n_kgrp;
    int32_t same;             // bra class == ket class: quartet (p,q) needs q <= p
    double tau;               // ket range: tau <= Q_p Q_q < tau_hi
    double tau_hi;
    // Mixed precision: the quartets of a block split at Q_p Q_q = cut /
    // (A_p A_g), A = E / Q the ratio of a pair's FP32 error scale to its
    // Schwarz factor (A_g: the largest of ket group g), i.e. FP32 where the
    // estimated FP32 error E_p E_q is below the cut.  part 0: no split;
    // 1: the FP64 side; 2: the FP32 side.
    int32_t part;
    double mixed_cut;
    const double *bra_A;      // per bra slot
    const double *ket_gA;     // per ket group
    // Density-weighted screening: 0 off; 1: a quartet of the range is
    // computed only if also Q_p Q_q D >= tau, D the largest |P| over the shell
    // blocks of its exchange digestion; 2: the Coulomb blocks count too.
    int32_t dens;
    int32_t nsh;              // shells (pmax is nsh x nsh)
    const double *pmax;       // largest |P| of every shell block
    // Periodic builds: the bra pairs contain a home-cell shell (index <
    // nhome), every (bra, ket) combination is evaluated (no unique-quartet
    // rule), and only K rows of home-cell shells are digested, into K with
    // its own leading dimension ldK.
    int32_t nhome;
    int64_t ldK;
    int32_t op;
    double om2;               // omega^2
    double prim_tau;          // primitive quartets with B_ab B_cd < prim_tau may be skipped
    const double *boys;
    const PrimRec32 *prim32;  // FP32 records and table (FP32 launches)
    const float *boys32;
    const double *P;
    double *K;
    double *J;                  // Coulomb J' of the same quartets, or null (exchange only)
    int64_t ld;
    unsigned long long *count;  // [0] quartets, [1] primitive quartets of this launch
};

// Workgroups are dealt to the 8 XCDs round-robin by block index.  Remap so
// that each XCD runs whole chunks of `chunk` consecutive logical blocks
// (chunks interleaved over the XCDs, which keeps them balanced): the slices of
// one tile and neighbouring tiles of one bra pair then share an L2.  The grid
// is padded to a multiple of 8 chunk; padding blocks return -1.
__device__ __forceinline__ int xcd_block(int nblk, int chunk) {
    const int b = (int)blockIdx.x;
    const int span = 8 * chunk;
    const int o = b % span;
    const int lb = (b - o) + (o & 7) * chunk + (o >> 3);
    return lb < nblk ? lb : -1;
}

// The dispatch packet holds the grid size as a 32-bit count of work-items, so
// a launch must stay well below 2^32 / 64 blocks.  A longer grid is launched in
// segments of whole XCD spans; each segment carries its first logical block.
long long max_blocks_per_launch();

// wpb: logical blocks (waves) per workgroup; span and the grid count
// workgroups.
template <class Launch>
inline void launch_segments(QuartetArgs a, long long total, long long span, Launch launch, int wpb = 1) {
    const long long capg = max_blocks_per_launch() / wpb / span * span;
    const long long seg = (capg > span ? capg : span) * wpb;
    for (long long base = 0; base < total; base += seg) {
        const long long n = total - base < seg ? total - base : seg;
        a.blk_base = base;
        a.nblk = (int32_t)n;
        const long long groups = (n + wpb - 1) / wpb;
        launch(a, (unsigned)((groups + span - 1) / span * span));
    }
}

// LDS of one wave becomes visible to the other lanes of the same wave: the
// wave's LDS operations complete in order, so only the compiler must keep
// them on their side of this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First slot q in [l, h) with !(Qp Q[q] >= t); Q is sorted descending.
__device__ __forceinline__ int first_below(const double *Q, int l, int h, double Qp, double t) {
    while (l < h) {
        const int m = (l + h) >> 1;
        if (Qp * Q[m] >= t) l = m + 1;
        else h = m;
    }
    return l;
}

// Ket range of block (p, g): slots [lo, cut) of ket group g with
// tau <= Q_p Q_q < tau_hi (and q <= p inside one class).
__device__ __forceinline__ int ket_cut(const QuartetArgs &a, int p, int g, int *lo_out) {
    const double Qp = a.bra_Q[p];
    int lo = a.ket_goff[g], hi = a.ket_goff[g + 1];
    *lo_out = lo;
    if (a.same) {
        const int gp = a.bra_grp[p];
        if (g > gp) return lo;  // empty: every slot of group g is after p
        if (g == gp) hi = p + 1;
    }
    double tlo = a.tau, thi = a.tau_hi;
    if (a.part) {
        const double ts = a.mixed_cut / (a.bra_A[p] * a.ket_gA[g]);
        if (a.part == 1) tlo = fmax(tlo, ts);
        else thi = ts;  // ts <= tau: empty
    }
    lo = first_below(a.ket_Q, lo, hi, Qp, thi);
    *lo_out = lo;
    return first_below(a.ket_Q, lo, hi, Qp, tlo);
}

// Density weight of the quartet (bra shells bA bB | ket pair k): the largest
// |P| over the shell blocks its digestion multiplies (pmax is symmetric).
__device__ __forceinline__ double dens_weight(const QuartetArgs &a, int bA, int bB, const PairHdr &k) {
    const double *M = a.pmax;
    const int64_t n = a.nsh;
    double d = fmax(fmax(M[bA * n + k.shA], M[bA * n + k.shB]), fmax(M[bB * n + k.shA], M[bB * n + k.shB]));
    if (a.dens == 2) d = fmax(d, fmax(M[bA * n + bB], M[k.shA * n + k.shB]));
    return d;
}

// Calls body(q) once per tile of up to 64 ket slots of [lo, cut), q < 0 on
// idle lanes.  With density screening the slots failing the density test are
// dropped first: candidates are tested 64 at a time and the survivors queued
// in LDS (wave ballot + prefix count), so every tile but the last is full.
template <class Body>
__device__ __forceinline__ void ket_tiles(const QuartetArgs &a, int p, const PairHdr &bh, int lo, int cut,
                                          Body body) {
    const int lane = threadIdx.x & 63;
    if (!a.dens) {
        for (int q0 = lo; q0 < cut; q0 += 64) body(q0 + lane < cut ? q0 + lane : -1);
        return;
    }
    // one queue per wave: the waves of a workgroup are independent blocks
    __shared__ int queues[MAX_WPB][128];
    int *queue = queues[threadIdx.x >> 6];
    const double Qp = a.bra_Q[p];
    int nq = 0;
    for (int c0 = lo; c0 < cut; c0 += 64) {
        const int q = c0 + lane;
        bool ok = false;
        if (q < cut) {
            const PairHdr kh = a.hdr[a.ket_ids[q]];
            ok = Qp * a.ket_Q[q] * dens_weight(a, bh.shA, bh.shB, kh) >= a.tau;
        }
        const unsigned long long m = __ballot(ok);
        if (ok) queue[nq + __popcll(m & ((1ull << lane) - 1ull))] = q;
        nq += __popcll(m);
        wave_sync();
        if (nq >= 64) {
            const int qq = queue[lane];
            const int rest = lane + 64 < nq ? queue[lane + 64] : 0;
            wave_sync();
            if (lane + 64 < nq) queue[lane] = rest;
            nq -= 64;
            wave_sync();
            body(qq);
        }
    }
    if (nq > 0) body(lane < nq ? queue[lane] : -1);
}

// One wave's work on one tile: 64 lanes walk the screened ket range of bra
// pair p in ket group g; each lane holds slice W of one quartet's contracted
// array, accumulated over all primitive quartets, and digests that slice's
// share of the quartet.
// SWAP: C is the class with the pairs' roles exchanged, (cd|ab): the lane's
// ket record enters the recurrence as its bra and the wave's bra record as
// its ket, and the digestion images are the transposes of the usual ones.
template <class C, int W, int VRRW, bool WJ, bool SWAP, bool PER>
__device__ __forceinline__ void tile_part(const QuartetArgs &a, int p, int g, int lo, int cut) {
    const PairHdr bh = a.hdr[a.bra_ids[p]];
    const int nkp = a.ket_gnp[g];
    const int lane = threadIdx.x & 63;
    const double eps = a.prim_tau;
    // the bra pair is the same for the whole wave: make that explicit so its
    // records are read with scalar loads
    const int boff = __builtin_amdgcn_readfirstlane(bh.off);
    const int bn = __builtin_amdgcn_readfirstlane(bh.n);
    // records are read-only during the kernel: the constant address space lets
    // the uniform loads go through the scalar cache
    const CPrimRec *brec = (const CPrimRec *)(a.prim + boff);
    const double bmax = brec->B;
    constexpr int NA = C::NACCP[W];
    unsigned long long nprim = 0, nquart = 0;
    ket_tiles(a, p, bh, lo, cut, [&](int q) {
        const bool act = q >= 0;
        nquart += __popcll(__ballot(act));
        const int kid = a.ket_ids[act ? q : lo];
        const PairHdr kh = a.hdr[kid];
        double acc[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) acc[i] = 0.0;
        for (int kp = 0; kp < nkp; ++kp) {
            const PrimRec k = a.prim[kh.off + kp];
            const double kb = act ? k.B : 0.0;
            // records are sorted by B: once no lane can reach eps, none will
            if (!__any(kb * bmax >= eps)) break;
            for (int bp = 0; bp < bn; ++bp) {
                const PrimRec b = load_rec(brec + bp);
                if (!__any(kb * b.B >= eps)) break;
                nprim += act;
                if constexpr (SWAP)
                    prim_quartet_p<C, W>(k, b.z, b.i2z, b.Px, b.Py, b.Pz, b.PAx, b.PAy, b.PAz, b.K, a.op, a.om2,
                                         a.boys, acc, a.om);
                else
                    prim_quartet_p<C, W>(b, k.z, k.i2z, k.Px, k.Py, k.Pz, k.PAx, k.PAy, k.PAz, k.K, a.op, a.om2,
                                         a.boys, acc, a.om);
            }
        }
        if constexpr (PER) {
            if (act) {
                // rows of the wave's pair that lie in the home cell; both orders of
                // the lane's pair are digested (half each when its shells coincide)
                const double dk = kh.diag ? 0.5 : 1.0;
                const double hA = bh.shA < a.nhome ? dk : 0.0;
                const double hB = (bh.shB < a.nhome && !bh.diag) ? dk : 0.0;
                const PairHdr &x = SWAP ? kh : bh, &y = SWAP ? bh : kh;
                C::template digR<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, x.bfA, x.bfB, y.bfA, y.bfB,
                                    SWAP ? 0.0 : hA, SWAP ? 0.0 : hB, SWAP ? hA : 0.0, SWAP ? hB : 0.0, a.P, a.ld,
                                    a.K, a.ldK);
            }
        } else if (act) {
            double deg = 1.0;
            if (bh.diag) deg *= 0.5;
            if (kh.diag) deg *= 0.5;
            if (bh.id == kh.id) deg *= 0.5;
            const PairHdr &x = SWAP ? kh : bh, &y = SWAP ? bh : kh;
            C::template dig<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, x.bfA, x.bfB, y.bfA, y.bfB, deg,
                               a.P, a.K, a.ld);
            if constexpr (WJ)
                C::template digJ<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, x.bfA, x.bfB, y.bfA,
                                    y.bfB, deg, a.P, a.J, a.ld);
        }
    });
    if (W == 0 && a.count) {
        if (lane == 0 && nquart) atomicAdd(&a.count[0], nquart);
        if (nprim) atomicAdd(&a.count[1], nprim);
    }
}

template <class C, int W, bool WJ = false, bool SWAP = false, bool PER = false>
__device__ __forceinline__ void tile_dispatch(const QuartetArgs &a, int w, int p, int g, int lo, int cut) {
    if (w == W) {
        tile_part<C, W, W, WJ, SWAP, PER>(a, p, g, lo, cut);
    } else if constexpr (W + 1 < C::NSPLIT) {
        tile_dispatch<C, W + 1, WJ, SWAP, PER>(a, w, p, g, lo, cut);
    }
}

// Quartet kernel of class C.  Block = (bra slot, ket group, slice): a class
// whose contracted array is too large for one lane is cut into NSPLIT slices
// of ket components, each evaluated by its own wave (the waves of one tile
// are adjacent block indices); the common part of the recurrence is
// recomputed per slice instead of exchanged.
// WJ: also digest the Coulomb matrix J from the same quartet values.
// SWAP: C is the exchanged class (see tile_part).
// PER: periodic build (see QuartetArgs::nhome).
// C::WPB waves per workgroup, each an independent logical block (a tuning
// option, one by default: four-wave workgroups made the light classes
// slower); the XCD chunks count workgroups.
template <class C, bool WJ = false, bool SWAP = false, bool PER = false>
__global__ __launch_bounds__(64 * C::WPB) __attribute__((amdgpu_waves_per_eu(C::WAVES))) void k_eri(QuartetArgs a) {
    const int ng = (a.nblk + C::WPB - 1) / C::WPB;
    const int lg = xcd_block(ng, C::XCH);
    if (lg < 0) return;
    const int lb0 = lg * C::WPB + (C::WPB > 1 ? (int)(threadIdx.x >> 6) : 0);
    if (lb0 >= a.nblk) return;
    const long long lb = a.blk_base + lb0;
    const int w = (int)(lb % C::NSPLIT);
    long long t = lb / C::NSPLIT;
    const int sub = (int)(t % a.nsub);
    t /= a.nsub;
    const int j = (int)(t / a.n_kgrp);
    const int g = (int)(t - (long long)j * a.n_kgrp);
    const int p = a.bra_first + j * a.bra_stride;
    if (p >= a.n_bra) return;
    int lo = 0;
    const int cut = ket_cut(a, p, g, &lo);
    const int lo2 = lo + sub * a.tq;
    const int cut2 = min(cut, lo2 + a.tq);
    if (cut2 <= lo2) return;
    tile_dispatch<C, 0, WJ, SWAP, PER>(a, w, p, g, lo2, cut2);
}

// FP32 counterpart of tile_part: FP32 records, recurrences and contraction,
// FP64 digestion into K.  SWAP as in tile_part.
template <class C, int W, bool WJ, bool SWAP>
__device__ __forceinline__ void tile_part32(const QuartetArgs &a, int p, int g, int lo, int cut) {
    const PairHdr bh = a.hdr[a.bra_ids[p]];
    const int nkp = a.ket_gnp[g];
    const int lane = threadIdx.x & 63;
    const float eps = (float)a.prim_tau;
    const int boff = __builtin_amdgcn_readfirstlane(bh.off);
    const int bn = __builtin_amdgcn_readfirstlane(bh.n);
    const CPrimRec32 *brec = (const CPrimRec32 *)(a.prim32 + boff);
    const float bmax = brec->B;
    const float om2 = (float)a.om2, om = sqrtf(om2);
    constexpr int NA = C::NACCP[W];
    unsigned long long nprim = 0, nquart = 0;
    ket_tiles(a, p, bh, lo, cut, [&](int q) {
        const bool act = q >= 0;
        nquart += __popcll(__ballot(act));
        const int kid = a.ket_ids[act ? q : lo];
        const PairHdr kh = a.hdr[kid];
        float acc[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) acc[i] = 0.0f;
        for (int kp = 0; kp < nkp; ++kp) {
            const PrimRec32 k = a.prim32[kh.off + kp];
            const float kb = act ? k.B : 0.0f;
            if (!__any(kb * bmax >= eps)) break;
            for (int bp = 0; bp < bn; ++bp) {
                const PrimRec32 b = load_rec(brec + bp);
                if (!__any(kb * b.B >= eps)) break;
                nprim += act;
                if constexpr (SWAP)
                    prim_quartet32<C, W>(k, b, a.op, om, om2, a.boys32, acc);
                else
                    prim_quartet32<C, W>(b, k, a.op, om, om2, a.boys32, acc);
            }
        }
        if (act) {
            double deg = 1.0;
            if (bh.diag) deg *= 0.5;
            if (kh.diag) deg *= 0.5;
            if (bh.id == kh.id) deg *= 0.5;
            // horizontal recurrence, spherical transform and digestion in FP64
            const PairHdr &x = SWAP ? kh : bh, &y = SWAP ? bh : kh;
            C::template dig<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, x.bfA, x.bfB, y.bfA, y.bfB, deg,
                               a.P, a.K, a.ld);
            if constexpr (WJ)
                C::template digJ<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, x.bfA, x.bfB, y.bfA,
                                    y.bfB, deg, a.P, a.J, a.ld);
        }
    });
    if (W == 0 && a.count) {
        if (lane == 0 && nquart) atomicAdd(&a.count[0], nquart);
        if (nprim) atomicAdd(&a.count[1], nprim);
    }
}

template <class C, int W, bool WJ = false, bool SWAP = false>
__device__ __forceinline__ void tile_dispatch32(const QuartetArgs &a, int w, int p, int g, int lo, int cut) {
    if (w == W) {
        tile_part32<C, W, WJ, SWAP>(a, p, g, lo, cut);
    } else if constexpr (W + 1 < C::NSPLIT) {
        tile_dispatch32<C, W + 1, WJ, SWAP>(a, w, p, g, lo, cut);
    }
}

// WJ: also digest the Coulomb matrix J from the same quartet values.
// SWAP: C is the exchanged class (see tile_part).
template <class C, bool WJ = false, bool SWAP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(C::WAVES))) void k_eri32(QuartetArgs a) {
    const int lb0 = xcd_block(a.nblk, 8 * C::NSPLIT);
    if (lb0 < 0) return;
    const long long lb = a.blk_base + lb0;
    const int w = (int)(lb % C::NSPLIT);
    long long t = lb / C::NSPLIT;
    const int sub = (int)(t % a.nsub);
    t /= a.nsub;
    const int j = (int)(t / a.n_kgrp);
    const int g = (int)(t - (long long)j * a.n_kgrp);
    const int p = a.bra_first + j * a.bra_stride;
    if (p >= a.n_bra) return;
    int lo = 0;
    const int cut = ket_cut(a, p, g, &lo);
    const int lo2 = lo + sub * a.tq;
    const int cut2 = min(cut, lo2 + a.tq);
    if (cut2 <= lo2) return;
    tile_dispatch32<C, 0, WJ, SWAP>(a, w, p, g, lo2, cut2);
}

// ----------------------------------------------------------------------
// Persistent launch over many systems: a device work queue.  Every job is one
// system's class pair (its QuartetArgs); its virtual blocks are
// (bra slot, ket group, ket sub-range, slice), numbered from vbase.  A fixed
// grid of workgroups pops `claim` virtual blocks at a time from an atomic
// head until the queue is drained (every wave reaches the exit once the head
// passes vtotal).  tq = ket quartets per sub-range (the quartet-block size).
struct BatchJob {
    QuartetArgs a;
    long long vbase;
    int nsub;
    int tq;
};

template <class C, bool F32, bool SWAP = false>
__device__ __forceinline__ void persist_loop(const BatchJob *__restrict__ jobs, int njobs, long long vtotal,
                                             unsigned long long *head, int claim) {
    for (;;) {
        unsigned long long v0 = 0;
        if (threadIdx.x == 0) v0 = atomicAdd(head, (unsigned long long)claim);
        v0 = __shfl(v0, 0);
        if ((long long)v0 >= vtotal) break;
        const long long vend = min((long long)v0 + claim, vtotal);
        for (long long v = (long long)v0; v < vend; ++v) {
            int lo_j = 0, hi_j = njobs;  // last job with vbase <= v
            while (hi_j - lo_j > 1) {
                const int m = (lo_j + hi_j) >> 1;
                if (jobs[m].vbase <= v) lo_j = m;
                else hi_j = m;
            }
            const BatchJob &J = jobs[lo_j];
            long long r = v - J.vbase;
            const int w = (int)(r % C::NSPLIT);
            r /= C::NSPLIT;
            const int sub = (int)(r % J.nsub);
            r /= J.nsub;
            const int g = (int)(r % J.a.n_kgrp);
            const int p = J.a.bra_first + (int)(r / J.a.n_kgrp) * J.a.bra_stride;
            int lo = 0;
            const int cut = ket_cut(J.a, p, g, &lo);
            const int lo2 = lo + sub * J.tq;
            const int cut2 = min(cut, lo2 + J.tq);
            if (cut2 <= lo2) continue;
            if constexpr (F32) tile_dispatch32<C, 0, false, SWAP>(J.a, w, p, g, lo2, cut2);
            else tile_dispatch<C, 0, false, SWAP>(J.a, w, p, g, lo2, cut2);
        }
    }
}

template <class C, bool SWAP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(C::WAVES))) void k_eri_persist(
    const BatchJob *__restrict__ jobs, int njobs, long long vtotal, unsigned long long *head, int claim) {
    persist_loop<C, false, SWAP>(jobs, njobs, vtotal, head, claim);
}

template <class C, bool SWAP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(C::WAVES))) void k_eri32_persist(
    const BatchJob *__restrict__ jobs, int njobs, long long vtotal, unsigned long long *head, int claim) {
    persist_loop<C, true, SWAP>(jobs, njobs, vtotal, head, claim);
}

// Slice W's share of the diagonal values (ab|ab) of pair h, then the next
// slice: the slices of a split class run one after the other in one lane,
// so only one slice's contracted array is live at a time.
template <class C, int W>
__device__ __forceinline__ void schwarz_slices(const PairHdr &h, const PrimRec *__restrict__ prim, int op,
                                               double om2, const double *__restrict__ tab, double om,
                                               double *diag, double *emax) {
    double acc[C::NACCP[W]];
#pragma unroll
    for (int i = 0; i < C::NACCP[W]; ++i) acc[i] = 0.0;
    for (int kp = 0; kp < h.n; ++kp) {
        const PrimRec k = prim[h.off + kp];
        for (int bp = 0; bp < h.n; ++bp) {
            const PrimRec b = prim[h.off + bp];
            prim_quartet_p<C, W>(b, k.z, k.i2z, k.Px, k.Py, k.Pz, k.PAx, k.PAy, k.PAz, k.K, op, om2, tab, acc, om);
        }
    }
    C::template diag<W>(acc, h.ABx, h.ABy, h.ABz, diag);
    C::template diagE<W>(acc, emax);
    if constexpr (W + 1 < C::NSPLIT) schwarz_slices<C, W + 1>(h, prim, op, om2, tab, om, diag, emax);
}

// Schwarz factor of each pair of a pair class: Q = sqrt(max_ab (ab|ab)), the
// diagonal class (IJ|IJ) evaluated slice by slice.  Also the scale of the
// integrals' rounding error in FP32:
//     E = s_la s_lb (1 + max_i |AB_i|)^lb sqrt(max_e [e0|e0]),
// where [e0|e0] (|e| = la .. la+lb) are the diagonal contracted inputs of the
// horizontal recurrence (so |[e0|f0]| <= sqrt([e0|e0] [f0|f0]) by Schwarz),
// (1 + |AB|)^lb bounds the sum of the absolute coefficients with which the
// recurrence combines them and s_l (1 for s and p, 2 for d) that of a
// spherical row.  Every value of a quartet is then at most E_IJ E_KL in size
// (so E >= Q), and rounding errors of its inputs reach it multiplied by at
// most those sums: evaluated in FP32 a quartet is in error by about
// eps32 E_IJ E_KL, however small its value and its bound Q_IJ Q_KL are.
template <class C>
__global__ __launch_bounds__(64) void k_schwarz(const PairHdr *__restrict__ hdr,
                                                const PrimRec *__restrict__ prim,
                                                const int32_t *__restrict__ ids, int n, int op,
                                                double om2, const double *__restrict__ tab,
                                                double *__restrict__ Q, double *__restrict__ E) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= n) return;
    const PairHdr h = hdr[ids[t]];
    const double om = sqrt(om2);
    constexpr int NA = 2 * C::LA + 1, NB = 2 * C::LB + 1;
    double diag[NA * NB];
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) diag[i] = 0.0;
    double emax = 0.0;
    schwarz_slices<C, 0>(h, prim, op, om2, tab, om, diag, &emax);
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) mx = fmax(mx, diag[i]);
    Q[h.id] = sqrt(mx);
    const double ab = 1.0 + fmax(fabs(h.ABx), fmax(fabs(h.ABy), fabs(h.ABz)));
    double amp = (C::LA == 2 ? 2.0 : 1.0) * (C::LB == 2 ? 2.0 : 1.0);
#pragma unroll
    for (int k = 0; k < C::LB; ++k) amp *= ab;
    E[h.id] = amp * sqrt(emax);
}

// Schwarz factor B of every primitive pair of the pairs of one pair class
// (the diagonal integral of the single primitive pair, spherical), then the
// records of each pair sorted by B, largest first.
template <class C>
__global__ __launch_bounds__(64) void k_primbound(const PairHdr *__restrict__ hdr, PrimRec *__restrict__ prim,
                                                  const int32_t *__restrict__ ids, int n, int op, double om2,
                                                  const double *__restrict__ tab) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= n) return;
    const PairHdr h = hdr[ids[t]];
    const double om = sqrt(om2);
    constexpr int NA = 2 * C::LA + 1, NB = 2 * C::LB + 1;
    for (int r = 0; r < h.n; ++r) {
        const PrimRec x = prim[h.off + r];
        double acc[C::NACC];
#pragma unroll
        for (int i = 0; i < C::NACC; ++i) acc[i] = 0.0;
        prim_quartet<C>(x, x.z, x.i2z, x.Px, x.Py, x.Pz, x.PAx, x.PAy, x.PAz, x.K, op, om2, tab, acc, om);
        double out[C::NOUT];
        C::post(acc, h.ABx, h.ABy, h.ABz, h.ABx, h.ABy, h.ABz, out);
        double mx = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) mx = fmax(mx, out[((i * NB + j) * NA + i) * NB + j]);
        prim[h.off + r].B = sqrt(mx);
    }
    for (int i = 1; i < h.n; ++i) {  // insertion sort by B, descending
        const PrimRec x = prim[h.off + i];
        int j = i - 1;
        while (j >= 0 && prim[h.off + j].B < x.B) {
            prim[h.off + j + 1] = prim[h.off + j];
            --j;
        }
        prim[h.off + j + 1] = x;
    }
}

// Raw integrals of listed quartets, one per lane, with the code of the
// exchange build: the per-slice recurrences, the exchanged class structs and
// the same horizontal recurrence and spherical transform; every primitive
// quartet is evaluated (no screening).  Each slice adds its share of every
// spherical value to the lane's output block.
// x: the pair whose records enter the recurrence as its bra, y: as its ket.
template <class C, int W>
__device__ __forceinline__ void eval_slices(const PairHdr &x, const PairHdr &y, const PrimRec *__restrict__ prim,
                                            int op, double om2, const double *__restrict__ tab, double om,
                                            int64_t sab, int64_t scd, double *out) {
    double acc[C::NACCP[W]];
#pragma unroll
    for (int i = 0; i < C::NACCP[W]; ++i) acc[i] = 0.0;
    for (int kp = 0; kp < y.n; ++kp) {
        const PrimRec k = prim[y.off + kp];
        for (int bp = 0; bp < x.n; ++bp) {
            const PrimRec b = prim[x.off + bp];
            prim_quartet_p<C, W>(b, k.z, k.i2z, k.Px, k.Py, k.Pz, k.PAx, k.PAy, k.PAz, k.K, op, om2, tab, acc, om);
        }
    }
    C::template store<W>(acc, x.ABx, x.ABy, x.ABz, y.ABx, y.ABy, y.ABz, sab, scd, out);
    if constexpr (W + 1 < C::NSPLIT) eval_slices<C, W + 1>(x, y, prim, op, om2, tab, om, sab, scd, out);
}

// bk: canonical pair ids (bra of the class's higher pair class, ket); out:
// NOUT values per quartet in [a][b][c][d] order of the canonical bra and ket.
// SWAP: C is the exchanged struct (cd|ab); its output index order is then
// the transpose, undone by the strides.
template <class C, bool SWAP = false>
__global__ __launch_bounds__(64) void k_eval(const PairHdr *__restrict__ hdr, const PrimRec *__restrict__ prim,
                                             const int32_t *__restrict__ bk, int n, int op, double om2,
                                             const double *__restrict__ tab, double *__restrict__ out) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= n) return;
    const PairHdr bh = hdr[bk[2 * t]], kh = hdr[bk[2 * t + 1]];
    const double om = sqrt(om2);
    double *o = out + (int64_t)t * C::NOUT;
    for (int i = 0; i < C::NOUT; ++i) o[i] = 0.0;
    // struct's (ab) block index runs over its own bra pair, (cd) over its ket
    constexpr int64_t nab = (2 * C::LA + 1) * (2 * C::LB + 1), ncd = (2 * C::LC + 1) * (2 * C::LD + 1);
    if constexpr (SWAP)
        eval_slices<C, 0>(kh, bh, prim, op, om2, tab, om, 1, nab, o);
    else
        eval_slices<C, 0>(bh, kh, prim, op, om2, tab, om, ncd, 1, o);
}

}  // namespace hfx
