/*
 * Plain FP64 CPU oracle for the Schwarz-screened exchange build
 *
 *     K_ik = sum_jl (ij|kl) P_jl
 *
 * over contracted Gaussian shells (l <= 2, spherical functions), for the bare
 * Coulomb kernel 1/r and the HSE-type attenuated kernel erfc(omega r)/r.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; it is built separately and used by the tests, the smoke
 * check and the CPU baseline of the benchmark.  It shares no code, tables or
 * helpers with the GPU path.  It is written for clarity, not speed: every
 * primitive quartet fills a full Obara-Saika table.
 *
 * What it follows (paper sections):
 *   - exchange matrix and its density contraction: Sec. 2, eq. (V^X); the -1/2
 *     and the hybrid mixing fraction are left to the caller;
 *   - the two-electron integral: Sec. 2 (ERI definition), with the attenuated
 *     kernel of HSE06 named in Sec. 4;
 *   - contracted shells chi(r) = sum_m D_m r^l exp(-alpha_m r^2): Sec. 3;
 *   - 8-fold permutational symmetry: Sec. 3, eq. (8-fold symmetry);
 *   - shell quartets with (2l+1) spherical functions per shell and the
 *     Cartesian->spherical transform: Sec. 3;
 *   - Schwarz inequality, pair preselection and quartet screening: Sec. 3,
 *     eq. (Schwarz) and the text after it.
 * Readings where the paper is silent are listed in the design notes; the ones
 * this file fixes are repeated at the function that applies them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_LMAX 2
#define OR_EMAX (2 * OR_LMAX)          /* highest l_a+l_b */
#define OR_MMAX (4 * OR_LMAX)          /* highest total L */
#define OR_NTRIP(n) (((n) + 1) * ((n) + 2) * ((n) + 3) / 6) /* triples of degree <= n */
#define OR_NT (OR_NTRIP(OR_EMAX))      /* 35 */
#define OR_MAXPRIM 16

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------- */
/* Cartesian monomials x^i y^j z^k of degree n, ordered with i descending, then
 * j descending.  Global index over all degrees <= n: degrees stacked.          */
static int tri_off(int n) { return n * (n + 1) * (n + 2) / 6; }
static int tri_idx(int i, int j, int k) {
    int n = i + j + k;
    return tri_off(n) + (n - i) * (n - i + 1) / 2 + (n - i - j);
}
static void tri_of(int idx, int *ijk) {
    int n = 0;
    while (tri_off(n + 1) <= idx) n++;
    int r = idx - tri_off(n);
    for (int i = n; i >= 0; i--) {
        int cnt = n - i + 1;
        if (r < cnt) {
            ijk[0] = i;
            ijk[1] = n - i - r;
            ijk[2] = r;
            return;
        }
        r -= cnt;
    }
}
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int nsph(int l) { return 2 * l + 1; }

/* ------------------------------------------------------------------------- */
/* Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt.
 * T < 30: the convergent series exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)).
 * T >= 30: F_0 = sqrt(pi) erf(sqrt T) / (2 sqrt T), then the upward recursion
 * F_(m+1) = ((2m+1) F_m - exp(-T)) / (2T), which is stable for large T.     */
double oracle_boys(int m, double T) {
    if (T < 30.0) {
        double term = 1.0 / (2 * m + 1), sum = term;
        for (int k = 1; k < 2000; k++) {
            term *= 2.0 * T / (2 * m + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return exp(-T) * sum;
    }
    double st = sqrt(T);
    double f = sqrt(OR_PI) * erf(st) / (2.0 * st);
    double e = exp(-T);
    for (int k = 0; k < m; k++) f = ((2 * k + 1) * f - e) / (2.0 * T);
    return f;
}

/* Kernel function G_m: F_m(T) for 1/r; for erfc(omega r)/r the Gaussian
 * transform of the kernel runs from omega to infinity, which in the Boys
 * variable t^2 = u^2/(u^2+rho) is the interval [theta, 1] with
 * theta^2 = omega^2/(omega^2+rho): G_m = F_m(T) - theta^(2m+1) F_m(theta^2 T).
 * The Obara-Saika recurrences hold pointwise in t, so they keep their
 * coefficients.                                                              */
static void kernel_G(int L, double T, double rho, double omega, double *G) {
    for (int m = 0; m <= L; m++) G[m] = oracle_boys(m, T);
    if (omega > 0.0) {
        double th2 = omega * omega / (omega * omega + rho);
        double th = sqrt(th2);
        double p = th;
        for (int m = 0; m <= L; m++) {
            G[m] -= p * oracle_boys(m, th2 * T);
            p *= th2;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Normalisation (reading of Sec. 3: coefficients multiply normalised
 * primitives; the contraction is rescaled to unit norm).
 *   primitive x^l exp(-a r^2):  N = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!)
 *   contraction: sum_pq c_p c_q [2 sqrt(a_p a_q)/(a_p+a_q)]^(l+3/2) = 1     */
static double dfact(int n) { double r = 1; for (int k = n; k > 1; k -= 2) r *= k; return r; }

void oracle_normalise(int nshell, const int32_t *sh_l, const int32_t *sh_nprim,
                      const int32_t *sh_off, const double *exps, const double *coefs,
                      double *out) {
    for (int s = 0; s < nshell; s++) {
        int l = sh_l[s], n = sh_nprim[s], o = sh_off[s];
        for (int p = 0; p < n; p++) {
            double a = exps[o + p];
            out[o + p] = coefs[o + p] * pow(2 * a / OR_PI, 0.75) * pow(4 * a, 0.5 * l) /
                         sqrt(dfact(2 * l - 1));
        }
        double ss = 0;
        for (int p = 0; p < n; p++)
            for (int q = 0; q < n; q++) {
                double ap = exps[o + p], aq = exps[o + q];
                ss += coefs[o + p] * coefs[o + q] * pow(2 * sqrt(ap * aq) / (ap + aq), l + 1.5);
            }
        double f = 1.0 / sqrt(ss);
        for (int p = 0; p < n; p++) out[o + p] *= f;
    }
}

/* Cartesian -> spherical rows, relative to Cartesians normalised like x^l.
 * s: 1.  p: x, y, z.  d (m=-2..2): sqrt3 xy, sqrt3 yz, z2 - (x2+y2)/2,
 * sqrt3 xz, sqrt3/2 (x2 - y2).  Cartesian d order: xx xy xz yy yz zz.       */
static void sph_matrix(int l, double M[5][6]) {
    memset(M, 0, sizeof(double) * 30);
    if (l == 0) { M[0][0] = 1; return; }
    if (l == 1) { M[0][0] = 1; M[1][1] = 1; M[2][2] = 1; return; }
    double r3 = sqrt(3.0);
    M[0][1] = r3;                        /* xy */
    M[1][4] = r3;                        /* yz */
    M[2][5] = 1; M[2][0] = -0.5; M[2][3] = -0.5; /* z2 */
    M[3][2] = r3;                        /* xz */
    M[4][0] = 0.5 * r3; M[4][3] = -0.5 * r3;     /* x2 - y2 */
}

/* ------------------------------------------------------------------------- */
typedef struct {
    const double *xyz;
    const int32_t *atom, *l, *nprim, *off;
    const double *exps;
    const double *cn;   /* normalised coefficients */
    int nshell;
} basis_t;

/* Contracted spherical shell quartet (AB|CD), with A,B,C,D shell indices.
 * Output layout out[a][b][c][d], a fastest last (row-major over
 * (2la+1, 2lb+1, 2lc+1, 2ld+1)).  Route: Obara-Saika vertical recurrence for
 * [e0|f0]^(m) on every primitive quartet (two-sided form, ket built on top of
 * the bra), contraction, Head-Gordon-Pople horizontal recurrence on the
 * contracted integrals, then the spherical transform of every index.        */
typedef struct { double v[OR_MMAX + 1][OR_NT][OR_NT]; } vtab_t;

static void shell_quartet_raw(const basis_t *B, int sA, int sB, int sC, int sD, double omega,
                              vtab_t *W, double *out) {
    int la = B->l[sA], lb = B->l[sB], lc = B->l[sC], ld = B->l[sD];
    int E = la + lb, F = lc + ld, L = E + F;
    const double *A = B->xyz + 3 * B->atom[sA], *Bc = B->xyz + 3 * B->atom[sB];
    const double *C = B->xyz + 3 * B->atom[sC], *D = B->xyz + 3 * B->atom[sD];
    int ntE = OR_NTRIP(E), ntF = OR_NTRIP(F);
    static const int zero = 0; (void)zero;
    double cont[OR_NT][OR_NT];
    memset(cont, 0, sizeof(cont));
    double AB2 = 0, CD2 = 0;
    for (int i = 0; i < 3; i++) {
        AB2 += (A[i] - Bc[i]) * (A[i] - Bc[i]);
        CD2 += (C[i] - D[i]) * (C[i] - D[i]);
    }
    for (int pa = 0; pa < B->nprim[sA]; pa++)
    for (int pb = 0; pb < B->nprim[sB]; pb++) {
        double a = B->exps[B->off[sA] + pa], b = B->exps[B->off[sB] + pb];
        double zeta = a + b;
        double Pc[3];
        for (int i = 0; i < 3; i++) Pc[i] = (a * A[i] + b * Bc[i]) / zeta;
        double Kab = exp(-a * b / zeta * AB2);
        double cab = B->cn[B->off[sA] + pa] * B->cn[B->off[sB] + pb];
        for (int pc = 0; pc < B->nprim[sC]; pc++)
        for (int pd = 0; pd < B->nprim[sD]; pd++) {
            double c = B->exps[B->off[sC] + pc], d = B->exps[B->off[sD] + pd];
            double eta = c + d;
            double Qc[3];
            for (int i = 0; i < 3; i++) Qc[i] = (c * C[i] + d * D[i]) / eta;
            double Kcd = exp(-c * d / eta * CD2);
            double ccd = B->cn[B->off[sC] + pc] * B->cn[B->off[sD] + pd];
            double rho = zeta * eta / (zeta + eta);
            double Wc[3], PQ2 = 0;
            for (int i = 0; i < 3; i++) {
                Wc[i] = (zeta * Pc[i] + eta * Qc[i]) / (zeta + eta);
                PQ2 += (Pc[i] - Qc[i]) * (Pc[i] - Qc[i]);
            }
            double T = rho * PQ2;
            double G[OR_MMAX + 1];
            kernel_G(L, T, rho, omega, G);
            double pref = 2.0 * pow(OR_PI, 2.5) / (zeta * eta * sqrt(zeta + eta)) * Kab * Kcd * cab * ccd;
            for (int m = 0; m <= L; m++) W->v[m][0][0] = pref * G[m];
            /* bra: [e+1_i,0|00]^(m) = PA_i [e]^(m) + WP_i [e]^(m+1)
             *                        + e_i/(2 zeta) ([e-1_i]^(m) - rho/zeta [e-1_i]^(m+1)) */
            for (int ie = 1; ie < ntE; ie++) {
                int e[3]; tri_of(ie, e);
                int n = e[0] + e[1] + e[2];
                int i = e[0] ? 0 : (e[1] ? 1 : 2);
                int e1[3] = {e[0], e[1], e[2]}; e1[i]--;
                int i1 = tri_idx(e1[0], e1[1], e1[2]);
                int i2 = -1;
                if (e1[i] > 0) { int e2[3] = {e1[0], e1[1], e1[2]}; e2[i]--; i2 = tri_idx(e2[0], e2[1], e2[2]); }
                for (int m = 0; m <= L - n; m++) {
                    double v = (Pc[i] - A[i]) * W->v[m][i1][0] + (Wc[i] - Pc[i]) * W->v[m + 1][i1][0];
                    if (i2 >= 0)
                        v += e1[i] / (2 * zeta) * (W->v[m][i2][0] - rho / zeta * W->v[m + 1][i2][0]);
                    W->v[m][ie][0] = v;
                }
            }
            /* ket: [e|f+1_i]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
             *       + f_i/(2 eta) ([e|f-1_i]^(m) - rho/eta [e|f-1_i]^(m+1))
             *       + e_i/(2(zeta+eta)) [e-1_i|f]^(m+1)                       */
            for (int jf = 1; jf < ntF; jf++) {
                int f[3]; tri_of(jf, f);
                int nf = f[0] + f[1] + f[2];
                int i = f[0] ? 0 : (f[1] ? 1 : 2);
                int f1[3] = {f[0], f[1], f[2]}; f1[i]--;
                int j1 = tri_idx(f1[0], f1[1], f1[2]);
                int j2 = -1;
                if (f1[i] > 0) { int f2[3] = {f1[0], f1[1], f1[2]}; f2[i]--; j2 = tri_idx(f2[0], f2[1], f2[2]); }
                for (int ie = 0; ie < ntE; ie++) {
                    int e[3]; tri_of(ie, e);
                    int ne = e[0] + e[1] + e[2];
                    int im = -1;
                    if (e[i] > 0) { int em[3] = {e[0], e[1], e[2]}; em[i]--; im = tri_idx(em[0], em[1], em[2]); }
                    for (int m = 0; m <= L - ne - nf; m++) {
                        double v = (Qc[i] - C[i]) * W->v[m][ie][j1] + (Wc[i] - Qc[i]) * W->v[m + 1][ie][j1];
                        if (j2 >= 0)
                            v += f1[i] / (2 * eta) * (W->v[m][ie][j2] - rho / eta * W->v[m + 1][ie][j2]);
                        if (im >= 0) v += e[i] / (2 * (zeta + eta)) * W->v[m + 1][im][j1];
                        W->v[m][ie][jf] = v;
                    }
                }
            }
            for (int ie = 0; ie < ntE; ie++)
                for (int jf = 0; jf < ntF; jf++) cont[ie][jf] += W->v[0][ie][jf];
        }
    }
    /* HRR on the bra: (e, b+1_i| = (e+1_i, b| + AB_i (e, b|, AB = A - B.
     * hb[e][b][f]: e over all degrees la..E-|b|, b over degrees <= lb.     */
    static const int NB = OR_NTRIP(OR_LMAX);
    double (*hb)[10][OR_NT] = calloc(OR_NT, sizeof(*hb));
    for (int ie = 0; ie < ntE; ie++)
        for (int jf = 0; jf < ntF; jf++) hb[ie][0][jf] = cont[ie][jf];
    for (int ib = 1; ib < OR_NTRIP(lb); ib++) {
        int bb[3]; tri_of(ib, bb);
        int i = bb[0] ? 0 : (bb[1] ? 1 : 2);
        int b1[3] = {bb[0], bb[1], bb[2]}; b1[i]--;
        int ib1 = tri_idx(b1[0], b1[1], b1[2]);
        int nb = bb[0] + bb[1] + bb[2];
        for (int ie = 0; ie < OR_NTRIP(E - nb); ie++) {
            int e[3]; tri_of(ie, e);
            int ep[3] = {e[0], e[1], e[2]}; ep[i]++;
            int iep = tri_idx(ep[0], ep[1], ep[2]);
            for (int jf = 0; jf < ntF; jf++)
                hb[ie][ib][jf] = hb[iep][ib1][jf] + (A[i] - Bc[i]) * hb[ie][ib1][jf];
        }
    }
    (void)NB;
    /* Cartesian bra block (a of degree la, b of degree lb). */
    int nca = ncart(la), ncb = ncart(lb), ncc = ncart(lc), ncd = ncart(ld);
    double *bra = calloc((size_t)nca * ncb * ntF, sizeof(double));
    for (int a = 0; a < nca; a++)
        for (int b = 0; b < ncb; b++)
            for (int jf = 0; jf < ntF; jf++)
                bra[(a * ncb + b) * ntF + jf] = hb[tri_off(la) + a][tri_off(lb) + b][jf];
    free(hb);
    /* HRR on the ket: (f, d+1_i) = (f+1_i, d) + CD_i (f, d), CD = C - D.     */
    double *car = calloc((size_t)nca * ncb * ncc * ncd, sizeof(double));
    double hk[OR_NT][10];
    for (int ab = 0; ab < nca * ncb; ab++) {
        for (int jf = 0; jf < ntF; jf++) hk[jf][0] = bra[ab * ntF + jf];
        for (int id = 1; id < OR_NTRIP(ld); id++) {
            int dd[3]; tri_of(id, dd);
            int i = dd[0] ? 0 : (dd[1] ? 1 : 2);
            int d1[3] = {dd[0], dd[1], dd[2]}; d1[i]--;
            int id1 = tri_idx(d1[0], d1[1], d1[2]);
            int nd = dd[0] + dd[1] + dd[2];
            for (int jf = 0; jf < OR_NTRIP(F - nd); jf++) {
                int f[3]; tri_of(jf, f);
                int fp[3] = {f[0], f[1], f[2]}; fp[i]++;
                hk[jf][id] = hk[tri_idx(fp[0], fp[1], fp[2])][id1] + (C[i] - D[i]) * hk[jf][id1];
            }
        }
        for (int c = 0; c < ncc; c++)
            for (int d = 0; d < ncd; d++) car[(ab * ncc + c) * ncd + d] = hk[tri_off(lc) + c][tri_off(ld) + d];
    }
    free(bra);
    /* Spherical transform of the four indices. */
    double Ma[5][6], Mb[5][6], Mc[5][6], Md[5][6];
    sph_matrix(la, Ma); sph_matrix(lb, Mb); sph_matrix(lc, Mc); sph_matrix(ld, Md);
    int nsa = nsph(la), nsb = nsph(lb), nsc = nsph(lc), nsd = nsph(ld);
    for (int A1 = 0; A1 < nsa; A1++)
    for (int B1 = 0; B1 < nsb; B1++)
    for (int C1 = 0; C1 < nsc; C1++)
    for (int D1 = 0; D1 < nsd; D1++) {
        double s = 0;
        for (int a = 0; a < nca; a++) {
            if (Ma[A1][a] == 0) continue;
            for (int b = 0; b < ncb; b++) {
                if (Mb[B1][b] == 0) continue;
                for (int c = 0; c < ncc; c++) {
                    if (Mc[C1][c] == 0) continue;
                    for (int d = 0; d < ncd; d++) {
                        if (Md[D1][d] == 0) continue;
                        s += Ma[A1][a] * Mb[B1][b] * Mc[C1][c] * Md[D1][d] *
                             car[((a * ncb + b) * ncc + c) * ncd + d];
                    }
                }
            }
        }
        out[((A1 * nsb + B1) * nsc + C1) * nsd + D1] = s;
    }
    free(car);
}

/* Shell quartet in the caller's index order (I J | K L): the recurrences want
 * the higher l first in each pair, so swap inside a pair where needed and
 * permute the result back.                                                   */
static void shell_quartet(const basis_t *B, int I, int J, int K, int L, double omega, vtab_t *W,
                          double *out) {
    int swab = B->l[J] > B->l[I], swcd = B->l[L] > B->l[K];
    int a = swab ? J : I, b = swab ? I : J, c = swcd ? L : K, d = swcd ? K : L;
    double tmp[625];
    shell_quartet_raw(B, a, b, c, d, omega, W, tmp);
    int ni = nsph(B->l[I]), nj = nsph(B->l[J]), nk = nsph(B->l[K]), nl = nsph(B->l[L]);
    int na = nsph(B->l[a]), nb = nsph(B->l[b]), nc = nsph(B->l[c]), nd = nsph(B->l[d]);
    for (int i = 0; i < ni; i++)
    for (int j = 0; j < nj; j++)
    for (int k = 0; k < nk; k++)
    for (int l = 0; l < nl; l++) {
        int ia = swab ? j : i, ib = swab ? i : j, ic = swcd ? l : k, id = swcd ? k : l;
        out[((i * nj + j) * nk + k) * nl + l] = tmp[((ia * nb + ib) * nc + ic) * nd + id];
    }
    (void)na;
}

/* ------------------------------------------------------------------------- */
static int setup_basis(basis_t *B, const double *xyz, int nshell, const int32_t *atom,
                       const int32_t *l, const int32_t *nprim, const int32_t *off,
                       const double *exps, const double *coefs, double **cn_out) {
    int ntot = 0;
    for (int s = 0; s < nshell; s++) {
        if (l[s] < 0 || l[s] > OR_LMAX || nprim[s] < 1 || nprim[s] > OR_MAXPRIM) return 1;
        if (off[s] + nprim[s] > ntot) ntot = off[s] + nprim[s];
    }
    double *cn = malloc(sizeof(double) * (ntot > 0 ? ntot : 1));
    oracle_normalise(nshell, l, nprim, off, exps, coefs, cn);
    B->xyz = xyz; B->atom = atom; B->l = l; B->nprim = nprim; B->off = off;
    B->exps = exps; B->cn = cn; B->nshell = nshell;
    *cn_out = cn;
    return 0;
}

/* One contracted spherical shell quartet, caller order, layout [i][j][k][l]. */
int oracle_shell_quartet(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                         const int32_t *nprim, const int32_t *off, const double *exps,
                         const double *coefs, int I, int J, int K, int L, double omega,
                         double *out) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    vtab_t *W = malloc(sizeof(vtab_t));
    shell_quartet(&B, I, J, K, L, omega, W, out);
    free(W); free(cn);
    return 0;
}

/* Full n_bf^4 tensor (tiny systems only), layout [i][j][k][l]. */
int oracle_eri_tensor(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                      const int32_t *nprim, const int32_t *off, const double *exps,
                      const double *coefs, double omega, double *out) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    int *bfo = malloc(sizeof(int) * (nshell + 1));
    bfo[0] = 0;
    for (int s = 0; s < nshell; s++) bfo[s + 1] = bfo[s] + nsph(l[s]);
    int64_t n = bfo[nshell];
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double blk[625];
        #pragma omp for schedule(dynamic) collapse(2)
        for (int I = 0; I < nshell; I++)
        for (int J = 0; J < nshell; J++)
        for (int K = 0; K < nshell; K++)
        for (int L = 0; L < nshell; L++) {
            shell_quartet(&B, I, J, K, L, omega, W, blk);
            int ni = nsph(l[I]), nj = nsph(l[J]), nk = nsph(l[K]), nl = nsph(l[L]);
            for (int i = 0; i < ni; i++)
            for (int j = 0; j < nj; j++)
            for (int k = 0; k < nk; k++)
            for (int q = 0; q < nl; q++)
                out[(((int64_t)(bfo[I] + i) * n + bfo[J] + j) * n + bfo[K] + k) * n + bfo[L] + q] =
                    blk[((i * nj + j) * nk + k) * nl + q];
        }
        free(W);
    }
    free(bfo); free(cn);
    return 0;
}

/* Schwarz factor Q_IJ = sqrt(max over spherical i in I, j in J of (ij|ij)),
 * with the same kernel as the exchange build (a valid bound for erfc because
 * its Fourier transform is non-negative).  Pairs are I >= J in the order
 * (0,0), (1,0), (1,1), (2,0), ... ; Q has n(n+1)/2 entries.                  */
int oracle_schwarz(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                   const int32_t *nprim, const int32_t *off, const double *exps,
                   const double *coefs, double omega, double *Q) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    int64_t npair = (int64_t)nshell * (nshell + 1) / 2;
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double blk[625];
        #pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < npair; p++) {
            int I = (int)((sqrt(8.0 * p + 1) - 1) / 2);
            while ((int64_t)I * (I + 1) / 2 > p) I--;
            while ((int64_t)(I + 1) * (I + 2) / 2 <= p) I++;
            int J = (int)(p - (int64_t)I * (I + 1) / 2);
            shell_quartet(&B, I, J, I, J, omega, W, blk);
            int ni = nsph(l[I]), nj = nsph(l[J]);
            double mx = 0;
            for (int i = 0; i < ni; i++)
                for (int j = 0; j < nj; j++) {
                    double v = blk[((i * nj + j) * ni + i) * nj + j];
                    if (v > mx) mx = v;
                }
            Q[p] = sqrt(mx);
        }
        free(W);
    }
    free(cn);
    return 0;
}

/* Schwarz factors of an explicit list of pair indices (same definition). */
int oracle_schwarz_list(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                        const int32_t *nprim, const int32_t *off, const double *exps,
                        const double *coefs, double omega, int64_t n, const int64_t *pids, double *Q) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double blk[625];
        #pragma omp for schedule(dynamic, 4)
        for (int64_t x = 0; x < n; x++) {
            int64_t p = pids[x];
            int I = (int)((sqrt(8.0 * p + 1) - 1) / 2);
            while ((int64_t)I * (I + 1) / 2 > p) I--;
            while ((int64_t)(I + 1) * (I + 2) / 2 <= p) I++;
            int J = (int)(p - (int64_t)I * (I + 1) / 2);
            shell_quartet(&B, I, J, I, J, omega, W, blk);
            int ni = nsph(l[I]), nj = nsph(l[J]);
            double mx = 0;
            for (int i = 0; i < ni; i++)
                for (int j = 0; j < nj; j++) {
                    double v = blk[((i * nj + j) * ni + i) * nj + j];
                    if (v > mx) mx = v;
                }
            Q[x] = sqrt(mx);
        }
        free(W);
    }
    free(cn);
    return 0;
}

/* Digest one unique shell quartet (IJ|KL) into K' (n x n, row-major):
 * with degeneracy d = (1/2 if I=J)(1/2 if K=L)(1/2 if IJ=KL) and value v of
 * function quartet (ijkl):
 *   K'_ik += d v P_jl,  K'_il += d v P_jk,  K'_jk += d v P_il,  K'_jl += d v P_ik.
 * These four images plus their transposes (K = K' + K'^T, P symmetric) are
 * the eight permutations of the quartet (Sec. 3, 8-fold symmetry).          */
static void digest(const double *blk, int I, int J, int K, int L, const int *bfo, const int32_t *l,
                   const double *P, int64_t n, double *Kp) {
    double d = 1.0;
    if (I == J) d *= 0.5;
    if (K == L) d *= 0.5;
    if (I == K && J == L) d *= 0.5;
    int ni = nsph(l[I]), nj = nsph(l[J]), nk = nsph(l[K]), nl = nsph(l[L]);
    for (int i = 0; i < ni; i++)
    for (int j = 0; j < nj; j++)
    for (int k = 0; k < nk; k++)
    for (int q = 0; q < nl; q++) {
        double v = d * blk[((i * nj + j) * nk + k) * nl + q];
        int64_t gi = bfo[I] + i, gj = bfo[J] + j, gk = bfo[K] + k, gl = bfo[L] + q;
        Kp[gi * n + gk] += v * P[gj * n + gl];
        Kp[gi * n + gl] += v * P[gj * n + gk];
        Kp[gj * n + gk] += v * P[gi * n + gl];
        Kp[gj * n + gl] += v * P[gi * n + gk];
    }
}

/* Coulomb digestion of the same unique quartet (the Hartree term):
 * J_ij = sum_kl (ij|kl) P_kl.  The eight permutations of (ij|kl) update
 * J_ij, J_ji with v P_kl twice each and J_kl, J_lk with v P_ij twice each
 * (P symmetric), so with the same degeneracy factor d:
 *   J'_ij += 2 d v P_kl,  J'_kl += 2 d v P_ij,  then J = J' + J'^T.        */
static void digest_J(const double *blk, int I, int J, int K, int L, const int *bfo, const int32_t *l,
                     const double *P, int64_t n, double *Jp) {
    double d = 2.0;
    if (I == J) d *= 0.5;
    if (K == L) d *= 0.5;
    if (I == K && J == L) d *= 0.5;
    int ni = nsph(l[I]), nj = nsph(l[J]), nk = nsph(l[K]), nl = nsph(l[L]);
    for (int i = 0; i < ni; i++)
    for (int j = 0; j < nj; j++)
    for (int k = 0; k < nk; k++)
    for (int q = 0; q < nl; q++) {
        double v = d * blk[((i * nj + j) * nk + k) * nl + q];
        int64_t gi = bfo[I] + i, gj = bfo[J] + j, gk = bfo[K] + k, gl = bfo[L] + q;
        Jp[gi * n + gj] += v * P[gk * n + gl];
        Jp[gk * n + gl] += v * P[gi * n + gj];
    }
}

static int pair_I(int64_t p) {
    int I = (int)((sqrt(8.0 * (double)p + 1) - 1) / 2);
    while ((int64_t)I * (I + 1) / 2 > p) I--;
    while ((int64_t)(I + 1) * (I + 2) / 2 <= p) I++;
    return I;
}

/* Screened exchange build.  Keep-rule for pairs (reading of the pair
 * preselection in Sec. 3): keep IJ iff Q_IJ * max(Q) >= tau.  Quartet rule
 * (Sec. 3, Schwarz screening): compute unique (IJ|KL), IJ >= KL in pair
 * order, iff Q_IJ * Q_KL >= tau.  With tau = 0 every quartet is computed.
 * counts[0] = quartets computed, counts[1] = primitive quartets,
 * counts[2 + c] = quartets of class c (c = 0..20, class order of
 * oracle_class_index).  Returns 0 on success.                              */
int oracle_class_index(int la, int lb, int lc, int ld) {
    /* pair class of (la >= lb): ss=0 ps=1 pp=2 ds=3 dp=4 dd=5 */
    int x = la >= lb ? la : lb, y = la >= lb ? lb : la;
    int u = lc >= ld ? lc : ld, w = lc >= ld ? ld : lc;
    int cb = x * (x + 1) / 2 + y, ck = u * (u + 1) / 2 + w;
    if (cb < ck) { int t = cb; cb = ck; ck = t; }
    return cb * (cb + 1) / 2 + ck;
}

/* Largest |P_xy| over the functions x of shell X and y of shell Y, for every
 * shell pair (n_shell x n_shell, row-major).                                */
static double *shell_pmax(int nshell, const int *bfo, const double *P, int64_t n) {
    double *M = malloc(sizeof(double) * (size_t)nshell * (nshell > 0 ? nshell : 1));
    for (int X = 0; X < nshell; X++)
        for (int Y = 0; Y < nshell; Y++) {
            double m = 0;
            for (int x = bfo[X]; x < bfo[X + 1]; x++)
                for (int y = bfo[Y]; y < bfo[Y + 1]; y++) {
                    double a = fabs(P[(int64_t)x * n + y]);
                    if (a > m) m = a;
                }
            M[(size_t)X * nshell + Y] = m;
        }
    return M;
}

/* Density weight of the unique quartet (IJ|KL): the largest |P| over the
 * shell blocks that multiply its integrals in the digestion.  Exchange: the
 * blocks (I,K), (I,L), (J,K), (J,L); with the Coulomb matrix also (I,J) and
 * (K,L).  Reading of the screening the paper adds after the Schwarz test
 * (Sec. 3, NAO screening): an integral that can change no element of K (or
 * J) by tau or more is skipped.                                             */
static double density_weight(const double *M, int nshell, int I, int J, int K, int L, int coulomb) {
    double d = M[(size_t)I * nshell + K];
    double v;
    v = M[(size_t)I * nshell + L]; if (v > d) d = v;
    v = M[(size_t)J * nshell + K]; if (v > d) d = v;
    v = M[(size_t)J * nshell + L]; if (v > d) d = v;
    if (coulomb) {
        v = M[(size_t)I * nshell + J]; if (v > d) d = v;
        v = M[(size_t)K * nshell + L]; if (v > d) d = v;
    }
    return d;
}

static int build_JK(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                    const int32_t *nprim, const int32_t *off, const double *exps,
                    const double *coefs, const double *P, double tau, double omega,
                    int nthreads, double *Jout, double *K, double *Q_out, int64_t *counts,
                    int density) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    int *bfo = malloc(sizeof(int) * (nshell + 1));
    bfo[0] = 0;
    for (int s = 0; s < nshell; s++) bfo[s + 1] = bfo[s] + nsph(l[s]);
    int64_t n = bfo[nshell];
    int64_t npair = (int64_t)nshell * (nshell + 1) / 2;
    double *Q = malloc(sizeof(double) * (npair > 0 ? npair : 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    oracle_schwarz(xyz, nshell, atom, l, nprim, off, exps, coefs, omega, Q);
    double qmax = 0;
    for (int64_t p = 0; p < npair; p++) if (Q[p] > qmax) qmax = Q[p];
    memset(K, 0, sizeof(double) * n * n);
    if (Jout) memset(Jout, 0, sizeof(double) * n * n);
    double *M = density ? shell_pmax(nshell, bfo, P, n) : NULL;
    int64_t cnt[2 + 21] = {0};
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double *Kp = calloc((size_t)(n * n), sizeof(double));
        double *Jp = Jout ? calloc((size_t)(n * n), sizeof(double)) : NULL;
        int64_t lc_[2 + 21] = {0};
        double blk[625];
        #pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npair; p++) {
            if (!(Q[p] * qmax >= tau)) continue;
            int I = pair_I(p), J = (int)(p - (int64_t)I * (I + 1) / 2);
            for (int64_t q = 0; q <= p; q++) {
                if (!(Q[q] * qmax >= tau)) continue;
                if (!(Q[p] * Q[q] >= tau)) continue;
                int Kk = pair_I(q), Ll = (int)(q - (int64_t)Kk * (Kk + 1) / 2);
                if (M && !(Q[p] * Q[q] * density_weight(M, nshell, I, J, Kk, Ll, Jout != NULL) >= tau)) continue;
                shell_quartet(&B, I, J, Kk, Ll, omega, W, blk);
                digest(blk, I, J, Kk, Ll, bfo, l, P, n, Kp);
                if (Jp) digest_J(blk, I, J, Kk, Ll, bfo, l, P, n, Jp);
                lc_[0]++;
                lc_[1] += (int64_t)nprim[I] * nprim[J] * nprim[Kk] * nprim[Ll];
                lc_[2 + oracle_class_index(l[I], l[J], l[Kk], l[Ll])]++;
            }
        }
        #pragma omp critical
        {
            for (int64_t x = 0; x < n * n; x++) K[x] += Kp[x];
            if (Jp) for (int64_t x = 0; x < n * n; x++) Jout[x] += Jp[x];
            for (int c = 0; c < 23; c++) cnt[c] += lc_[c];
        }
        free(Kp); free(Jp); free(W);
    }
    /* K = K' + K'^T, J = J' + J'^T */
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i; j < n; j++) {
            double s = K[i * n + j] + K[j * n + i];
            K[i * n + j] = s; K[j * n + i] = s;
            if (Jout) {
                double t = Jout[i * n + j] + Jout[j * n + i];
                Jout[i * n + j] = t; Jout[j * n + i] = t;
            }
        }
    if (Q_out) memcpy(Q_out, Q, sizeof(double) * npair);
    if (counts) memcpy(counts, cnt, sizeof(cnt));
    free(Q); free(bfo); free(cn); free(M);
    return 0;
}

int oracle_build_K(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                   const int32_t *nprim, const int32_t *off, const double *exps,
                   const double *coefs, const double *P, double tau, double omega,
                   int nthreads, double *K, double *Q_out, int64_t *counts) {
    return build_JK(xyz, nshell, atom, l, nprim, off, exps, coefs, P, tau, omega, nthreads,
                    NULL, K, Q_out, counts, 0);
}

/* Exchange (and, with J non-NULL, Coulomb) build with the density-weighted
 * test added to the Schwarz test: a unique quartet passing Q_IJ Q_KL >= tau
 * is computed iff also Q_IJ Q_KL D_IJKL >= tau, D the density weight above. */
int oracle_build_JK_density(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                            const int32_t *nprim, const int32_t *off, const double *exps,
                            const double *coefs, const double *P, double tau, double omega,
                            int nthreads, double *J, double *K, double *Q_out, int64_t *counts) {
    return build_JK(xyz, nshell, atom, l, nprim, off, exps, coefs, P, tau, omega, nthreads,
                    J, K, Q_out, counts, 1);
}

/* Coulomb and exchange from the same screened quartets: J_ij = sum_kl (ij|kl)
 * P_kl next to K_ik = sum_jl (ij|kl) P_jl (the Hartree and exchange terms of
 * the total-energy expression, Sec. 2).  Same screening and counts.         */
int oracle_build_JK(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                    const int32_t *nprim, const int32_t *off, const double *exps,
                    const double *coefs, const double *P, double tau, double omega,
                    int nthreads, double *J, double *K, double *Q_out, int64_t *counts) {
    return build_JK(xyz, nshell, atom, l, nprim, off, exps, coefs, P, tau, omega, nthreads,
                    J, K, Q_out, counts, 0);
}

/* Digest an explicit list of unique shell quartets (I,J,K,L given as pair
 * indices p >= q) into K' (not symmetrised).  Used to time the oracle on a
 * bounded sample of a large workload and to check sampled outputs.         */
int oracle_digest_list(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                       const int32_t *nprim, const int32_t *off, const double *exps,
                       const double *coefs, const double *P, double omega, int64_t nq,
                       const int64_t *pairs_pq, int nthreads, double *Kp_out) {
    basis_t B; double *cn;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    int *bfo = malloc(sizeof(int) * (nshell + 1));
    bfo[0] = 0;
    for (int s = 0; s < nshell; s++) bfo[s + 1] = bfo[s] + nsph(l[s]);
    int64_t n = bfo[nshell];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    memset(Kp_out, 0, sizeof(double) * n * n);
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double *Kp = calloc((size_t)(n * n), sizeof(double));
        double blk[625];
        #pragma omp for schedule(dynamic, 16)
        for (int64_t x = 0; x < nq; x++) {
            int64_t p = pairs_pq[2 * x], q = pairs_pq[2 * x + 1];
            int I = pair_I(p), J = (int)(p - (int64_t)I * (I + 1) / 2);
            int Kk = pair_I(q), Ll = (int)(q - (int64_t)Kk * (Kk + 1) / 2);
            shell_quartet(&B, I, J, Kk, Ll, omega, W, blk);
            digest(blk, I, J, Kk, Ll, bfo, l, P, n, Kp);
        }
        #pragma omp critical
        for (int64_t y = 0; y < n * n; y++) Kp_out[y] += Kp[y];
        free(Kp); free(W);
    }
    free(bfo); free(cn);
    return 0;
}


/* ------------------------------------------------------------------------- */
/* Periodic exchange (Sec. 2, eq. V^X without its -1/2):
 *     K^G_{mu lambda} = sum_{nu, sigma} sum_{N, H} (mu^0 nu^N | lambda^G sigma^H) P^{H-N}_{nu sigma},
 * mu in the home cell, the lattice sums over N, H (and the output cells G)
 * truncated to the cells of a finite cluster.  The caller lays the cluster
 * out as one basis: the home cell's shells first (shells 0 .. nhome-1), then
 * the image shells; Pbig[a][b] = P^{cell(b)-cell(a)}_{f(a) f(b)} (n x n over the
 * cluster's functions) and Kout[mu][b] = K^{cell(b)}_{mu f(b)} (rows: the home
 * cell's functions, the first ones of the basis; n columns).  In cluster terms
 * Kout[i][k] = sum_{j,l} (ij|kl) Pbig[j][l] for i in the home cell.
 * Screening: the shell quartet (IJ|KL) is evaluated iff Q_IJ Q_KL >= tau, with
 * the cluster's Schwarz factors.  Plain loops over ordered shell quartets
 * with I in the home cell; no permutational symmetry is used.
 * counts[0] = the screened combinations (unordered pair {I,J} with I or J in
 * the home cell, unordered pair {K,L}); counts[1] = their primitive quartets;
 * counts[2 + c] = per class (oracle_class_index).                           */
int oracle_build_K_periodic(const double *xyz, int nshell, const int32_t *atom, const int32_t *l,
                            const int32_t *nprim, const int32_t *off, const double *exps,
                            const double *coefs, int nhome, const double *Pbig, double tau, double omega,
                            int nthreads, double *Kout, int64_t *counts) {
    basis_t B; double *cn;
    if (nhome < 0 || nhome > nshell) return 1;
    if (setup_basis(&B, xyz, nshell, atom, l, nprim, off, exps, coefs, &cn)) return 1;
    int *bfo = malloc(sizeof(int) * (nshell + 1));
    bfo[0] = 0;
    for (int s = 0; s < nshell; s++) bfo[s + 1] = bfo[s] + nsph(l[s]);
    int64_t n = bfo[nshell], nh = bfo[nhome];
    int64_t npair = (int64_t)nshell * (nshell + 1) / 2;
    double *Q = malloc(sizeof(double) * (npair > 0 ? npair : 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    oracle_schwarz(xyz, nshell, atom, l, nprim, off, exps, coefs, omega, Q);
    memset(Kout, 0, sizeof(double) * nh * n);
    #pragma omp parallel
    {
        vtab_t *W = malloc(sizeof(vtab_t));
        double *Kp = calloc((size_t)(nh * n), sizeof(double));
        double blk[625];
        #pragma omp for schedule(dynamic, 1) collapse(2)
        for (int I = 0; I < nhome; I++)
        for (int J = 0; J < nshell; J++) {
            int64_t pij = I >= J ? (int64_t)I * (I + 1) / 2 + J : (int64_t)J * (J + 1) / 2 + I;
            for (int K = 0; K < nshell; K++)
            for (int L = 0; L < nshell; L++) {
                int64_t pkl = K >= L ? (int64_t)K * (K + 1) / 2 + L : (int64_t)L * (L + 1) / 2 + K;
                if (!(Q[pij] * Q[pkl] >= tau)) continue;
                shell_quartet(&B, I, J, K, L, omega, W, blk);
                int ni = nsph(l[I]), nj = nsph(l[J]), nk = nsph(l[K]), nl = nsph(l[L]);
                for (int i = 0; i < ni; i++)
                for (int j = 0; j < nj; j++)
                for (int k = 0; k < nk; k++)
                for (int q = 0; q < nl; q++) {
                    double v = blk[((i * nj + j) * nk + k) * nl + q];
                    Kp[(int64_t)(bfo[I] + i) * n + bfo[K] + k] += v * Pbig[(int64_t)(bfo[J] + j) * n + bfo[L] + q];
                }
            }
        }
        #pragma omp critical
        for (int64_t x = 0; x < nh * n; x++) Kout[x] += Kp[x];
        free(Kp); free(W);
    }
    if (counts) {
        int64_t cnt[2 + 21] = {0};
        for (int I = 0; I < nshell; I++)
        for (int J = 0; J <= I; J++) {
            if (!(I < nhome || J < nhome)) continue;
            int64_t pij = (int64_t)I * (I + 1) / 2 + J;
            for (int K = 0; K < nshell; K++)
            for (int L = 0; L <= K; L++) {
                int64_t pkl = (int64_t)K * (K + 1) / 2 + L;
                if (!(Q[pij] * Q[pkl] >= tau)) continue;
                cnt[0]++;
                cnt[1] += (int64_t)nprim[I] * nprim[J] * nprim[K] * nprim[L];
                cnt[2 + oracle_class_index(l[I], l[J], l[K], l[L])]++;
            }
        }
        memcpy(counts, cnt, sizeof(cnt));
    }
    free(Q); free(bfo); free(cn);
    return 0;
}
