/*
 * hfx.h -- C ABI of libhfx: Schwarz-screened exchange (HFX) build on MI355X.
 *
 * The library evaluates contracted Gaussian electron repulsion integrals over
 * screened shell quartets and digests them against a density matrix P into
 *
 *     K_ik = sum_jl (ij|kl) P_jl                                   (1)
 *
 * (the exchange matrix of Sec. 2, eq. for V^X, without its -1/2 and without a
 * hybrid mixing fraction, for an open-boundary cluster: no lattice sums);
 * optionally also the Coulomb matrix J_ij = sum_kl (ij|kl) P_kl from the same
 * integrals (hfx_build_JK).
 * Two kernels are supported: the bare Coulomb 1/r of the ERI definition in
 * Sec. 2 and the attenuated erfc(omega r)/r of the HSE06 functional named in
 * Sec. 4.  Shells are contracted Gaussians sum_m D_m r^l exp(-alpha_m r^2)
 * (Sec. 3) with l <= 2; results are over spherical functions, 2l+1 per shell
 * (Sec. 3, Cartesian->spherical transformation).  Screening follows the
 * Schwarz inequality of Sec. 3: pairs are preselected and every unique shell
 * quartet (8-fold permutational symmetry, Sec. 3) is computed iff
 * Q_IJ Q_KL >= tau.
 *
 * Conventions shared by every call
 *   - Units: bohr and hartree.
 *   - Spherical function order: shells in the order given; p = (x, y, z);
 *     d = (xy, yz, z^2 - (x^2+y^2)/2, xz, (x^2-y^2) sqrt(3)/2) with sqrt(3)
 *     on xy, yz, xz; all relative to Cartesians normalised like x^l.
 *   - Normalisation: coefficients multiply normalised primitives and every
 *     contracted shell is rescaled to unit norm.
 *   - Device buffers (P, K) are caller-owned device memory (hipMalloc,
 *     coarse-grained, e.g. a torch CUDA tensor), row-major with leading
 *     dimension ld >= n_bf.  K must not alias P.
 *   - `stream` is a hipStream_t (NULL = default stream).  Device work is
 *     stream-ordered; a call may synchronise the stream where documented.
 *   - Every call returns an hfx_status; hfx_last_error() gives the message
 *     of the last failing call on the calling thread.  After an error, K
 *     holds no promised content.
 *   - Handles (hfx_pairs, hfx_server) are owned by the library and freed by
 *     their *_destroy call.  A handle is used by one host thread at a time.
 */
#ifndef HFX_H
#define HFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HFX_OK = 0,
    HFX_EINVAL = 1,       /* bad size, pointer, exponent, tolerance, omega */
    HFX_EUNSUPPORTED = 2, /* l > 2, too many primitives or basis functions */
    HFX_ENOMEM = 3,       /* device allocation or HBM admission failed */
    HFX_EBUSY = 4,        /* server queue full */
    HFX_ENOTFOUND = 5,    /* unknown ticket */
    HFX_EDEVICE = 6,      /* HIP runtime error (message kept) */
    HFX_EASYM = 7         /* P not symmetric within 1e-12 max|P| */
} hfx_status;

typedef enum { HFX_OP_COULOMB = 0, HFX_OP_ERFC = 1 } hfx_op;
typedef enum { HFX_PREC_FP64 = 0, HFX_PREC_MIXED = 1 } hfx_prec;

#define HFX_MAX_L 2
#define HFX_MAX_PRIM 16
#define HFX_MAX_NBF 65535 /* n_bf limit: n_bf^2 work-items per element kernel */
#define HFX_NCLASS 21

/* One contracted shell: centre index, angular momentum, primitive count and
 * offset of its primitives in the exps/coefs arrays (Sec. 3). */
typedef struct {
    int32_t atom;
    int32_t l;
    int32_t nprim;
    int32_t prim_off;
} hfx_shell;

/* Options.  tau: Schwarz drop tolerance (>= 0; Sec. 3 uses 1e-5, the
 * synthetic workloads 1e-10).  op/omega: kernel; ERFC with omega == 0 is
 * the Coulomb kernel.  prec: FP64, or MIXED, where quartets whose FP32
 * error scale E_IJ E_KL is below mixed_cut are evaluated in FP32 (FP64
 * large-T Boys, FP64 bounds, horizontal recurrence and accumulation into K).
 * E_IJ = s_la s_lb (1 + max_i |AB_i|)^lb sqrt(max_e [e0|e0]) >= Q_IJ (s_l =
 * 1, 1, 2 for s, p, d) bounds the values the horizontal recurrence takes in,
 * times the sum of its coefficients: the size of a quartet's FP32 rounding
 * error relative to FP32 epsilon.  prim_tau (>= 0): inside a
 * computed quartet, primitive quartets whose bound B_ab B_cd is below
 * prim_tau may be skipped, where B_ab is the Schwarz factor of the single
 * primitive pair (a bound on every primitive contribution); 0 keeps every
 * primitive quartet (exact evaluation of each computed quartet).  flags: 0,
 * or HFX_FLAG_DENSITY_SCREEN: a quartet that passes the Schwarz test is
 * computed only if also Q_IJ Q_KL D >= tau, where D is the largest |P|
 * over the shell blocks its digestion multiplies -- (I,K) (I,L) (J,K) (J,L)
 * for K, and (I,J) (K,L) as well when J is built (the density screening that
 * Sec. 3 adds after the Schwarz test, read for Gaussian shells). */
#define HFX_FLAG_DENSITY_SCREEN 1
typedef struct {
    double tau;
    int32_t op;
    double omega;
    int32_t prec;
    double mixed_cut;
    double prim_tau;
    int32_t flags;
} hfx_opts;

typedef struct hfx_pairs_s *hfx_pairs;
typedef struct hfx_server_s *hfx_server;

/* Per-call statistics (filled when a non-NULL pointer is passed; this
 * synchronises the stream).  class_quartets uses the class order
 * (ss|ss) (ps|ss) (ps|ps) (pp|ss) (pp|ps) (pp|pp) (ds|ss) ... (dd|dd):
 * pair classes ss ps pp ds dp dd numbered 0..5, class index
 * cb(cb+1)/2 + ck with cb >= ck. */
typedef struct {
    double latency_s;      /* host wall time of the call */
    double device_s;       /* device time of the quartet kernels */
    int64_t quartets;      /* unique shell quartets evaluated */
    int64_t quartets_fp32; /* of which in FP32 (mixed mode) */
    int64_t prim_quartets; /* primitive quartets evaluated */
    double flops;          /* algorithmic FLOPs (model, FMA = 2) */
    int64_t class_quartets[HFX_NCLASS];
    double class_device_s[HFX_NCLASS]; /* device time of each class kernel */
    double class_flops[HFX_NCLASS];    /* algorithmic FLOPs of each class */
} hfx_stats;

/* Validate and normalise the basis, enumerate all shell pairs I >= J (A =
 * the shell of higher l within a pair), and build the device-resident
 * primitive-pair data (exponent sums, Gaussian product centres, prefactors)
 * on `stream` (Sec. 3, pair lists).  xyz: host, natom*3.  shells: host,
 * nshell entries.  exps, coefs: host, indexed by prim_off.  o: only checked
 * for validity here.  Errors: EINVAL (natom/nshell < 1, atom index, nprim
 * < 1, alpha <= 0 or not finite, offsets out of range), EUNSUPPORTED (l > 2,
 * nprim > HFX_MAX_PRIM, n_bf > HFX_MAX_NBF), ENOMEM, EDEVICE.  On success *out owns the device
 * memory until hfx_pairs_destroy. */
hfx_status hfx_build_shell_pairs(const double *xyz, int32_t natom, const hfx_shell *shells,
                                 int32_t nshell, const double *exps, const double *coefs,
                                 const hfx_opts *o, void *stream, hfx_pairs *out);

/* Schwarz factors Q_IJ = sqrt(max_{i in I, j in J} (ij|ij)) for every pair,
 * in FP64, with the kernel of `o` (Sec. 3, Schwarz inequality).  Stored in
 * the handle; if q_host_or_null is non-NULL it receives nshell(nshell+1)/2
 * values in pair order (0,0), (1,0), (1,1), (2,0), ... (shell indices
 * I >= J).  Synchronises the stream.  Errors: EINVAL, EDEVICE. */
hfx_status hfx_schwarz_bounds(hfx_pairs p, const hfx_opts *o, double *q_host_or_null, void *stream);

/* Exchange build (1): K is overwritten with sum over the unique screened
 * quartets, digested with their permutation images.  P_dev, K_dev: device,
 * n_bf x n_bf, leading dimension ld.  Computes the bounds first if they are
 * missing or were made for another kernel.  Synchronises the stream for the
 * symmetry check of P and for the screening lists (these are cached in the
 * handle for repeated calls with the same tau).  Errors: EINVAL (NULL, ld <
 * n_bf, tau < 0, omega < 0, aliasing), EASYM, ENOMEM, EDEVICE. */
hfx_status hfx_build_K(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                       const hfx_opts *o, void *stream, hfx_stats *st_or_null);

/* Coulomb and exchange from the same screened quartets: J_ij = sum_kl
 * (ij|kl) P_kl (the Hartree term of the total-energy expression, Sec. 2)
 * is digested from every quartet value that also feeds K (1), so the
 * integrals are evaluated once for both.  J_dev, K_dev: device, n_bf x n_bf,
 * leading dimension ld, both overwritten; J must alias neither P nor K.
 * Screening, precision modes and stats are those of hfx_build_K (stats
 * flops include the Coulomb digestion).  Errors: as hfx_build_K, EINVAL if
 * J_dev is NULL or aliases P or K. */
hfx_status hfx_build_JK(hfx_pairs p, const double *P_dev, double *J_dev, double *K_dev, int64_t ld,
                        const hfx_opts *o, void *stream, hfx_stats *st_or_null);

/* One device's share of the exchange build when it is distributed over
 * nshards devices: the bra pairs of every class (slots of the Q-sorted
 * lists) are dealt round-robin, slot s going to shard s mod nshards, and
 * this call digests the quartets of shard `shard` only.  K receives that
 * share's symmetrised partial K; the sum over all shards is the K of
 * hfx_build_K (the cross-device step is then one all-reduce of K).  The
 * round-robin deal balances cost the way the quartet-level distribution of
 * Sec. 3.1 does, without replicated screening.  nshards = 1 is hfx_build_K.
 * Errors: as hfx_build_K, EINVAL if shard is not in [0, nshards). */
hfx_status hfx_build_K_shard(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                             const hfx_opts *o, int32_t shard, int32_t nshards, void *stream,
                             hfx_stats *st_or_null);

/* One device's share of the joint Coulomb + exchange build: the shard of
 * hfx_build_K_shard with the Coulomb digestion of hfx_build_JK.  J and K
 * receive that share's symmetrised partial matrices; the sums over shards
 * are the J and K of hfx_build_JK.  Errors: as hfx_build_JK and
 * hfx_build_K_shard. */
hfx_status hfx_build_JK_shard(hfx_pairs p, const double *P_dev, double *J_dev, double *K_dev, int64_t ld,
                              const hfx_opts *o, int32_t shard, int32_t nshards, void *stream,
                              hfx_stats *st_or_null);

/* Periodic exchange (Sec. 2, eq. V^X without its -1/2): for a crystal
 * written as a finite cluster of image cells,
 *     K^G_{mu lambda} = sum_{nu sigma} sum_{N H} (mu^0 nu^N | lambda^G sigma^H) P^{H-N}_{nu sigma}
 * with mu in the home cell (the paper's list-IJ: first index in the unit
 * cell) and nu, sigma, lambda over every cell of the cluster (list-KL over
 * the supercell); the lattice sums run over the cluster's cells and are
 * screened by Q_IJ Q_KL >= tau.  p: pair handle of the cluster, whose first
 * nhome_shell shells (and functions) are the home cell's.  P_dev: device,
 * n_bf x n_bf (leading dimension ldP), P_big[a][b] = P^{cell(b)-cell(a)}_{f(a)
 * f(b)} -- symmetric.  K_dev: device, n_home x n_bf (leading dimension ldK,
 * n_home = functions of the home cell), overwritten: K_dev[mu][b] =
 * K^{cell(b)}_{mu f(b)}.  Every combination of a kept pair with a home-cell
 * shell and a kept pair of the cluster is evaluated (the ket pair's two
 * orders digested together), FP64 only.  Synchronises the stream.  Errors:
 * as hfx_build_K; EINVAL (nhome_shell not in [1, nshell], ldP or ldK <
 * n_bf, aliasing), EUNSUPPORTED (mixed precision or flags). */
hfx_status hfx_build_K_periodic(hfx_pairs p, int32_t nhome_shell, const double *P_dev, int64_t ldP,
                                double *K_dev, int64_t ldK, const hfx_opts *o, void *stream,
                                hfx_stats *st_or_null);

/* Many independent systems in one persistent launch per pass, fed by a
 * device work queue (Sec. 5 proposes dynamic distribution of the quartet
 * work; here the queue is shared by all systems).  A system with at least
 * 250 basis functions (environment HFX_BATCH_DIRECT_NBF; 0 = never) fills
 * the device on its own and is built with the kernels of hfx_build_K
 * instead, one after another on the same stream.  Arrays of length nsys;
 * every system follows the rules of hfx_build_K.  st (optional) sums over
 * the systems.  Errors as hfx_build_K. */
hfx_status hfx_build_K_batch(int32_t nsys, const hfx_pairs *p, const double *const *P_dev,
                             double *const *K_dev, const int64_t *ld, const hfx_opts *o,
                             void *stream, hfx_stats *st_or_null);

/* Serving: a request loop that admits K-builds against an HBM budget
 * (bytes of device memory the server may hold for queued work) and runs
 * at most max_inflight of them concurrently on its own streams, so work of
 * requests that arrive while others run overlaps on the device.  At most
 * 4096 requests wait at a time (the environment variable HFX_SERVER_QUEUE,
 * read here, sets another capacity).  Errors: EINVAL (budget <= 0,
 * max_inflight not in [1, 64]), EDEVICE. */
hfx_status hfx_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, hfx_server *s);

/* Queue one K-build (non-blocking).  P_dev/K_dev must stay valid until the
 * ticket is done.  The pair handle (and its device pair data) stays
 * resident and may be submitted again for the next SCF iteration.  Errors:
 * EINVAL, ENOMEM (request larger than the whole budget), EBUSY (queue
 * full). */
hfx_status hfx_submit(hfx_server s, hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                      const hfx_opts *o, uint64_t *ticket);

/* Poll a ticket: *done = 1 when K is complete (then st, if non-NULL, holds
 * its statistics; latency_s counts from submission).  Errors: ENOTFOUND,
 * or the status of the failed build. */
hfx_status hfx_poll(hfx_server s, uint64_t ticket, int32_t *done, hfx_stats *st);

/* Number of spherical functions and of shell pairs, n_shell (n_shell + 1) / 2, of a pair handle. */
int64_t hfx_pairs_nbf(hfx_pairs p);
int64_t hfx_pairs_npair(hfx_pairs p);
/* Device bytes held by a pair handle. */
int64_t hfx_pairs_device_bytes(hfx_pairs p);

/* Raw spherical integrals of listed shell quartets (used to check sampled
 * outputs of large builds) evaluated with the code of the FP64 exchange
 * build: its per-slice vertical recurrences, its exchanged class layouts and
 * its horizontal recurrence and spherical transform, one quartet per lane,
 * every primitive quartet included (no screening, no digestion).
 * quartets: host, 4*n shell indices (I,J,K,L) in any order.
 * out: host, receives for each quartet its (2lI+1)(2lJ+1)(2lK+1)(2lL+1)
 * values in [i][j][k][l] order, packed one after another.  Synchronises.
 * Errors: EINVAL, EDEVICE. */
hfx_status hfx_eval_quartets(hfx_pairs p, const hfx_opts *o, int64_t n, const int32_t *quartets,
                             double *out, void *stream);

/* Exchange build that allocates no device memory: for callers that cannot
 * allocate (code under HIP stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and errors as hfx_build_K
 * (same kernels), with two differences.  (1) Nothing is built on demand: the
 * handle must already hold the Schwarz bounds for this kernel and omega, the
 * screening lists for this tau, in mixed precision the FP32 records and with
 * density screening the array of |P| block maxima -- one hfx_build_K with the
 * same options on the handle leaves them resident; otherwise EINVAL, with
 * nothing allocated.  (2) Its workspace (the P
 * symmetry check's partial maxima and the quartet counters) is a fixed
 * static device array of HFX_NOALLOC_SCRATCH_BYTES per GPU, independent of
 * the system size, held until the process ends and shared by every call on
 * that GPU: calls that overlap in time on one GPU race on it.  Synchronises
 * the stream (the symmetry check of P). */
#define HFX_NOALLOC_SCRATCH_BYTES 17152
hfx_status hfx_build_K_noalloc(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                               const hfx_opts *o, void *stream, hfx_stats *st_or_null);

void hfx_pairs_destroy(hfx_pairs p);
void hfx_server_destroy(hfx_server s);
const char *hfx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HFX_H */
