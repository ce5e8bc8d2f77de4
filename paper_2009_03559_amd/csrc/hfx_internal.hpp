// Host-side state of a pair handle (device pair data, bounds, screening lists).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hfx.h"
#include "hfx_device.hpp"

namespace hfx {

struct ClassList {
    int n = 0, ngrp = 0;
    int32_t *d_ids = nullptr, *d_grp = nullptr, *d_goff = nullptr, *d_gnp = nullptr;
    double *d_Q = nullptr;
    double *d_A = nullptr, *d_gA = nullptr;  // mixed lists: E/Q per slot, largest per group
    std::vector<int> goff, gnp;
    std::vector<int32_t> h_ids, h_grp;
    std::vector<double> h_Q;
};

// Device scratch of one build: per-block partial maxima of the P symmetry
// check (2 doubles per block, at most PCHECK_BLOCKS blocks) and the quartet
// counters (4 per class).  A pair handle owns one; the no-allocation entry
// point passes its own.
constexpr int PCHECK_BLOCKS = 1024;
constexpr int NCOUNT = 4 * HFX_NCLASS;
struct Workspace {
    double *part;                // 2 * PCHECK_BLOCKS doubles
    unsigned long long *count;   // NCOUNT counters
};

hfx_status fail(hfx_status s, const std::string &msg);
int kernel_op(const hfx_opts *o);
int quartet_block(int L);
extern const int PAIR_L[6][2];
hfx_status check_opts(const hfx_opts *o);
hfx_status check_P(const double *P, int64_t n, int64_t ld, hipStream_t st, double *part);
hfx_status compute_bounds(hfx_pairs p, const hfx_opts *o, hipStream_t st);
hfx_status build_lists(hfx_pairs p, double tau, bool mixed, hipStream_t st);
const ClassList *class_lists(hfx_pairs p, bool mixed);
hfx_status ensure_prim32(hfx_pairs p, hipStream_t st);
// ws == nullptr: the handle's own workspace, and bounds, lists and FP32
// records are made if missing.  ws != nullptr: the caller's workspace, and
// nothing is allocated: the handle must already hold the bounds, lists and
// FP32 records these options need (else HFX_EINVAL).
hfx_status build_K_impl(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld, const hfx_opts *o,
                        int shard, int nshards, void *stream, hfx_stats *st_out, double *J_dev = nullptr,
                        const Workspace *ws = nullptr);
void launch_fill_K(double *K, int64_t n, int64_t ld, hipStream_t st);
void launch_fill_u64(unsigned long long *c, int n, hipStream_t st);
void launch_symmetrize(double *K, int64_t n, int64_t ld, hipStream_t st);
hfx_status shell_pmax(hfx_pairs p, const double *P, int64_t ld, bool may_allocate, hipStream_t st);
int density_mode(const hfx_opts *o, bool coulomb);
const double *model_vrr();
const double *model_post();
double model_prim_overhead(int op, int L);

}  // namespace hfx

struct hfx_pairs_s;
typedef struct hfx_pairs_s *hfx_pairs;

struct hfx_pairs_s {
    int natom = 0, nshell = 0;
    int64_t nbf = 0, npair = 0, nrec = 0, dev_bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<hfx_shell> sh;
    std::vector<double> xyz, exps, cn;
    std::vector<int> bfo;
    std::vector<int8_t> pcls;
    std::vector<int32_t> class_ids[6];
    std::vector<hfx::PairHdr> hdr_host;
    hfx::PairHdr *d_hdr = nullptr;
    hfx::PrimRec *d_prim = nullptr;
    double *d_Q = nullptr;
    double *d_E = nullptr;                  // FP32 error scale of every pair (see k_schwarz)
    const double *d_boys = nullptr;
    const float *d_boys32 = nullptr;
    hfx::PrimRec32 *d_prim32 = nullptr;
    bool prim32_valid = false;
    unsigned long long *d_count = nullptr;  // workspace of builds on this handle
    double *d_part = nullptr;
    int32_t *d_class_ids = nullptr;         // pair ids of every pair class, concatenated
    int32_t *d_bfo = nullptr;               // first function of every shell (nshell + 1)
    double *d_pmax = nullptr;               // largest |P| of every shell block (density screening)
    hipEvent_t ev[HFX_NCLASS + 1] = {};      // class-kernel timing events
    bool have_Q = false;
    int q_op = -1;
    double q_om2 = -1.0;
    std::vector<double> Q, E;
    double qmax = 0.0;
    bool lists_valid = false;   // FP64 lists: groups of equal primitive-pair count
    double list_tau = -1.0;
    hfx::ClassList lists[6];
    bool mlists_valid = false;  // mixed-precision lists: groups of equal count and error-scale bin
    double mlist_tau = -1.0;
    hfx::ClassList mlists[6];
    bool hlists_valid = false;  // periodic builds: kept pairs with a home-cell shell
    double hlist_tau = -1.0;
    int hlist_nhome = -1;
    hfx::ClassList hlists[6];
    void drop_lists();
    ~hfx_pairs_s();
};
