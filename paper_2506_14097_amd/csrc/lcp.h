// lcp.h -- launch arguments of the contact-row and LCP kernels (lcp.hip).
#pragma once

#include "common.h"

namespace relcp {

// Rows (constraints) of the LCP in one precision.  SoA with leading
// dimension ld: n, ta = r_a x n, tb = r_b x n have 3 comps each.
template <typename T>
struct RowsT {
    int m, ld;
    const int *ia, *ib;
    const T *n, *ta, *tb;
    const T *qv;  // constant term of g = qv + dt D^T K D gamma
    const T *dA;  // diagonal of A = dt D^T K D
    T *gam, *g;
};

// Bodies for the LCP: operator K (9 comps: kt xyz, Kr xx yy zz xy xz yz),
// contact-induced velocity vc = K D gamma (6 comps), CSR of incident rows
// (entry = row << 1 | side, side 0 = body a, 1 = body b).
template <typename T>
struct BodiesT {
    int nb, ld;
    const T *K;
    T *vc;
    const int *off, *ent;
};

struct RowBuildArgs {
    int nsel;
    const int *sel;  // selected pair indices
    const int *pa, *pb;
    const double *snsd;  // 10 comps, ld = ldp
    int ldp;
    int m0;              // first row written
    int rec;             // recursion at which the rows are generated
    double dt;
    const double *K;     // 9 comps, ld = ldb
    const double *vfree; // 6 comps
    const double *vc;    // 6 comps (new rows: V_n - U_free) or null (iteration-0 rows)
    int ldb;
    // warm start from the previous step (sorted pair list) or null
    int nprev;
    const int *prev_a, *prev_b;
    const double *prev_lam;
    // outputs, ld = ldr
    int ldr;
    int *ia, *ib, *pair, *rec_out;
    double *n64, *ta64, *tb64, *qv64, *dA64, *gam64, *phi64;
    float *n32, *ta32, *tb32, *qv32, *dA32, *gam32;
};

void launch_rows_build(const RowBuildArgs &a, hipStream_t s);
void launch_compact(int n, const int *flags, const int *scanned, int *out, hipStream_t s);
void launch_csr(int nb, int m, const int *ia, const int *ib, int *cnt, int *off, int *cursor, int *ent,
                DBuf<int> &scan_scratch, hipStream_t s);

// Device control block of one solve: ping-pong states S[0], S[1], the
// final state, the done flag and the gather's per-block partial sums.
struct PgdCtl {
    PgdState *S;
    PgdState *fin;
    int *done;
    double *partials;
    int nbg;
    double tol;
};

// Passes of the projected-gradient loop.  Iteration j (j = 1, 2, ...) is
// scatter(mode 1, par = j & 1) then gather(mode 1, par = j & 1); a solve
// starts with pgd_init, scatter(mode 0), gather(mode 0).  All mode-1
// passes return at once after convergence (done flag).
template <typename T>
void launch_lcp_scatter(int mode, const RowsT<T> &r, const BodiesT<T> &b, const PgdCtl &C, int par, hipStream_t s);
template <typename T>
void launch_lcp_gather(int mode, const RowsT<T> &r, const BodiesT<T> &b, double dt, const PgdCtl &C, int par,
                       hipStream_t s);
void launch_pgd_init(const PgdCtl &C, hipStream_t s);
void launch_pgd_finalize(const PgdCtl &C, int par, hipStream_t s);
int lcp_gather_blocks(int m);

// Resident mode: one workgroup per packing solves that packing's LCP in one
// launch.  Rows of packing p are rlist[roff[p] .. roff[p+1]).  out[p]
// receives the packing's final state.  block in {256, 512, 1024}; lds
// stages the velocities of a packing (6 lds_ld values) in LDS.  Returns 0,
// or -1 if the launch configuration is not available.
template <typename T>
struct ResidentArgs {
    RowsT<T> R;
    BodiesT<T> B;
    int npk;
    const int *boff, *roff, *rlist;
    double dt, tol;
    int cap;
    PgdState *out;
    int lds_ld;
};
template <typename T>
int launch_lcp_resident(const ResidentArgs<T> &a, int block, bool lds, hipStream_t s);
void launch_rows_per_packing(int m0, int m1, const int *ia, const int *body_batch, int *cnt, hipStream_t s);
void launch_rlist_merge(int m_old, int nv, const int *rlist_old, const int *ia, const int *body_batch,
                        const int *roff_old, const int *E, int *rlist_new, hipStream_t s);
void launch_add_arrays(int n, const int *a, const int *b, int *c, hipStream_t s);
void launch_iota(int n, int *v, hipStream_t s);

// gamma64 <- gamma32 ; gamma32 <- gamma64
void launch_promote(int m, const float *g32, double *g64, hipStream_t s);
void launch_demote(int m, const double *g64, float *g32, hipStream_t s);

// sum over rows of gamma (g - qv) = gamma^T A gamma, FP64, into out[0]
void launch_work(int m, const double *gam, const double *g, const double *qv, double *partials, unsigned *ticket,
                 double *out, hipStream_t s);

// lam[pair[r]] += gamma[r] for the rows generated at recursion `level`
void launch_pair_lambda(int m, const int *rec, const int *pair, const double *gam, int level, double *lam,
                        hipStream_t s);

int lcp_partials_needed(int m);

}  // namespace relcp
