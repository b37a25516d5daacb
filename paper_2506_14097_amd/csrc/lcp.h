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
    // K: 9 comps (ld); with kiso the mobility is diag(k0 I, k3 I) (overdamped
    // bodies in 3-D) and only comps 0 and 3 are read
    const T *K;
    int kiso = 0;
    T *vc;
    // incidence lists: body i's entries at ent[off[i]] .. before off[i + 1]
    // (CSR), or with lcnt the first lcnt[i] of them (lists in the slots of
    // longer ones, as filter_lists leaves them)
    const int *off, *ent;
    const int *lcnt = nullptr;
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
    int kiso;            // as BodiesT::kiso
    const double *vfree; // 6 comps, or null where U_free is zero
    const double *vc;    // 6 comps (new rows: V_n - U_free) or null (iteration-0 rows)
    int ldb;
    // warm start from the previous step (sorted pair list) or null; with
    // prev_direct the previous list is the current candidate list and the
    // pair's multiplier is prev_lam[pair] (no search)
    int nprev;
    const int *prev_a, *prev_b;
    const double *prev_lam;
    int prev_direct;
    // outputs, ld = ldr
    int ldr;
    int *ia, *ib, *pair, *rec_out;
    double *n64, *ta64, *tb64, *qv64, *dA64, *gam64, *phi64;
    float *n32, *ta32, *tb32, *qv32, *dA32, *gam32;  // n32, ta32, tb32, gam32 may be null (not written)
};

void launch_rows_build(const RowBuildArgs &a, hipStream_t s);
// The iteration-0 rows selected and built in one pass over the np candidate
// pairs (a.sel and a.nsel unused; rows a.m0 + k): flags (np) the selection,
// gcount the set flags of each group of 256 pairs; writes sel (row ->
// pair), pos (pair -> row or -1) and the row count to *total (a device
// int, host-mapped or not) and, if not null, to *total_dev as well.  Only
// for np <= select_rows_max_pairs() (nothing is launched past it, nor for
// np <= 0).  The rows need room for all np pairs.
int select_rows_max_pairs();
void launch_select_rows(const RowBuildArgs &a, int np, const int *flags, const int *gcount, int *sel, int *pos,
                        int *total, hipStream_t s, int *total_dev = nullptr);
// CSR of the rows at each body; cleared: cnt and cursor (2 (nb + 1) ints)
// are known to be zero (every build leaves them so).  rg (or null): also
// the row graph's entry count of each row with their sum (as
// launch_rowgraph_counts).
struct CsrRowGraphOut {
    int *count, *rcnt;
};
void launch_csr(int nb, int m, const int *ia, const int *ib, int *cnt, int *off, int *cursor, int *ent,
                bool cleared, DBuf<int> &scan_scratch, hipStream_t s, const CsrRowGraphOut *rg = nullptr);

// Device control block of one solve: ping-pong states S[0], S[1], the
// final state, the done flag and the per-block partial sums of the last
// pass (read by the next pass; the row-graph pass writes its own partials
// to a second buffer, `pout` of its launch).
struct PgdCtl {
    PgdState *S;
    PgdState *fin;
    int *done;
    double *partials;
    int nbg;
    double tol;
    // host-mapped mirrors of fin and done (or null), written with them
    PgdState *fin_h;
    int *done_h;
    // iterations without halving the best residual after which the solve
    // stops as stalled (0: never); set for FP32 solves, which an FP64 polish
    // continues
    int stall = 0;
};

// Row-graph form of the LCP matrix A = dt D^T K D off its diagonal: one
// entry per pair of distinct rows sharing a body and per shared body (two
// rows sharing both bodies have two entries); the diagonal is the rows'
// A_aa, applied by the pass itself.
// Sliced ELL with a fixed stride S: slice s holds rows [64 s, 64 s + 64),
// entry k of row r at 64 (s S + k) + r % 64, so that no load of the graph
// waits on another (no slice offsets).  A row with more than S entries does
// not fit: the assembly skips it and reports the overflow, and the passes
// read no entry of it (the solve is re-sized and restarted).
template <typename T>
struct RowGraphT {
    int m;
    int stride;  // S: entry slots per row
    const int *col;
    const T *val;
    size_t cap;  // entry slots allocated (at least 64 S per slice)
    const int *rcnt;  // entries of each row (slots past them are not written)
};

// Iteration state of a row seen by the rows it couples to: multiplier and
// scaled gradient h = g / A_rr (its projected step is max(0, gam - alpha h)).
template <typename T>
struct alignas(2 * sizeof(T)) RowStep {
    T gam, h;
};

struct RowGraphFill {
    int m, ldr;
    const int *ia, *ib;
    const double *n, *ta, *tb;
    int ldb;
    const double *K;   // 9 comps, ld = ldb
    int kiso;          // as BodiesT::kiso
    const int *off, *ent;
    const int *lcnt;   // list lengths (as BodiesT::lcnt), or null for CSR
    int nslots;        // incidence slots (one thread each): 2 m for CSR, off[nb] with lcnt
    // entries of each row: read (CSR: from the count pass), or with lcnt
    // formed here from the lists' lengths and written for the passes
    int *rcnt;
    const int *bsums;  // with lcnt: filter_lists' block sums of the entry count
    int nbsums;
    int stride;        // entry slots per row (RowGraphT)
    double dt;
    size_t cap;        // entry slots allocated
    int *count;        // device entry counter of the count pass (read here, then cleared for the next build)
    int *need;         // device: raised to the entry count of every row that does not fit (left otherwise)
    int *report;       // host-mapped: [1] entries, [2] set to 1 on overflow
    int *col;
    double *val64;
    float *val32;
};

int rowgraph_slices(int m);
// rcnt[r] = count of other rows at row r's two bodies (its entries);
// *count += their sum, unless count is null
void launch_rowgraph_counts(int m, const int *ia, const int *ib, const int *off, int *count, int *rcnt,
                            hipStream_t s);
void launch_rowgraph_fill(const RowGraphFill &a, hipStream_t s);
// One pass of the row-graph LCP loop over m rows with A in G and the
// diagonal dA.  mode 0: start, gamma0 = max(0, start) (FP64 start rounded to
// T), g at gamma0, and the control block C reset for a new solve; mode 1:
// iteration with parity par, reading the previous pass's state (zin, gin)
// and partials, writing (zout, gout) and its own partials pout; mode 2: the
// same iteration with the partials reduced first by a one-block launch
// (for passes over many blocks; identical iterates).  save (mode 0, or
// null): receives the start in FP64 (kept for a restart, or as the FP64
// multipliers when the start is an FP32 solve's state).
// The start gamma0 of a row-graph solve: gam64 (FP64 multipliers), or, with
// gam64 null, the final state of an FP32 row-graph solve widened to FP64 --
// z[fin.iter & 1], or z[last_par & 1] while its done flag is not set (the
// state k_rowstate_unpack would pick).
struct StartSrc {
    const double *gam64;
    const RowStep<float> *z[2];
    const PgdState *fin;
    const int *done;
    int last_par;
    // FP64 starts (or null): the start pass also writes what the unpack of
    // a solve that converges at its start would -- gamma (into the pass's
    // save array), g into g_final and the work's per-block partial sums into
    // work_final (work_blocks(m) slots) -- so that no unpack need follow
    double *g_final = nullptr;
    double *work_final = nullptr;
};
template <typename T>
void launch_lcp_spmv(int mode, const RowGraphT<T> &G, const T *qv, const T *dA, const StartSrc &start,
                     const RowStep<T> *zin, const T *gin, RowStep<T> *zout, T *gout, const PgdCtl &C, double *pout,
                     int par, hipStream_t s, double *save = nullptr);
// Parameters of a row-graph solve in device memory, read by k_spmv_dev:
// the passes of a solve are then identical launches (parity aside) and can
// be recorded once in a graph.  nbg = blocks of a pass over m rows; a pass
// stops the solve (done) once converged or after cap iterations.
template <typename T>
struct LcpDev {
    int m, nbg, cap;
    double tol;
    int stall;  // as PgdCtl::stall
    int stride;
    const int *col;
    const T *val;
    size_t slots;
    const int *rcnt;
    const T *qv, *dA;
    RowStep<T> *z[2];
    T *g[2];
    double *part[2];
    PgdState *S, *fin;
    int *done;
    PgdState *fin_h;
    int *done_h;
};
template <typename T>
void launch_set_lcpdev(LcpDev<T> *D, const LcpDev<T> &v, hipStream_t s);
// one iteration pass of parity par over a grid covering grid_rows rows (>= m)
template <typename T>
void launch_spmv_dev(const LcpDev<T> *D, int grid_rows, int par, hipStream_t s);
// An instantiated graph of k passes (k even; parities 1, 0, 1, ..., so a
// chunk starts at an odd iteration) over a grid covering grid_rows rows, all
// reading *D.  Returns 0, or -1 with *out = null.
template <typename T>
int make_spmv_graph(const LcpDev<T> *D, int grid_rows, int k, hipGraphExec_t *out);
// gamma, g <- the state of the pass that holds the final iterate (fin.iter &
// 1), or, while the done flag (if given) is not set, that of the last pass
// launched (parity last_par); gam64 (or null) <- the same gamma in FP64;
// work (or null): the per-block sums of gamma (g - qv) of launch_work
// (work_blocks(m) slots)
template <typename T>
void launch_rowstate_unpack(int m, const RowStep<T> *z0, const RowStep<T> *z1, const T *g0, const T *g1,
                            const PgdState *fin, const int *done, int last_par, T *gam, T *g, double *gam64,
                            hipStream_t s, const T *qv = nullptr, double *work = nullptr);
// whether launch_report_check can reduce the start pass of m rows (its
// partial sums fit one workgroup's registers)
bool unpack_can_check(int m);
// The tail report (report.h) after checking a solve of which only the start
// pass ran: its partial sums (C.partials) reduced in the order the first
// iteration pass would, the state advanced, and the final state and done
// flags recorded if the start meets the tolerance (else the caller finds the
// solve unfinished and continues it).  One workgroup.
struct TailReport;
void launch_report_check(const TailReport &R, const PgdCtl &C, hipStream_t s);

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
    int stall;  // as PgdCtl::stall
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

// gamma^T A gamma = sum over rows of gamma (g - qv), FP64, as work_blocks(m)
// per-block partial sums
int work_blocks(int m);
void launch_work(int m, const double *gam, const double *g, const double *qv, double *partials, hipStream_t s);

// lam[pair[r]] += gamma[r] for the rows generated at recursion `level`
void launch_pair_lambda(int m, const int *rec, const int *pair, const double *gam, int level, double *lam,
                        hipStream_t s);

int lcp_partials_needed(int m);

}  // namespace relcp
