// relcp.hip -- context, step orchestration and the C ABI of librelcp.
//
// One call of relcp_step runs Alg. 1 of Palmer, Aktulga, Gao (arXiv
// 2506.14097) -- or its inertial form, Eq. relcp_inertial -- on the GPU:
//   candidate pairs at C^k -> SNSD at C^k -> rows of A_0 -> LCP (BB-PGD)
//   -> trial C_{n+1} = C^k (+) dt V_n -> SNSD at C_{n+1} -> violators
//   Phi < -eps -> append pulled-back rows -> LCP ... -> accept.
// The host only launches kernels and reads back a few counters per
// recursion (pair count, violator count, convergence flag of the LCP).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/relcp.h"
#include "geometry.h"
#include "lcp.h"
#include "mlp.h"
#include "report.h"

static_assert(RELCP_MLP_NPARAM == relcp::MLP_NPARAM && RELCP_MLP_NORM == relcp::MLP_NORM, "model layout");

using namespace relcp;

namespace {

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

// (re)allocate an SoA buffer of `comps` components with leading dimension
// new_ld, keeping the first `keep` items of each component
template <typename T>
void realloc_soa(DBuf<T> &b, int comps, size_t old_ld, size_t new_ld, size_t keep, hipStream_t s) {
    T *np_ = nullptr;
    if (hipMalloc(&np_, std::max<size_t>(1, new_ld * comps) * sizeof(T)) != hipSuccess)
        throw Error{RELCP_E_OOM, "device allocation failed"};
    if (b.p && keep) {
        for (int k = 0; k < comps; ++k)
            HIP_OK(hipMemcpyAsync(np_ + k * new_ld, b.p + k * old_ld, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    if (b.p) HIP_OK(hipFree(b.p));
    b.p = np_;
    b.cap = new_ld * comps;
}

__global__ void k_bbox(int nb, const double *__restrict__ x, int ldx, const int *__restrict__ body_batch,
                       unsigned long long *__restrict__ keys) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    int pk = body_batch ? body_batch[i] : 0;
    for (int k = 0; k < 3; ++k) {
        double v = x[k * ldx + i];
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        unsigned long long key = (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
        atomicMin(keys + 6 * pk + k, key);
        atomicMax(keys + 6 * pk + 3 + k, key);
    }
}

__global__ void k_aos_to_soa(int n, int comps, const double *__restrict__ in, double *__restrict__ out, int ld) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < comps; ++k) out[k * ld + i] = in[(size_t)comps * i + k];
}
__global__ void k_soa_to_aos(int n, int comps, const double *__restrict__ in, int ld, int c0, double *__restrict__ out,
                             int ocomps, const int *__restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t o = (size_t)ocomps * perm[i];
    for (int k = 0; k < ocomps; ++k) out[o + k] = in[(c0 + k) * ld + i];
}
__global__ void k_scale(int n, double *__restrict__ x, int nbox, double *__restrict__ box, double s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= s;
    if (i < nbox) box[i] *= s;
}

int env_int(const char *name, int dflt, int lo = 1) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    const long x = std::strtol(v, &end, 10);
    return (end && *end == 0 && x >= lo && x < (1L << 30)) ? (int)x : dflt;
}

struct Timer {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    double ms() {
        auto now = std::chrono::steady_clock::now();
        double v = std::chrono::duration<double, std::milli>(now - t).count();
        t = now;
        return v;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// small bookkeeping kernels of the step
// ---------------------------------------------------------------------------
namespace {
// The tail report as its own kernel (used where no compaction runs).
__global__ void __launch_bounds__(256) k_report(TailReport R) { tail_report(R); }
}  // namespace

// ===========================================================================
// context
// ===========================================================================
struct relcp_ctx {
    // configuration
    int n = 0, nbatch = 1;
    int dynamics = 0, precision = 64, warm_start = 1, planar = 0, max_rec = 64, lcp_max_iters = 100000,
        lcp_fixed = 0;
    double skin = 0.05;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<int> boff;      // nbatch + 1
    std::vector<double> box;    // 3 nbatch
    std::vector<double> rmax;   // nbatch
    bool has_fext = false;
    // overdamped bodies: K, K32, Rb and U_free are constant and the geometry
    // at C^k is the accepted trial's (geo and geot swap on acceptance), so
    // the set-up pass runs only after the bodies or forces change
    bool setup_valid = false;

    // bodies (SoA, ld = n)
    DBuf<double> x, q, u, p, rho, fext, xt, qt, geo, geot, Rb, K, vfree, vc64, vout, boxes;
    DBuf<float> K32, vc32;
    DBuf<int> kind, body_batch, perm_d;
    std::vector<int> perm, inv;  // internal -> caller index, caller -> internal

    // broadphase
    DBuf<PackGrid> grids;
    DBuf<int> body_cell, cell_count, cell_start, cell_cursor, cell_items, pair_count, pair_off;
    DBuf<unsigned long long> keys;
    std::vector<PackGrid> grids_h;

    // pairs (ld = ldp)
    int np = 0, ldp = 0;
    const int *csr_clear = nullptr;      // csr_cnt while its counters are known to be zero
    DBuf<int> pa, pb, pflag, pcnt, sel;  // pcnt: set flags per block of 256 pairs
    DBuf<double> snsd0, snsdt, lam;
    // previous step (warm start): sorted pairs and multiplier sums
    int nprev = 0, ldprev = 0;
    DBuf<int> prev_a, prev_b;
    // the candidate list pa, pb is kept across steps (a Verlet list): built
    // with bounding-sphere gap and centre-line support gap (a lower bound of
    // Phi) both <= skin + 2 margin, it holds every pair within skin as long
    // as the accumulated bound on how much any gap has shrunk since the build
    // (vl_used) stays below 2 margin; pairs of the list beyond skin are cut by
    // a bounding-sphere test in the narrowphase
    bool vl_valid = false, prev_is_list = false;
    bool hint_ok = false;  // snsdt holds the normals of the last accepted trial for the current list
    double vl_used = 0.0;
    double vl_margin() const { return 0.5 * skin; }
    double vl_radius() const { return skin + 2.0 * vl_margin(); }
    void candidate_pairs(relcp_step_stats &S);
    DBuf<double> prev_lam;

    // rows (ld = ldr)
    int m = 0, ldr = 0, m_acc = 0;
    DBuf<int> ria, rib, rpair, rrec;
    DBuf<double> rn64, rta64, rtb64, rqv64, rdA64, rgam64, rg64, rphi64;
    DBuf<float> rn32, rta32, rtb32, rqv32, rdA32, rgam32, rg32;
    DBuf<int> csr_cnt, csr_off, csr_cur, csr_ent;
    // incidence lists of the candidate pairs (entries (pair << 1) | side, each
    // body's in pair order), built once per candidate list; the step's first
    // rows are the selected pairs in pair order, so their lists are these
    // lists filtered through prow (the pair's row, or -1), already in row
    // order: no atomics and no sort per step
    DBuf<int> pcsr_cnt, pcsr_off, pcsr_ent, prow, fl_cnt, fl_bsums;
    // the incidence lists are the first rows' filtered ones (in the candidate
    // lists' slots, lengths fl_cnt) rather than rebuild_csr's CSR
    bool lists_gapped = false;
    bool pcsr_valid = false;
    const int *pcsr_clear = nullptr;  // pcsr_cnt while its counters are known to be zero

    // LCP state and reductions
    DBuf<PgdState> pst;
    DBuf<double> partials, work_out;
    DBuf<unsigned long long> red;  // per-block trial results: displacement bits, then min-Phi and margin keys
    DBuf<int> scan_scratch, dtotal;
    // optional kernel timing (HIP events on the stream)
    static constexpr int kClasses = 12;
    static constexpr int kIdlePass = 9;  // row-graph passes launched after the solve had finished
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_class;
    struct PassEv {
        size_t slot;
        int j, pk;
    };
    std::vector<PassEv> pass_ev;  // (event pair, pass, precision) of the current row-graph solves
    size_t ev_used = 0;
    long long t_count[kClasses] = {};
    double t_ms[kClasses] = {};
    void ev_reserve() {
        if (ev_used + 2 > ev_pool.size()) {
            for (int k = 0; k < 256; ++k) {
                hipEvent_t e;
                HIP_OK(hipEventCreate(&e));
                ev_pool.push_back(e);
            }
            ev_class.resize(ev_pool.size() / 2);
        }
    }
    // when timing is on, time the one kernel that `f` launches through
    // launch_k by the dispatch's own start and end (nothing is counted if f
    // launches none)
    template <typename F>
    void timed(int cls, F &&f) {
        if (!timing) {
            f();
            return;
        }
        ev_reserve();
        LaunchEvents &a = armed_launch_events();
        a = LaunchEvents{ev_pool[ev_used], ev_pool[ev_used + 1]};
        f();
        if (a.start) {
            a = LaunchEvents{};
            return;
        }
        ev_class[ev_used / 2] = cls;
        ev_used += 2;
    }
    // an event pair recorded on the stream around f (a graph launch): the
    // span includes any wait of the stream for the host between the two
    template <typename F>
    void timed_span(int cls, F &&f) {
        if (!timing) {
            f();
            return;
        }
        ev_reserve();
        HIP_OK(hipEventRecord(ev_pool[ev_used], stream));
        f();
        HIP_OK(hipEventRecord(ev_pool[ev_used + 1], stream));
        ev_class[ev_used / 2] = cls;
        ev_used += 2;
    }
    // fold the recorded pairs into the totals (stream must be idle)
    void collect_timing() {
        for (size_t k = 0; k + 1 < ev_used; k += 2) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, ev_pool[k], ev_pool[k + 1]));
            int c = ev_class[k / 2];
            t_count[c] += 1;
            t_ms[c] += ms;
        }
        ev_used = 0;
    }

    // pinned host mirrors
    // small host buffers written by kernels directly (mapped, coherent; read
    // after the stream is synchronised) and their device addresses
    PgdState *pst_h = nullptr, *pst_d = nullptr;  // fin and the done slot
    int last_iters[2] = {8, 8};  // previous solve's iteration count (FP32, FP64)
    int zero_run[2] = {0, 0};    // solves in a row that converged at their start pass
    // LCP execution: mode 0 = automatic, 1 = grid (two passes per iteration
    // over all rows), 2 = resident (one workgroup per packing, one launch),
    // 3 = row graph (A assembled over rows, one pass per iteration)
    int lcp_mode = 0, res_block = 256, res_lds = 1;
    DBuf<int> rg_col, rg_flags;  // flags: [0] entry count, [1] largest count of a row that did not fit
    DBuf<int> rg_rcnt;  // entries of each row
    DBuf<double> rg_val64;
    DBuf<float> rg_val32;
    DBuf<RowStep<double>> z64;
    DBuf<RowStep<float>> z32;
    DBuf<double> zg64;
    DBuf<float> zg32;
    bool rg_valid = false;
    double rg_dt = 0.0;
    // row-graph passes replayed from an instantiated graph (per precision):
    // parameters in device memory, grid covering graph_rows rows
    static constexpr int kGraphPasses = 8;
    // iteration passes over at least this many blocks reduce the last pass's
    // partial sums in a separate one-block launch (RELCP_REDUCE_SPLIT_BLOCKS)
    // (at most 1024: a pass that reduces by itself holds the partial sums of
    // up to 4 x 256 blocks in registers)
    int reduce_split_blocks = std::min(1024, env_int("RELCP_REDUCE_SPLIT_BLOCKS", 1024));
    // the row graph's entry slots per row, at first RELCP_RG_SLOTS_PER_ROW: an
    // assembly with a row that does not fit raises it and restarts its solve
    int rg_stride = env_int("RELCP_RG_SLOTS_PER_ROW", 16);
    // the first rows' incidence lists filtered from the candidate pairs' (1)
    // or built from the rows (0) (RELCP_FIRST_LISTS); the same lists
    int first_lists = env_int("RELCP_FIRST_LISTS", 1, 0);
    // the iteration-0 rows selected and built in one pass (1) or compacted
    // first (0) (RELCP_FUSED_SELECT); the same rows
    int fused_select = env_int("RELCP_FUSED_SELECT", 1, 0);
    // an FP32 solve whose residual has not halved in this many iterations
    // stops (its rounding floor is above the tolerance) and the FP64
    // polish continues from its last iterate; fixed-iteration runs never stop
    template <typename T>
    int stall_iters() const {
        return sizeof(T) == 4 && lcp_fixed == 0 ? 400 : 0;
    }
    int rg_restarts = 0;  // of the current step
    DBuf<LcpDev<double>> lcpdev64;
    DBuf<LcpDev<float>> lcpdev32;
    hipGraphExec_t spmv_graph[2] = {nullptr, nullptr};
    int graph_rows[2] = {0, 0};
    bool graph_ok = true;
    template <typename T>
    hipGraphExec_t spmv_graph_for(int rows, LcpDev<T> **dev);
    size_t rg_cap = 0;     // entry slots allocated
    int rg_entries = 0;    // entries of the current graph (known after the solve's first read-back)
    bool rowgraph_mode() const { return !resident_mode() && lcp_mode != 1; }
    // K as the body set-up forms it for overdamped bodies in 3-D:
    // diag(k0 I, k3 I), so that kernels read components 0 and 3 only (false
    // where the caller supplies K)
    bool k_from_setup = true;
    // the rows' FP32 geometry (n, ta, tb) is current (rows built for the row
    // graph leave it out; a matrix-free FP32 solve forms it first)
    bool rows32_ok = false;
    bool k_iso() const { return k_from_setup && dynamics == RELCP_OVERDAMPED && !planar; }
    void build_rowgraph(double dt);
    void rg_reserve(size_t slots);
    void rg_prepare(int mcap = -1);  // buffers for mcap rows (default m)
    bool rg_pre = false;  // the incidence build made this graph's entry counts
    int maxpk = 0;                       // bodies of the largest packing
    DBuf<int> boff_d, roff, rlist, rlist2, rcnt, rE;
    DBuf<PgdState> pk_state;
    PgdState *pk_state_h = nullptr;
    // automatic choice: one workgroup per packing suits many packings or
    // small ones; a few large packings leave most of the GPU idle there and
    // run their passes over many workgroups instead
    bool resident_mode() const {
        if (lcp_mode == 1 || lcp_mode == 3 || lcp_mode == 4) return false;
        if (lcp_mode == 2) return true;
        return maxpk <= 256 || (maxpk <= 8192 && nbatch >= 32);
    }
    void rows_by_packing_init(int m0);
    void rows_by_packing_append(int m_old, int nv);
    // learned warm start: model (fp32 master weights + standardisation),
    // features of the iteration-0 rows, contact log of the last accepted step
    bool has_model = false, log_on = false, log_valid = false;
    bool has_torus = false;  // some body is a torus (no learned warm start then)
    bool all_torus = false;  // every body is a torus (the SNSD kernel built for tori alone)
    float mlp_norm[MLP_NORM] = {};
    DBuf<float> mlp_w, feat;
    DBuf<double> rowscale;
    int m0_last = 0;
    int *int_h = nullptr;
    unsigned long long *red_h = nullptr, *red_hd = nullptr;
    double *dbl_h = nullptr, *dbl_hd = nullptr;
    int *int_d = nullptr;
    // host-mapped token written last by the report kernel of a recursion
    int *tok_h = nullptr, *tok_d = nullptr;
    int tok_seq = 0;
    void alloc_host();

    ~relcp_ctx() {
        DBuf<double> *ds[] = {&x, &q, &u, &p, &rho, &fext, &xt, &qt, &geo, &geot, &Rb, &K, &vfree, &vc64, &vout,
                              &boxes, &snsd0, &snsdt, &lam, &prev_lam, &rn64, &rta64, &rtb64, &rqv64, &rdA64,
                              &rgam64, &rg64, &rphi64, &partials, &work_out};
        for (auto *b : ds) b->release();
        DBuf<float> *fs[] = {&K32, &vc32, &rn32, &rta32, &rtb32, &rqv32, &rdA32, &rgam32, &rg32};
        for (auto *b : fs) b->release();
        DBuf<int> *is[] = {&kind, &body_batch, &perm_d, &body_cell, &cell_count, &cell_start, &cell_cursor, &cell_items,
                           &pair_count, &pair_off, &pa, &pb, &pflag, &pcnt, &sel, &prev_a, &prev_b, &ria, &rib,
                           &rpair, &rrec, &csr_cnt, &csr_off, &csr_cur, &csr_ent, &scan_scratch, &dtotal,
                           &pcsr_cnt, &pcsr_off, &pcsr_ent, &prow, &fl_cnt, &fl_bsums};
        for (auto *b : is) b->release();
        grids.release();
        keys.release();
        pst.release();
        red.release();
        if (pst_h) (void)hipHostFree(pst_h);
        if (int_h) (void)hipHostFree(int_h);
        if (red_h) (void)hipHostFree(red_h);
        if (dbl_h) (void)hipHostFree(dbl_h);
        if (tok_h) (void)hipHostFree(tok_h);
        if (pk_state_h) (void)hipHostFree(pk_state_h);
        gam_save.release();
        boff_d.release(); roff.release(); rlist.release(); rlist2.release(); rcnt.release(); rE.release();
        pk_state.release();
        mlp_w.release(); feat.release(); rowscale.release();
        rg_col.release(); rg_flags.release(); rg_val64.release();
        rg_rcnt.release();
        rg_val32.release(); z64.release(); z32.release(); zg64.release(); zg32.release();
        lcpdev64.release(); lcpdev32.release();
        for (auto &ge : spmv_graph)
            if (ge) (void)hipGraphExecDestroy(ge);
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    // ---------------------------------------------------------------------
    void upload_bodies(const relcp_bodies *B, const relcp_shapes *S);
    void ensure_pairs(int need);
    void ensure_rows(int need);
    void broadphase(const double *xs, double skin_, bool bound = false);
    void build_rows(int nsel, int rec, const double *snsd, const double *vc, bool warm, double dt);
    RowBuildArgs row_args(int nsel, int rec, const double *snsd, const double *vc, bool warm, double dt);
    void rebuild_csr();
    void first_rows_csr(int mcap);
    void warm_start_rows(int m0, double dt);
    template <typename T>
    int solve(double dt, double tol, int &iters, double &res);
    template <typename T>
    RowsT<T> rows_of() const;
    template <typename T>
    BodiesT<T> bodies_of() const;
    template <typename T>
    int solve_rowgraph(const RowsT<T> &R, const BodiesT<T> &Bd, double dt, double tol, int &iters, double &res);
    template <typename T>
    int solve_rowgraph_graph(const RowsT<T> &R, const BodiesT<T> &Bd, double dt, double tol, int &iters,
                             double &res);
    // pieces of a row-graph solve with one launch per pass (per precision)
    struct RgRun {
        int j = 1, chunk = 2, pass_mode = 1;
        bool fresh = false;  // the graph was assembled by this solve's start
        // the FP64 polish ran only its start pass, which wrote the unpack's
        // results; the tail's report checks its convergence
        bool final_start = false;
    };
    RgRun rgr[2];
    template <typename T>
    struct RgBufs {
        RowStep<T> *z0, *z1;
        T *g0, *g1;
        double *part;
        size_t stride;
        PgdCtl C;
        RowGraphT<T> G;
    };
    template <typename T>
    RgBufs<T> rg_bufs(const RowsT<T> &R, double tol);
    template <typename T>
    void rg_passes(const RgBufs<T> &B, const RowsT<T> &R, int k);
    template <typename T>
    void rg_start(const RowsT<T> &R, double dt, double tol, const double *gam0, double *save,
                  const StartSrc *src = nullptr, bool allow_final = false);
    DBuf<double> gam_save;  // the start of the first solve of a recursion, for a restart
    template <typename T>
    void rg_unpack(const RowsT<T> &R, const BodiesT<T> &Bd, double tol);
    template <typename T>
    int rg_finish(const RowsT<T> &R, const BodiesT<T> &Bd, double tol, int &iters, double &res, bool &relaunched);
    bool rg_overflowed();
    int step(double dt, double eps, double tol, relcp_step_stats *st);
    // host waits on the stream (counted per step)
    int n_waits = 0;
    double t_wait = 0.0;
    void sync() {
        Timer t;
        HIP_OK(hipStreamSynchronize(stream));
        t_wait += t.ms();
        ++n_waits;
    }
    // Wait until a kernel has written a host-mapped int (coherent memory,
    // written with plain stores) different from `unset`, by polling it:
    // waking on the stream's completion costs 5-20 us more per wait.  After
    // 10 s without it, the stream is synchronised (which reports a failed
    // kernel) and the value read as it is.
    int wait_mapped(const int *h, int unset) {
        Timer t;
        const auto t0 = std::chrono::steady_clock::now();
        int v;
        int spins = 0;
        while ((v = __atomic_load_n(h, __ATOMIC_ACQUIRE)) == unset) {
            if (++spins == 4096) {
                spins = 0;
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) {
                    HIP_OK(hipStreamSynchronize(stream));
                    v = __atomic_load_n(h, __ATOMIC_ACQUIRE);
                    break;
                }
            }
        }
        t_wait += t.ms();
        ++n_waits;
        return v;
    }
    // the report kernel's token of the last recursion launched
    void wait_report() {
        if (wait_mapped(tok_h, tok_seq - 1) != tok_seq) throw Error{RELCP_E_DEVICE, "report token not written"};
    }
};

template <typename T>
static T *host_mapped(size_t n, T **dev) {
    void *h = nullptr, *d = nullptr;
    HIP_OK(hipHostMalloc(&h, n * sizeof(T), hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(h, 0, n * sizeof(T));
    HIP_OK(hipHostGetDevicePointer(&d, h, 0));
    *dev = static_cast<T *>(d);
    return static_cast<T *>(h);
}

void relcp_ctx::alloc_host() {
    if (!pst_h) pst_h = host_mapped<PgdState>(4, &pst_d);  // final state and done flag per precision
    if (!int_h) int_h = host_mapped<int>(16, &int_d);
    if (!red_h) red_h = host_mapped<unsigned long long>(8, &red_hd);
    if (!dbl_h) dbl_h = host_mapped<double>(8, &dbl_hd);
    if (!tok_h) tok_h = host_mapped<int>(1, &tok_d);
}

// ---------------------------------------------------------------------------
// validation and upload
// ---------------------------------------------------------------------------
// Bounding radius of a shape: largest semiaxis, l/2 + r, or R + r.
static double bound_radius(int kind, const double *pp) {
    if (kind == RELCP_ELLIPSOID) return std::max(pp[0], std::max(pp[1], pp[2]));
    if (kind == RELCP_TORUS) return pp[0] + pp[1];
    return 0.5 * pp[1] + pp[0];
}

static void validate(const relcp_bodies *B, const relcp_shapes *S, const relcp_params *P, double skin) {
    if (!B || !S || !B->x || !B->q || !S->kind || !S->p || !S->rho_or_xi) throw Error{RELCP_E_INVALID, "null input"};
    if (B->n <= 0) throw Error{RELCP_E_INVALID, "need at least one body"};
    int nbt = B->n_batch <= 0 ? 1 : B->n_batch;
    if (nbt > 1 && !B->batch_off) throw Error{RELCP_E_INVALID, "batch_off required for n_batch > 1"};
    if (B->batch_off) {
        if (B->batch_off[0] != 0 || B->batch_off[nbt] != B->n) throw Error{RELCP_E_INVALID, "bad batch offsets"};
        for (int k = 0; k < nbt; ++k)
            if (B->batch_off[k + 1] <= B->batch_off[k]) throw Error{RELCP_E_INVALID, "empty or unordered packing"};
    }
    for (int i = 0; i < B->n; ++i) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(B->x[3 * i + k])) throw Error{RELCP_E_INVALID, "non-finite position"};
        double qn = 0;
        for (int k = 0; k < 4; ++k) {
            if (!std::isfinite(B->q[4 * i + k])) throw Error{RELCP_E_INVALID, "non-finite quaternion"};
            qn += B->q[4 * i + k] * B->q[4 * i + k];
        }
        if (std::fabs(std::sqrt(qn) - 1.0) > 1e-10) throw Error{RELCP_E_INVALID, "quaternion not of unit norm"};
        int kd = S->kind[i];
        const double *pp = S->p + 3 * i;
        if (kd == RELCP_ELLIPSOID) {
            if (!(pp[0] > 0 && pp[1] > 0 && pp[2] > 0)) throw Error{RELCP_E_INVALID, "semiaxes must be positive"};
        } else if (kd == RELCP_SPHEROCYLINDER) {
            if (!(pp[0] > 0 && pp[1] >= 0)) throw Error{RELCP_E_INVALID, "bad spherocylinder radius or length"};
            if (P && P->dynamics == RELCP_INERTIAL)
                throw Error{RELCP_E_INVALID, "inertial dynamics needs ellipsoids (mass properties)"};
        } else if (kd == RELCP_TORUS) {
            if (!(pp[0] >= 0 && pp[1] > 0 && std::isfinite(pp[0]) && std::isfinite(pp[1])))
                throw Error{RELCP_E_INVALID, "bad torus radii (R >= 0, r > 0)"};
            if (P && P->dynamics == RELCP_INERTIAL)
                throw Error{RELCP_E_INVALID, "inertial dynamics needs ellipsoids (mass properties)"};
            if (P && P->planar) throw Error{RELCP_E_INVALID, "tori are not supported in a monolayer"};
        } else {
            throw Error{RELCP_E_INVALID, "unknown shape kind"};
        }
        if (!(S->rho_or_xi[i] > 0) || !std::isfinite(S->rho_or_xi[i]))
            throw Error{RELCP_E_INVALID, "density / drag must be positive"};
        if (B->u)
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(B->u[3 * i + k])) throw Error{RELCP_E_INVALID, "non-finite velocity"};
        if (B->w)
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(B->w[3 * i + k])) throw Error{RELCP_E_INVALID, "non-finite angular velocity"};
    }
    for (int pk = 0; pk < nbt; ++pk) {
        int b0 = B->batch_off ? B->batch_off[pk] : 0, b1 = B->batch_off ? B->batch_off[pk + 1] : B->n;
        double R = 0;
        for (int i = b0; i < b1; ++i) {
            if (S->kind[i] != S->kind[b0]) throw Error{RELCP_E_INVALID, "one shape kind per packing"};
            const double *pp = S->p + 3 * i;
            R = std::max(R, bound_radius(S->kind[i], pp));
        }
        for (int k = 0; k < 3; ++k) {
            double L = B->box ? B->box[3 * pk + k] : 0.0;
            if (!(L >= 0) || !std::isfinite(L)) throw Error{RELCP_E_INVALID, "bad box"};
            if (L > 0 && L < 2.0 * (R + skin))
                throw Error{RELCP_E_INVALID, "periodic box smaller than 2 (R_max + skin)"};
        }
    }
}

// Bodies are stored in the order of a Morton (Z-order) curve over a grid
// of their positions, packing by packing, so that bodies close in space are
// close in memory: neighbouring lanes then touch neighbouring cache lines in
// every pass (pairs, SNSD, LCP scatter and gather).  perm[i] is the caller's
// index of internal body i.
static uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

void relcp_ctx::upload_bodies(const relcp_bodies *B, const relcp_shapes *S) {
    n = B->n;
    csr_clear = nullptr;
    pcsr_clear = nullptr;
    pcsr_valid = false;
    lists_gapped = false;
    log_valid = false;
    vl_valid = false;
    prev_is_list = false;
    hint_ok = false;
    nbatch = B->n_batch <= 0 ? 1 : B->n_batch;
    boff.assign(nbatch + 1, 0);
    for (int k = 0; k <= nbatch; ++k) boff[k] = B->batch_off ? B->batch_off[k] : (k ? n : 0);
    box.assign(3 * nbatch, 0.0);
    if (B->box)
        for (int k = 0; k < 3 * nbatch; ++k) box[k] = B->box[k];
    rmax.assign(nbatch, 0.0);
    has_torus = false;
    all_torus = true;
    std::vector<int> bb(n);
    for (int pk = 0; pk < nbatch; ++pk)
        for (int i = boff[pk]; i < boff[pk + 1]; ++i) {
            bb[i] = pk;
            const double *pp = S->p + 3 * i;
            rmax[pk] = std::max(rmax[pk], bound_radius(S->kind[i], pp));
            if (S->kind[i] == RELCP_TORUS)
                has_torus = true;
            else
                all_torus = false;
        }
    // spatial order inside each packing
    perm.resize(n);
    for (int pk = 0; pk < nbatch; ++pk) {
        int b0 = boff[pk], b1 = boff[pk + 1];
        double lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = 1e300;
            hi[k] = -1e300;
        }
        for (int i = b0; i < b1; ++i)
            for (int k = 0; k < 3; ++k) {
                double v = B->x[3 * i + k];
                if (box[3 * pk + k] > 0) v -= box[3 * pk + k] * std::floor(v / box[3 * pk + k]);
                lo[k] = std::min(lo[k], v);
                hi[k] = std::max(hi[k], v);
            }
        double cell = std::max(1e-12, rmax[pk]);
        std::vector<std::pair<uint64_t, int>> key(b1 - b0);
        for (int i = b0; i < b1; ++i) {
            uint64_t code = 0;
            for (int k = 0; k < 3; ++k) {
                double v = B->x[3 * i + k];
                if (box[3 * pk + k] > 0) v -= box[3 * pk + k] * std::floor(v / box[3 * pk + k]);
                double c = std::floor((v - lo[k]) / cell);
                uint64_t ci = (uint64_t)std::min(std::max(c, 0.0), 2097151.0);
                code |= spread3(ci) << k;
            }
            key[i - b0] = {code, i};
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<uint64_t, int> &a, const std::pair<uint64_t, int> &b) {
                             return a.first < b.first;
                         });
        for (int i = b0; i < b1; ++i) perm[i] = key[i - b0].second;
    }
    inv.resize(n);
    for (int i = 0; i < n; ++i) inv[perm[i]] = i;
    size_t N = (size_t)n;
    auto alloc = [&](auto &b, int comps) {
        b.release();
        b.ensure(N * comps);
        b.cap = N * comps;  // ld = n exactly
    };
    alloc(x, 3); alloc(q, 4); alloc(u, 6); alloc(p, 3); alloc(rho, 1); alloc(fext, 6); alloc(xt, 3); alloc(qt, 4);
    alloc(geo, 6); alloc(geot, 6); alloc(Rb, 1); alloc(K, 9); alloc(vfree, 6); alloc(vc64, 6); alloc(vout, 6);
    alloc(K32, 9); alloc(vc32, 6); alloc(kind, 1); alloc(body_batch, 1); alloc(perm_d, 1);
    // host transposes to SoA in internal order
    std::vector<double> t(6 * N, 0.0);
    auto up = [&](const double *src, int comps, int c0, int stride) {
        for (size_t i = 0; i < N; ++i)
            for (int k = 0; k < comps; ++k) t[(c0 + k) * N + i] = src ? src[(size_t)stride * perm[i] + k] : 0.0;
    };
    up(B->x, 3, 0, 3);
    HIP_OK(hipMemcpyAsync(x.p, t.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, stream));
    sync();
    up(B->q, 4, 0, 4);
    HIP_OK(hipMemcpyAsync(q.p, t.data(), 4 * N * sizeof(double), hipMemcpyHostToDevice, stream));
    sync();
    up(B->u, 3, 0, 3);
    up(B->w, 3, 3, 3);
    HIP_OK(hipMemcpyAsync(u.p, t.data(), 6 * N * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(vout.p, t.data(), 6 * N * sizeof(double), hipMemcpyHostToDevice, stream));
    sync();
    up(S->p, 3, 0, 3);
    HIP_OK(hipMemcpyAsync(p.p, t.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, stream));
    sync();
    std::vector<double> rh(N);
    std::vector<int> kh(N), bh(N);
    for (size_t i = 0; i < N; ++i) {
        rh[i] = S->rho_or_xi[perm[i]];
        kh[i] = S->kind[perm[i]];
        bh[i] = bb[perm[i]];
    }
    HIP_OK(hipMemcpyAsync(rho.p, rh.data(), N * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(kind.p, kh.data(), N * sizeof(int), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(body_batch.p, bh.data(), N * sizeof(int), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(perm_d.p, perm.data(), N * sizeof(int), hipMemcpyHostToDevice, stream));
    boxes.ensure(3 * nbatch);
    HIP_OK(hipMemcpyAsync(boxes.p, box.data(), 3 * nbatch * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemsetAsync(fext.p, 0, 6 * N * sizeof(double), stream));
    boff_d.ensure(nbatch + 1);
    HIP_OK(hipMemcpyAsync(boff_d.p, boff.data(), (nbatch + 1) * sizeof(int), hipMemcpyHostToDevice, stream));
    maxpk = 0;
    for (int pk = 0; pk < nbatch; ++pk) maxpk = std::max(maxpk, boff[pk + 1] - boff[pk]);
    roff.ensure(nbatch + 2);
    rcnt.ensure(nbatch + 2);
    rE.ensure(nbatch + 2);
    pk_state.ensure(nbatch);
    if (pk_state_h) HIP_OK(hipHostFree(pk_state_h));
    HIP_OK(hipHostMalloc((void **)&pk_state_h, nbatch * sizeof(PgdState), hipHostMallocDefault));
    has_fext = false;
    setup_valid = false;
    nprev = 0;
    m = 0;
    m_acc = 0;
    sync();
}

void relcp_ctx::ensure_pairs(int need) {
    if (need <= ldp) return;
    size_t nld = std::max<size_t>((size_t)need + need / 4 + 1024, 2 * (size_t)ldp);
    pa.release(); pb.release(); pflag.release(); pcnt.release(); sel.release();
    snsd0.release(); snsdt.release(); lam.release();
    pa.ensure(nld); pb.ensure(nld); pflag.ensure(nld + 1); pcnt.ensure(snsd_blocks((int)nld) + 1); sel.ensure(nld);
    snsd0.ensure(10 * nld); snsdt.ensure(10 * nld); lam.ensure(nld);
    ldp = (int)nld;
}

void relcp_ctx::ensure_rows(int need) {
    if (need <= ldr) return;
    size_t old = ldr, nld = std::max<size_t>((size_t)need + need / 2 + 1024, 2 * (size_t)ldr);
    realloc_soa(ria, 1, old, nld, m, stream);
    realloc_soa(rib, 1, old, nld, m, stream);
    realloc_soa(rpair, 1, old, nld, m, stream);
    realloc_soa(rrec, 1, old, nld, m, stream);
    realloc_soa(rn64, 3, old, nld, m, stream);
    realloc_soa(rta64, 3, old, nld, m, stream);
    realloc_soa(rtb64, 3, old, nld, m, stream);
    realloc_soa(rqv64, 1, old, nld, m, stream);
    realloc_soa(rdA64, 1, old, nld, m, stream);
    realloc_soa(rgam64, 1, old, nld, m, stream);
    realloc_soa(rg64, 1, old, nld, m, stream);
    realloc_soa(rphi64, 1, old, nld, m, stream);
    realloc_soa(rn32, 3, old, nld, m, stream);
    realloc_soa(rta32, 3, old, nld, m, stream);
    realloc_soa(rtb32, 3, old, nld, m, stream);
    realloc_soa(rqv32, 1, old, nld, m, stream);
    realloc_soa(rdA32, 1, old, nld, m, stream);
    realloc_soa(rgam32, 1, old, nld, m, stream);
    realloc_soa(rg32, 1, old, nld, m, stream);
    csr_ent.release();
    csr_ent.ensure(2 * nld);
    realloc_soa(rlist, 1, old, nld, m, stream);
    rlist2.release();
    rlist2.ensure(nld);
    ldr = (int)nld;
}

// ---------------------------------------------------------------------------
// candidate pairs (all a < b of one packing with bounding gap <= skin)
// ---------------------------------------------------------------------------
// Candidate pairs within skin_ of each other's bounding sphere; with bound,
// also within skin_ by the support gap along the centre line (a lower bound
// of Phi; needs the geometry of the positions xs in geo).
void relcp_ctx::broadphase(const double *xs, double skin_, bool bound) {
    const PairShapes shp{geo.p, n, kind.p, p.p, n};
    const int N = n;
    keys.ensure(6 * nbatch + 1);
    bool any_open = false;
    for (int pk = 0; pk < nbatch; ++pk)
        for (int k = 0; k < 3; ++k) any_open |= !(box[3 * pk + k] > 0);
    std::vector<unsigned long long> kh(6 * nbatch);
    if (any_open) {
        std::vector<unsigned long long> init(6 * nbatch);
        for (int pk = 0; pk < nbatch; ++pk)
            for (int k = 0; k < 3; ++k) {
                init[6 * pk + k] = ~0ull;
                init[6 * pk + 3 + k] = 0ull;
            }
        HIP_OK(hipMemcpyAsync(keys.p, init.data(), 6 * nbatch * sizeof(unsigned long long), hipMemcpyHostToDevice,
                              stream));
        hipLaunchKernelGGL(k_bbox, dim3(nblk(N, 256)), dim3(256), 0, stream, N, xs, N, body_batch.p, keys.p);
        HIP_OK(hipMemcpyAsync(kh.data(), keys.p, 6 * nbatch * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              stream));
        sync();
    }
    grids_h.resize(nbatch);
    long long total = 0;
    for (int pk = 0; pk < nbatch; ++pk) {
        PackGrid &g = grids_h[pk];
        double csmin = 2.0 * rmax[pk] + skin_;
        int nbody = boff[pk + 1] - boff[pk];
        long long cap_cells = std::max<long long>(64, 8LL * nbody);
        for (int k = 0; k < 3; ++k) {
            double L = box[3 * pk + k];
            g.box[k] = L;
            if (L > 0) {
                g.periodic[k] = 1;
                g.nc[k] = std::max(1, (int)std::floor(L / csmin));
                g.cs[k] = L / g.nc[k];
                g.org[k] = 0.0;
            } else {
                g.periodic[k] = 0;
                double lo = order_key_value(kh[6 * pk + k]), hi = order_key_value(kh[6 * pk + 3 + k]);
                double ext = std::max(0.0, hi - lo);
                g.org[k] = lo;
                g.cs[k] = csmin;
                g.nc[k] = std::max(1, (int)std::ceil(ext / csmin + 1e-9));
            }
        }
        // keep the cell count bounded for sparse open domains
        while ((long long)g.nc[0] * g.nc[1] * g.nc[2] > cap_cells) {
            for (int k = 0; k < 3; ++k)
                if (!g.periodic[k] && g.nc[k] > 1) {
                    g.cs[k] *= 2.0;
                    g.nc[k] = std::max(1, (g.nc[k] + 1) / 2);
                }
            bool shrinkable = false;
            for (int k = 0; k < 3; ++k) shrinkable |= (!g.periodic[k] && g.nc[k] > 1);
            if (!shrinkable) break;
        }
        g.cell_off = total;
        total += (long long)g.nc[0] * g.nc[1] * g.nc[2];
    }
    if (total > (1LL << 30)) throw Error{RELCP_E_CAPACITY, "too many broadphase cells"};
    int nc = (int)total;
    grids.ensure(nbatch);
    HIP_OK(hipMemcpyAsync(grids.p, grids_h.data(), nbatch * sizeof(PackGrid), hipMemcpyHostToDevice, stream));
    body_cell.ensure(N);
    cell_count.ensure(2 * (size_t)(nc + 1));  // counts, then cursors
    cell_start.ensure(nc + 1);
    cell_items.ensure(N);
    pair_count.ensure(N + 1);
    pair_off.ensure(N + 1);
    dtotal.ensure(4);
    HIP_OK(hipMemsetAsync(cell_count.p, 0, 2 * (nc + 1) * sizeof(int), stream));
    int *cell_cur = cell_count.p + (nc + 1);
    launch_cell_assign(N, xs, N, body_batch.p, grids.p, body_cell.p, cell_count.p, stream);
    exclusive_scan(cell_count.p, cell_start.p, nc, nullptr, scan_scratch, stream);
    launch_cell_fill(N, body_cell.p, cell_start.p, cell_cur, cell_items.p, stream);
    timed(3, [&] {
        launch_pairs(false, N, xs, N, Rb.p, body_batch.p, grids.p, body_cell.p, cell_start.p, cell_count.p,
                     cell_items.p, skin_, pair_count.p, nullptr, nullptr, nullptr, 0, stream, bound ? &shp : nullptr);
    });
    exclusive_scan(pair_count.p, pair_off.p, N, int_d, scan_scratch, stream);  // total -> int_h[0]
    sync();
    np = N > 0 ? int_h[0] : 0;
    if (np < 0) throw Error{RELCP_E_CAPACITY, "pair count overflow"};
    ensure_pairs(std::max(np, 1));
    timed(3, [&] {
        launch_pairs(true, N, xs, N, Rb.p, body_batch.p, grids.p, body_cell.p, cell_start.p, cell_count.p,
                     cell_items.p, skin_, pair_count.p, pair_off.p, pa.p, pb.p, ldp, stream, bound ? &shp : nullptr);
    });
    pcsr_valid = false;
}

void relcp_ctx::candidate_pairs(relcp_step_stats &S) {
    if (!vl_valid || vl_used >= 2.0 * vl_margin()) {
        // the kept list: bounding spheres and the centre-line support gap
        // within the list radius (the displacement bound covers Phi too)
        broadphase(x.p, vl_radius(), true);
        vl_valid = true;
        vl_used = 0.0;
        prev_is_list = false;
        hint_ok = false;
        S.pairs_rebuilt = 1;
    }
    S.n_pairs = np;
}

// ---------------------------------------------------------------------------
// rows and incidence
// ---------------------------------------------------------------------------
void relcp_ctx::build_rows(int nsel, int rec, const double *snsd, const double *vc, bool warm, double dt) {
    const RowBuildArgs a = row_args(nsel, rec, snsd, vc, warm, dt);
    launch_rows_build(a, stream);
    m += nsel;
}

RowBuildArgs relcp_ctx::row_args(int nsel, int rec, const double *snsd, const double *vc, bool warm, double dt) {
    RowBuildArgs a{};
    a.nsel = nsel;
    a.sel = sel.p;
    a.pa = pa.p;
    a.pb = pb.p;
    a.snsd = snsd;
    a.ldp = ldp;
    a.m0 = m;
    a.rec = rec;
    a.dt = dt;
    a.K = K.p;
    a.kiso = k_iso() ? 1 : 0;
    // overdamped bodies without external forces: U_free = 0
    a.vfree = dynamics == RELCP_OVERDAMPED && !has_fext ? nullptr : vfree.p;
    a.vc = vc;
    a.ldb = n;
    a.nprev = warm ? nprev : 0;
    a.prev_a = prev_a.p;
    a.prev_b = prev_b.p;
    a.prev_lam = warm ? prev_lam.p : nullptr;
    a.prev_direct = warm && prev_is_list ? 1 : 0;
    a.ldr = ldr;
    a.ia = ria.p; a.ib = rib.p; a.pair = rpair.p; a.rec_out = rrec.p;
    a.n64 = rn64.p; a.ta64 = rta64.p; a.tb64 = rtb64.p; a.qv64 = rqv64.p; a.dA64 = rdA64.p; a.gam64 = rgam64.p;
    a.phi64 = rphi64.p;
    a.qv32 = rqv32.p; a.dA32 = rdA32.p;
    // the FP32 geometry and start are read only by the matrix-free FP32
    // solves (the row graph's are formed from the FP64 rows)
    if (!rowgraph_mode()) {
        a.n32 = rn32.p; a.ta32 = rta32.p; a.tb32 = rtb32.p; a.gam32 = rgam32.p;
    }
    rows32_ok = !rowgraph_mode() && (rows32_ok || rec == 0);
    return a;
}

// Rows grouped by packing for the resident LCP kernel: rlist holds row
// indices packing by packing, roff the packing offsets into rlist.
void relcp_ctx::rows_by_packing_init(int m0) {
    HIP_OK(hipMemsetAsync(rcnt.p, 0, (nbatch + 1) * sizeof(int), stream));
    launch_rows_per_packing(0, m0, ria.p, body_batch.p, rcnt.p, stream);
    exclusive_scan(rcnt.p, roff.p, nbatch + 1, nullptr, scan_scratch, stream);
    launch_iota(m0, rlist.p, stream);
}

void relcp_ctx::rows_by_packing_append(int m_old, int nv) {
    HIP_OK(hipMemsetAsync(rcnt.p, 0, (nbatch + 1) * sizeof(int), stream));
    launch_rows_per_packing(m_old, m_old + nv, ria.p, body_batch.p, rcnt.p, stream);
    exclusive_scan(rcnt.p, rE.p, nbatch + 1, nullptr, scan_scratch, stream);
    launch_rlist_merge(m_old, nv, rlist.p, ria.p, body_batch.p, roff.p, rE.p, rlist2.p, stream);
    launch_add_arrays(nbatch + 1, roff.p, rE.p, roff.p, stream);
    std::swap(rlist.p, rlist2.p);
    std::swap(rlist.cap, rlist2.cap);
}

void relcp_ctx::rebuild_csr() {
    rg_valid = false;
    lists_gapped = false;
    csr_cnt.ensure(2 * (size_t)(n + 1));
    csr_off.ensure(n + 1);
    csr_ent.ensure(2 * (size_t)std::max(m, 1));
    const bool cleared = csr_clear == csr_cnt.p;
    csr_clear = nullptr;
    // in the row-graph mode the fill pass also produces the graph's slice widths
    CsrRowGraphOut rgo{};
    // (a build whose graph was never assembled left its width sum in the
    // entry counter: clear it)
    if (rg_pre && rg_flags.p) HIP_OK(hipMemsetAsync(rg_flags.p, 0, sizeof(int), stream));
    rg_pre = rowgraph_mode() && m > 0;
    if (rg_pre) {
        rg_prepare();
        rgo = CsrRowGraphOut{rg_flags.p, rg_rcnt.p};
    }
    launch_csr(n, m, ria.p, rib.p, csr_cnt.p, csr_off.p, csr_cnt.p + (n + 1), csr_ent.p, cleared, scan_scratch,
               stream, rg_pre ? &rgo : nullptr);
    csr_clear = csr_cnt.p;  // the build's last pass clears the counters again
}

// Incidence lists of the step's first rows (the selected candidate pairs,
// row k = the k-th selected pair, prow filled by the selection): the
// candidate pairs' lists (built when the candidate list changed) filtered
// through prow in one pass, each body's list in the slots of its candidate
// list, with its length in fl_cnt.  Each list holds the entries rebuild_csr
// gives it, in the same order.  The row graph's assembly forms the rows'
// entry counts from the lengths and adds up the filter's block sums for the
// entry count.  The filter reads no row count, so it can run before the count
// reaches the host (mcap: the rows' capacity).
void relcp_ctx::first_rows_csr(int mcap) {
    if (!pcsr_valid) {
        pcsr_cnt.ensure(2 * (size_t)(n + 1));
        pcsr_off.ensure(n + 1);
        pcsr_ent.ensure(2 * (size_t)std::max(np, 1));
        launch_csr(n, np, pa.p, pb.p, pcsr_cnt.p, pcsr_off.p, pcsr_cnt.p + (n + 1), pcsr_ent.p,
                   pcsr_clear == pcsr_cnt.p, scan_scratch, stream, nullptr);
        pcsr_clear = pcsr_cnt.p;
        pcsr_valid = true;
    }
    rg_valid = false;
    rg_pre = false;
    if (np > 0) {
        csr_ent.ensure(2 * (size_t)np);
        fl_cnt.ensure(n + 1);
        fl_bsums.ensure(filter_blocks(n));
        if (rowgraph_mode() && mcap > 0) rg_prepare(mcap);
        filter_lists(n, pcsr_off.p, pcsr_ent.p, prow.p, fl_cnt.p, csr_ent.p, fl_bsums.p, stream);
        lists_gapped = true;
    } else {
        csr_off.ensure(n + 1);
        HIP_OK(hipMemsetAsync(csr_off.p, 0, (n + 1) * sizeof(int), stream));
        lists_gapped = false;
    }
}

// Features of the iteration-0 rows (their multipliers hold the previous
// step's pair sums) and, for the learned start, the MLP's prediction in
// their place; a cold start clears them again.
void relcp_ctx::warm_start_rows(int m0, double dt) {
    feat.ensure(8 * (size_t)std::max(m0, 1));
    rowscale.ensure(std::max(m0, 1));
    FeatureArgs fa{};
    fa.m0 = m0; fa.ldr = ldr; fa.ia = ria.p; fa.ib = rib.p;
    fa.n = rn64.p; fa.ta = rta64.p; fa.tb = rtb64.p; fa.phi = rphi64.p; fa.lam = rgam64.p; fa.dA = rdA64.p;
    fa.ldb = n; fa.kind = kind.p; fa.p = p.p; fa.u = u.p; fa.off = lists_gapped ? pcsr_off.p : csr_off.p; fa.ent = csr_ent.p;
    fa.lcnt = lists_gapped ? fl_cnt.p : nullptr;
    fa.perm = perm_d.p;
    fa.dt = dt; fa.feat = feat.p; fa.rowscale = rowscale.p;
    timed(6, [&] { launch_features(fa, stream); });
    if (warm_start == RELCP_WS_LEARNED) {
        MlpArgs ma{};
        ma.n = m0; ma.X = feat.p; ma.params = mlp_w.p;
        std::memcpy(ma.norm, mlp_norm, sizeof(mlp_norm));
        ma.rowscale = rowscale.p;
        ma.out64 = rgam64.p;
        timed(6, [&] { launch_mlp_forward(ma, stream); });
    } else if (warm_start == RELCP_WS_COLD && m0 > 0) {
        HIP_OK(hipMemsetAsync(rgam64.p, 0, (size_t)m0 * sizeof(double), stream));
    }
}

// Entry slots of the row graph: at least `slots` in every array.  Buffers
// are replaced only when too small, with half again as much headroom (a
// growing contact set would otherwise free and re-allocate, and so wait on
// the device, at every step); rg_cap is what all three actually hold.
void relcp_ctx::rg_reserve(size_t slots) {
    if (rg_col.cap < slots || rg_val64.cap < slots || rg_val32.cap < slots) {
        rg_col.release(); rg_val64.release(); rg_val32.release();
        rg_col.ensure(slots + slots / 2);
        rg_val64.ensure(slots + slots / 2);
        rg_val32.ensure(slots + slots / 2);
    }
    rg_cap = std::min(rg_col.cap, std::min(rg_val64.cap, rg_val32.cap));
}

// Row graph of the current rows: the rows' entry counts (unless the
// incidence build made them), then the entries (one thread per incidence
// entry) at a fixed stride per row.  Nothing is read back here: a row with
// more entries than the stride is flagged by the fill, which the solve
// checks at its first read-back (then raises the stride, rebuilds and
// restarts).
// buffers of the row graph's counts and counters
void relcp_ctx::rg_prepare(int mcap) {
    if (mcap < 0) mcap = m;
    rg_rcnt.ensure(std::max(mcap, 1));
    if (!rg_flags.p) {
        rg_flags.ensure(2);
        // the entry counter (cleared by each fill) and the overflow's count
        // (cleared after it is read)
        HIP_OK(hipMemsetAsync(rg_flags.p, 0, 2 * sizeof(int), stream));
    }
}

void relcp_ctx::build_rowgraph(double dt) {
    const int ns = rowgraph_slices(m);
    rg_prepare();
    rg_reserve(std::max<size_t>((size_t)RELCP_WAVE * ns * rg_stride, 64));
    int_h[5] = int_h[6] = 0;  // entries, overflow (written by the fill)
    if (!rg_pre && !lists_gapped) {
        // counts not made by the incidence build (a rebuild; with the first
        // rows' filtered lists the fill forms them)
        timed(8, [&] {
            launch_rowgraph_counts(m, ria.p, rib.p, csr_off.p, rg_flags.p, rg_rcnt.p, stream);
        });
    }
    rg_pre = false;

    RowGraphFill f{};
    f.m = m; f.ldr = ldr; f.ia = ria.p; f.ib = rib.p; f.n = rn64.p; f.ta = rta64.p; f.tb = rtb64.p;
    f.ldb = n; f.K = K.p; f.kiso = k_iso() ? 1 : 0;
    f.off = lists_gapped ? pcsr_off.p : csr_off.p; f.ent = csr_ent.p;
    f.lcnt = lists_gapped ? fl_cnt.p : nullptr;
    f.nslots = lists_gapped ? 2 * np : 2 * m;
    f.bsums = fl_bsums.p; f.nbsums = filter_blocks(n);
    f.rcnt = rg_rcnt.p; f.stride = rg_stride;
    f.dt = dt; f.cap = rg_cap; f.count = rg_flags.p; f.need = rg_flags.p + 1; f.report = int_d + 4;
    f.col = rg_col.p; f.val64 = rg_val64.p; f.val32 = rg_val32.p;
    timed(8, [&] { launch_rowgraph_fill(f, stream); });  // reports entries and overflow, read after the solve's first sync
    rg_valid = true;
    rg_dt = dt;
}

// ---------------------------------------------------------------------------
// LCP of one recursion
// ---------------------------------------------------------------------------
template <typename T>
RowsT<T> relcp_ctx::rows_of() const {
    RowsT<T> R{};
    R.m = m;
    R.ld = ldr;
    R.ia = ria.p;
    R.ib = rib.p;
    if constexpr (sizeof(T) == 8) {
        R.n = rn64.p; R.ta = rta64.p; R.tb = rtb64.p; R.qv = rqv64.p; R.dA = rdA64.p; R.gam = rgam64.p; R.g = rg64.p;
    } else {
        R.n = rn32.p; R.ta = rta32.p; R.tb = rtb32.p; R.qv = rqv32.p; R.dA = rdA32.p; R.gam = rgam32.p; R.g = rg32.p;
    }
    return R;
}

template <typename T>
BodiesT<T> relcp_ctx::bodies_of() const {
    BodiesT<T> Bd{};
    if constexpr (sizeof(T) == 8) {
        Bd.K = K.p; Bd.vc = vc64.p;
    } else {
        Bd.K = K32.p; Bd.vc = vc32.p;
    }
    Bd.kiso = k_iso() ? 1 : 0;
    Bd.nb = n;
    Bd.ld = n;
    Bd.off = lists_gapped ? pcsr_off.p : csr_off.p;
    Bd.ent = csr_ent.p;
    Bd.lcnt = lists_gapped ? fl_cnt.p : nullptr;
    return Bd;
}

template <typename T>
int relcp_ctx::solve(double dt, double tol, int &iters, double &res) {
    if (sizeof(T) == 4 && !rowgraph_mode() && !rows32_ok) {
        // rows built for the row graph have no FP32 geometry: from the FP64
        launch_demote(3 * ldr, rn64.p, rn32.p, stream);
        launch_demote(3 * ldr, rta64.p, rta32.p, stream);
        launch_demote(3 * ldr, rtb64.p, rtb32.p, stream);
        rows32_ok = true;
    }
    const RowsT<T> R = rows_of<T>();
    const BodiesT<T> Bd = bodies_of<T>();
    if (resident_mode()) {
        ResidentArgs<T> a{R, Bd, nbatch, boff_d.p, roff.p, rlist.p, dt, lcp_fixed > 0 ? -1.0 : tol,
                          lcp_fixed > 0 ? lcp_fixed : lcp_max_iters, pk_state.p, maxpk, stall_iters<T>()};
        const bool lds = res_lds && (size_t)6 * maxpk * sizeof(T) <= 150 * 1024;
        int rc = 0;
        timed(5, [&] { rc = launch_lcp_resident<T>(a, res_block, lds, stream); });
        if (rc != 0 && lds) timed(5, [&] { rc = launch_lcp_resident<T>(a, res_block, false, stream); });
        if (rc != 0) throw Error{RELCP_E_DEVICE, "resident LCP launch failed"};
        HIP_OK(hipMemcpyAsync(pk_state_h, pk_state.p, nbatch * sizeof(PgdState), hipMemcpyDeviceToHost, stream));
        sync();
        bool conv = true;
        iters = 0;
        res = 0.0;
        for (int k = 0; k < nbatch; ++k) {
            iters = std::max(iters, pk_state_h[k].iter);
            res = std::max(res, pk_state_h[k].res);
            conv = conv && pk_state_h[k].conv;
        }
        if (!std::isfinite(res)) return RELCP_E_NAN;
        if (lcp_fixed > 0) return RELCP_OK;
        return conv ? RELCP_OK : RELCP_E_LCP_MAXITER;
    }
    if (rowgraph_mode()) return solve_rowgraph<T>(R, Bd, dt, tol, iters, res);
    partials.ensure(lcp_partials_needed(m));
    // pst: S[0], S[1], fin, then a slot whose first int is the done flag
    pst.ensure(4);
    PgdCtl C{pst.p, pst.p + 2, reinterpret_cast<int *>(pst.p + 3), partials.p, lcp_gather_blocks(m),
             lcp_fixed > 0 ? -1.0 : tol, pst_d, reinterpret_cast<int *>(pst_d + 1), stall_iters<T>()};
    const int cap = lcp_fixed > 0 ? lcp_fixed : lcp_max_iters;
    const int pk = sizeof(T) == 8 ? 1 : 0;
    launch_pgd_init(C, stream);
    timed(0, [&] { launch_lcp_scatter<T>(0, R, Bd, C, 0, stream); });
    timed(1, [&] { launch_lcp_gather<T>(0, R, Bd, dt, C, 0, stream); });
    // iterations are launched in chunks; passes after convergence return at
    // once, so a chunk only over-runs by empty launches
    int j = 1;
    int chunk = std::max(2, std::min(64, (last_iters[pk] + 3) & ~1));
    bool done = false;
    for (;;) {
        int k = std::min(chunk, cap - (j - 1));
        if (k <= 0) break;
        for (int t = 0; t < k; ++t, ++j) {
            const int par = j & 1;
            timed(0, [&] { launch_lcp_scatter<T>(1, R, Bd, C, par, stream); });
            timed(1, [&] { launch_lcp_gather<T>(1, R, Bd, dt, C, par, stream); });
        }
        sync();
        if (*reinterpret_cast<int *>(pst_h + 1)) {
            done = true;
            break;
        }
        chunk = std::min(64, std::max(8, 2 * chunk));
    }
    if (!done) {
        // account for the last gather (iteration cap or fixed-iteration run):
        // the state after it follows S[(j - 1) & 1] into slot j & 1
        launch_pgd_finalize(C, j & 1, stream);
        sync();
    }
    const bool conv = *reinterpret_cast<int *>(pst_h + 1) != 0;
    iters = pst_h[0].iter;
    res = pst_h[0].res;
    last_iters[pk] = iters;
    if (!std::isfinite(res)) return RELCP_E_NAN;
    if (lcp_fixed > 0) return RELCP_OK;
    return conv ? RELCP_OK : RELCP_E_LCP_MAXITER;
}

// The instantiated pass graph of precision T for at least `rows` rows and
// its parameter block; null if graphs are unavailable (per-pass launches).
template <typename T>
hipGraphExec_t relcp_ctx::spmv_graph_for(int rows, LcpDev<T> **dev) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    if constexpr (sizeof(T) == 8) {
        lcpdev64.ensure(1);
        *dev = lcpdev64.p;
    } else {
        lcpdev32.ensure(1);
        *dev = lcpdev32.p;
    }
    if (spmv_graph[pk] && graph_rows[pk] >= rows) return spmv_graph[pk];
    if (spmv_graph[pk]) {
        sync();
        (void)hipGraphExecDestroy(spmv_graph[pk]);
        spmv_graph[pk] = nullptr;
    }
    // grid headroom so that a growing contact set rarely re-instantiates
    const int want = std::max(4096, rows + rows / 4);
    if (make_spmv_graph<T>(*dev, want, kGraphPasses, &spmv_graph[pk]) != 0) {
        (void)hipGetLastError();
        graph_ok = false;
        return nullptr;
    }
    graph_rows[pk] = want;
    return spmv_graph[pk];
}

// Row-graph LCP loop: pass 0 forms g at the start, pass j (parity j & 1)
// reads state buffer z[(j - 1) & 1] and the partials of pass j - 1 and
// writes z[j & 1] and its own partials; the final iterate is unpacked into
// the rows' gamma and g, and (FP64) the contact velocities K D gamma that
// the trial integration needs are formed once.
template <typename T>
relcp_ctx::RgBufs<T> relcp_ctx::rg_bufs(const RowsT<T> &R, double tol) {
    const size_t mz = std::max(m, 1);
    const int pk = sizeof(T) == 8 ? 1 : 0;
    RgBufs<T> B{};
    if constexpr (sizeof(T) == 8) {
        z64.ensure(2 * mz);
        zg64.ensure(2 * mz);
        B.z0 = z64.p; B.z1 = z64.p + mz; B.g0 = zg64.p; B.g1 = zg64.p + mz;
    } else {
        z32.ensure(2 * mz);
        zg32.ensure(2 * mz);
        B.z0 = z32.p; B.z1 = z32.p + mz; B.g0 = zg32.p; B.g1 = zg32.p + mz;
    }
    // each precision has its own control block and partial sums, so that an
    // FP32 solve can continue after FP64 passes were launched behind it
    B.stride = lcp_partials_needed(m);
    partials.ensure(4 * B.stride);
    B.part = partials.p + 2 * B.stride * pk;
    pst.ensure(8);
    PgdState *cb = pst.p + 4 * pk;
    B.C = PgdCtl{cb, cb + 2, reinterpret_cast<int *>(cb + 3), B.part, lcp_gather_blocks(m),
                 lcp_fixed > 0 ? -1.0 : tol, pst_d + 2 * pk, reinterpret_cast<int *>(pst_d + 2 * pk + 1),
                 stall_iters<T>()};
    B.G = RowGraphT<T>{m, rg_stride, rg_col.p, nullptr, rg_cap, rg_rcnt.p};
    if constexpr (sizeof(T) == 8)
        B.G.val = rg_val64.p;
    else
        B.G.val = rg_val32.p;
    (void)R;
    return B;
}

// k iteration passes from pass rgr[pk].j on
template <typename T>
void relcp_ctx::rg_passes(const RgBufs<T> &B, const RowsT<T> &R, int k) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    RgRun &st = rgr[pk];
    for (int t = 0; t < k; ++t, ++st.j) {
        const int par = st.j & 1;
        PgdCtl c = B.C;
        c.partials = B.part + (size_t)(par ^ 1) * B.stride;  // the previous pass's partial sums
        if (timing) pass_ev.push_back(PassEv{ev_used / 2, st.j, pk});
        timed(sizeof(T) == 4 ? 7 : 10, [&] {
            launch_lcp_spmv<T>(st.pass_mode, B.G, R.qv, R.dA, StartSrc{}, par ? B.z0 : B.z1, par ? B.g0 : B.g1,
                               par ? B.z1 : B.z0, par ? B.g1 : B.g0, c, B.part + (size_t)par * B.stride, par, stream);
        });
    }
}

// Row-graph solve, launch part: the graph of the current rows (if not
// valid), the start pass and a first chunk of iteration passes (the last
// solve's count plus the pass that sees convergence and a spare).  Nothing
// is waited for.
template <typename T>
// Start of a row-graph solve from gam0, or from src (with gam0 null): the
// final state of the FP32 solve, for the FP64 polish.
void relcp_ctx::rg_start(const RowsT<T> &R, double dt, double tol, const double *gam0, double *save,
                         const StartSrc *src, bool allow_final) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    RgRun &st = rgr[pk];
    st.fresh = false;
    if (!rg_valid || rg_dt != dt) {
        build_rowgraph(dt);
        st.fresh = true;
    }
    const RgBufs<T> B = rg_bufs<T>(R, tol);
    // the last solve's count, the pass that sees convergence and headroom: a
    // short first chunk costs a wait and, in a step, the work launched behind
    // it, while a spare pass returns at once
    st.chunk = std::max(2, std::min(64, last_iters[pk] + std::max(2, last_iters[pk] / 6) + 1));
    // a solve that last converged at its start: the pass that sees it and a
    // spare one; only the first once it has done so several times in a row.
    // The FP64 polish of a step (allow_final) then runs no pass at all: its
    // start pass writes what the unpack would, and the tail's report checks
    // its convergence (a miss costs a wait, as a short chunk does)
    st.final_start = false;
    if (last_iters[pk] == 0) {
        st.chunk = zero_run[pk] >= 4 ? 1 : 2;
        if (sizeof(T) == 8 && src && allow_final && zero_run[pk] >= 4 && unpack_can_check(m)) {
            st.chunk = 0;
            st.final_start = true;
            work_out.ensure(work_blocks(m));
        }
    }
    // the start pass also resets the control block
    timed(11, [&] {
        StartSrc start = src ? *src : StartSrc{gam0, {nullptr, nullptr}, nullptr, nullptr, 0};
        if (st.final_start) {
            start.g_final = rg64.p;
            start.work_final = work_out.p;
        }
        launch_lcp_spmv<T>(0, B.G, R.qv, R.dA, start, nullptr, nullptr, B.z0, B.g0, B.C, B.part, 0, stream, save);
    });
    st.j = 1;
    // over many blocks the partial sums are reduced once per pass by a
    // separate launch instead of by every block
    st.pass_mode = B.C.nbg >= reduce_split_blocks ? 2 : 1;
    const int cap = lcp_fixed > 0 ? lcp_fixed : lcp_max_iters;
    rg_passes<T>(B, R, std::min(st.chunk, cap));
}

// The rows' gamma and g from the solve's final iterate, or from its last
// pass while it has not finished (chosen on the device); FP32 also widens
// gamma into the FP64 multipliers.
template <typename T>
void relcp_ctx::rg_unpack(const RowsT<T> &R, const BodiesT<T> &Bd, double tol) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    const RgBufs<T> B = rg_bufs<T>(R, tol);
    // FP64 also forms the work gamma^T A gamma's partial sums (the trial
    // forms the contact velocities K D gamma itself)
    if constexpr (sizeof(T) == 8) work_out.ensure(work_blocks(m));
    // (a polish of which only the start pass ran wrote the results itself)
    if (rgr[pk].final_start) return;
    launch_rowstate_unpack<T>(m, B.z0, B.z1, B.g0, B.g1, B.C.fin, B.C.done, (rgr[pk].j - 1) & 1, R.gam, R.g,
                              sizeof(T) == 4 ? rgam64.p : nullptr, stream, sizeof(T) == 8 ? R.qv : nullptr,
                              sizeof(T) == 8 ? work_out.p : nullptr);
}

// After a wait: true if the last graph assembly overflowed its slots (then
// they are re-sized and the graph is marked for re-assembly).
bool relcp_ctx::rg_overflowed() {
    rg_entries = int_h[5];
    if (!int_h[6]) return false;
    // the largest count of a row that did not fit, then cleared for the next
    // overflow; the stride takes it with half again as much headroom
    int need = 0;
    HIP_OK(hipMemcpyAsync(&need, rg_flags.p + 1, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemsetAsync(rg_flags.p + 1, 0, sizeof(int), stream));
    HIP_OK(hipStreamSynchronize(stream));
    rg_stride = std::max(rg_stride + 1, need + need / 2);
    rg_valid = false;
    ++rg_restarts;
    return true;
}

// Row-graph solve, completion (after a wait that covered the launched
// passes): if the solve has not converged, further chunks (waiting after
// each), the state after the last pass if the cap is reached, and the unpack
// again (relaunched = true: everything launched after the first unpack is
// stale).  Returns the status; iters and res from the final state.
template <typename T>
int relcp_ctx::rg_finish(const RowsT<T> &R, const BodiesT<T> &Bd, double tol, int &iters, double &res,
                         bool &relaunched) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    RgRun &st = rgr[pk];
    const RgBufs<T> B = rg_bufs<T>(R, tol);
    const int *done_h = reinterpret_cast<const int *>(pst_h + 2 * pk + 1);
    const int cap = lcp_fixed > 0 ? lcp_fixed : lcp_max_iters;
    relaunched = false;
    if (!*done_h) {
        relaunched = true;
        st.chunk = std::max(st.chunk, 2);  // (a first chunk of no passes)
        for (;;) {
            const int k = std::min(st.chunk, cap - (st.j - 1));
            if (k <= 0) break;
            rg_passes<T>(B, R, k);
            sync();
            if (*done_h) break;
            st.chunk = std::min(64, std::max(8, 2 * st.chunk));
        }
        if (!*done_h) {
            // the state after the last pass (iteration cap or fixed iterations)
            PgdCtl cf = B.C;
            cf.partials = B.part + (size_t)((st.j - 1) & 1) * B.stride;
            launch_pgd_finalize(cf, st.j & 1, stream);
        }
        rg_unpack<T>(R, Bd, tol);
        sync();
    }
    const bool conv = *done_h != 0;
    iters = pst_h[2 * pk].iter;
    res = pst_h[2 * pk].res;
    last_iters[pk] = iters;
    zero_run[pk] = iters == 0 ? zero_run[pk] + 1 : 0;
    // passes past the last iteration only reduced (or returned at once):
    // timed apart from the iteration passes
    for (auto &pe : pass_ev)
        if (pe.pk == pk && pe.j > iters && pe.slot < ev_class.size()) ev_class[pe.slot] = kIdlePass;
    if (!std::isfinite(res)) return RELCP_E_NAN;
    if (lcp_fixed > 0) return RELCP_OK;
    return conv ? RELCP_OK : RELCP_E_LCP_MAXITER;
}

// Row-graph LCP loop, one solve waited for: pass 0 forms g at the start,
// pass j (parity j & 1) reads state buffer z[(j - 1) & 1] and the partials
// of pass j - 1 and writes z[j & 1] and its own partials; the final iterate
// is unpacked into the rows' gamma and g (FP64: with the work's partial
// sums; the trial forms the contact velocities K D gamma).  LCP mode 3
// replays the passes from an instantiated graph.
template <typename T>
int relcp_ctx::solve_rowgraph(const RowsT<T> &R, const BodiesT<T> &Bd, double dt, double tol, int &iters,
                              double &res) {
    if (lcp_mode == 3 && graph_ok && lcp_fixed == 0) return solve_rowgraph_graph<T>(R, Bd, dt, tol, iters, res);
    gam_save.ensure(std::max(m, 1));
    for (int attempt = 0;; ++attempt) {
        // a restart (the graph did not fit its slots) begins from the same start
        rg_start<T>(R, dt, tol, attempt ? gam_save.p : rgam64.p, attempt ? nullptr : gam_save.p);
        rg_unpack<T>(R, Bd, tol);
        sync();
        if (rgr[sizeof(T) == 8 ? 1 : 0].fresh && rg_overflowed()) {
            if (attempt > 0) throw Error{RELCP_E_DEVICE, "row graph sizing failed"};
            continue;
        }
        bool again = false;
        return rg_finish<T>(R, Bd, tol, iters, res, again);
    }
}

// Graph replay of the passes (LCP mode 3): whole graphs of kGraphPasses
// passes reading their parameters from device memory; passes past the end
// of the solve return at once.
template <typename T>
int relcp_ctx::solve_rowgraph_graph(const RowsT<T> &R, const BodiesT<T> &Bd, double dt, double tol, int &iters,
                                    double &res) {
    const int pk = sizeof(T) == 8 ? 1 : 0;
    const int cap = lcp_max_iters;
    const int *done_h = reinterpret_cast<const int *>(pst_h + 2 * pk + 1);
    for (int attempt = 0;; ++attempt) {
        bool fresh = false;
        if (!rg_valid || rg_dt != dt) {
            build_rowgraph(dt);
            fresh = true;
        }
        const RgBufs<T> B = rg_bufs<T>(R, tol);
        LcpDev<T> *dev = nullptr;
        hipGraphExec_t ge = spmv_graph_for<T>(m, &dev);
        if (!ge) {
            // graphs unavailable: per-pass launches from here on
            graph_ok = false;
            return solve_rowgraph<T>(R, Bd, dt, tol, iters, res);
        }
        LcpDev<T> v{};
        v.m = m; v.nbg = B.C.nbg; v.cap = cap; v.tol = B.C.tol; v.stall = B.C.stall;
        v.stride = B.G.stride; v.col = B.G.col; v.val = B.G.val; v.slots = B.G.cap; v.rcnt = B.G.rcnt;
        v.qv = R.qv; v.dA = R.dA;
        v.z[0] = B.z0; v.z[1] = B.z1; v.g[0] = B.g0; v.g[1] = B.g1;
        v.part[0] = B.part; v.part[1] = B.part + B.stride;
        v.S = B.C.S; v.fin = B.C.fin; v.done = B.C.done; v.fin_h = B.C.fin_h; v.done_h = B.C.done_h;
        launch_set_lcpdev<T>(dev, v, stream);
        timed(11, [&] {
            launch_lcp_spmv<T>(0, B.G, R.qv, R.dA, StartSrc{rgam64.p, {nullptr, nullptr}, nullptr, nullptr, 0}, nullptr,
                               nullptr, B.z0, B.g0, B.C, B.part, 0, stream);
        });
        int j = 1;
        int chunk = std::max(2, std::min(64, (last_iters[pk] + 3) & ~1));
        bool first = true, overflow = false;
        for (;;) {
            const int ng = (chunk + kGraphPasses - 1) / kGraphPasses;
            for (int t = 0; t < ng; ++t, j += kGraphPasses)
                timed_span(sizeof(T) == 4 ? 7 : 10, [&] { HIP_OK(hipGraphLaunch(ge, stream)); });
            sync();
            if (first && fresh) {
                first = false;
                if (rg_overflowed()) {
                    overflow = true;
                    break;
                }
            }
            if (*done_h || pst_h[2 * pk].iter >= cap) break;
            if (j > cap + 1) throw Error{RELCP_E_DEVICE, "LCP passes ran past the iteration cap"};
            chunk = std::min(64, std::max(8, 2 * chunk));
        }
        if (overflow) {
            if (attempt > 0) throw Error{RELCP_E_DEVICE, "row graph sizing failed"};
            continue;
        }
        // done is set (the stop pass wrote the final state)
        if constexpr (sizeof(T) == 8) work_out.ensure(work_blocks(m));
        launch_rowstate_unpack<T>(m, B.z0, B.z1, B.g0, B.g1, B.C.fin, nullptr, 0, R.gam, R.g,
                                  sizeof(T) == 4 ? rgam64.p : nullptr, stream, sizeof(T) == 8 ? R.qv : nullptr,
                                  sizeof(T) == 8 ? work_out.p : nullptr);
        sync();
        // the stop pass marks done on convergence and at the cap; done_h
        // mirrors convergence only
        const bool conv = *done_h != 0;
        iters = pst_h[2 * pk].iter;
        res = pst_h[2 * pk].res;
        last_iters[pk] = iters;
        if (!std::isfinite(res)) return RELCP_E_NAN;
        return conv ? RELCP_OK : RELCP_E_LCP_MAXITER;
    }
}

// ---------------------------------------------------------------------------
// one time-step (Alg. 1 / Eq. relcp_inertial)
// ---------------------------------------------------------------------------
int relcp_ctx::step(double dt, double eps, double tol, relcp_step_stats *st) {
    relcp_step_stats S;
    std::memset(&S, 0, sizeof(S));
    Timer tm;
    double t_narrow = 0, t_lcp = 0, t_other = 0;
    const int N = n;
    n_waits = 0;
    t_wait = 0.0;
    rg_restarts = 0;
    pass_ev.clear();

    // set-up at C^k: geometry, K, U_free
    BodySetupArgs ba{};
    ba.nb = N; ba.q = q.p; ba.ldq = N; ba.kind = kind.p; ba.p = p.p; ba.ldp = N; ba.rho_xi = rho.p;
    ba.u = u.p; ba.ldu = N; ba.fext = has_fext ? fext.p : nullptr; ba.ldf = N;
    ba.dynamics = dynamics; ba.planar = planar; ba.dt = dt;
    ba.geo = geo.p; ba.ldg = N; ba.Rb = Rb.p; ba.K = K.p; ba.ldk = N; ba.K32 = K32.p; ba.vfree = vfree.p; ba.ldv = N;
    if (!(dynamics == RELCP_OVERDAMPED && setup_valid)) {
        launch_body_setup(ba, stream);
        setup_valid = dynamics == RELCP_OVERDAMPED;
    }

    // candidate pairs at C^k
    candidate_pairs(S);
    t_other += tm.ms();

    // SNSD at C^k, iteration-0 set A_0 = {Phi_0 <= skin}
    SnsdArgs sa{};
    sa.m = np; sa.pa = pa.p; sa.pb = pb.p; sa.body_batch = body_batch.p; sa.x = x.p; sa.ldx = N; sa.geo = geo.p;
    sa.ldg = N; sa.kind = kind.p; sa.p = p.p; sa.ldp = N; sa.boxes = boxes.p; sa.planar = planar; sa.hint = nullptr;
    sa.only_kind = all_torus ? 2 : -1;
    sa.out = snsd0.p; sa.ldo = ldp; sa.mode = 0; sa.thresh = skin; sa.eps = eps; sa.flag = pflag.p;
    sa.bcount = pcnt.p;
    sa.minphi = nullptr; sa.minmarg = nullptr; sa.Rb = Rb.p;
    // Newton starts from the normals of the accepted trial of the previous
    // step (the same configuration up to the caller's rescale)
    if (hint_ok) sa.hint = snsdt.p + ldp;
    int_h[0] = -1;  // no GPU work in flight writes it: the compaction below sets the count
    timed(2, [&] { launch_snsd_pairs(sa, stream); });
    const bool learned = warm_start == RELCP_WS_LEARNED;
    const bool need_feat = learned || log_on;
    const bool warm0 = warm_start == RELCP_WS_PREV || need_feat;
    log_valid = false;
    m = 0;
    // count -> int_h[0]; each pair's row (or -1) -> prow; with fused_select
    // the rows are built by the same pass (room for every pair)
    prow.ensure(std::max(np, 1));
    const bool fused = fused_select && np > 0 && np <= select_rows_max_pairs();
    // with the rows built on the device, their incidence lists are launched
    // before the count reaches the host (they read it on the device), so
    // the GPU keeps working through the host's wait
    const bool early_lists = fused && first_lists;
    if (fused) {
        ensure_rows(np);
        dtotal.ensure(4);
        launch_select_rows(row_args(0, 0, snsd0.p, nullptr, warm0, dt), np, pflag.p, pcnt.p, sel.p, prow.p, int_d,
                           stream, dtotal.p + 1);
        if (early_lists) first_rows_csr(np);
    } else {
        compact_flags(pflag.p, np, pcnt.p, sel.p, int_d, scan_scratch, stream, nullptr, prow.p);
    }
    const int m0 = wait_mapped(int_h, -1);
    if (m0 < 0 || m0 > np) throw Error{RELCP_E_DEVICE, "bad contact count"};
    t_narrow += tm.ms();
    if (fused) {
        m = m0;
    } else {
        ensure_rows(m0);
        build_rows(m0, 0, snsd0.p, nullptr, warm0, dt);
    }
    if (early_lists) {
    } else if (first_lists) {
        first_rows_csr(m0);
    } else {
        rebuild_csr();
    }
    if (need_feat) warm_start_rows(m0, dt);
    if (resident_mode()) rows_by_packing_init(m0);
    t_other += tm.ms();

    int status = RELCP_OK;
    int rec = 0;
    int iters_total = 0;
    double minphi = 0.0;
    // Row-graph mode with one launch per pass: each recursion's FP32 solve
    // (if any), FP64 polish and trial are launched before one wait; a solve
    // found unfinished at that wait is continued and what follows it redone
    const bool spec = rowgraph_mode() && !(lcp_mode == 3 && graph_ok) && lcp_fixed == 0;
    for (;; ++rec) {
        // LCP of recursion rec
        int it = 0, it64 = 0;
        double res = 0, res64 = 0;
        const int nw = work_blocks(m), nt = trial_blocks(N), nsb = snsd_blocks(np);
        // W_n = gamma^T A gamma, trial configuration C_{n+1} = C^k (+) dt V_n,
        // SNSD of every candidate pair there, violators, report
        auto launch_tail = [&]() {
            work_out.ensure(nw);
            red.ensure((size_t)nt + 2 * (size_t)nsb);
            // (row-graph solves: the FP64 unpack has formed the work's partials)
            if (!rowgraph_mode()) launch_work(m, rgam64.p, rg64.p, rqv64.p, work_out.p, stream);
            timed(4, [&] {
                // row-graph solves leave the contact velocities to the trial,
                // which does not store them: only an augmentation needs them
                // (formed then by the LCP's scatter from the same multipliers)
                const RowsT<double> Rt = rows_of<double>();
                BodiesT<double> Bt = bodies_of<double>();
                Bt.vc = nullptr;
                const bool vrows = rowgraph_mode();
                // (overdamped bodies without external forces: U_free = 0)
                const double *vf = dynamics == RELCP_OVERDAMPED && !has_fext ? nullptr : vfree.p;
                launch_trial(N, x.p, N, q.p, N, vf, vc64.p, N, dt, kind.p, p.p, N, Rb.p, xt.p, qt.p, geot.p, N,
                             vout.p, red.p, stream, vrows ? &Rt : nullptr, vrows ? &Bt : nullptr);
            });
            SnsdArgs sb = sa;
            sb.x = xt.p; sb.geo = geot.p; sb.hint = snsd0.p + ldp; sb.out = snsdt.p; sb.mode = 1; sb.flag = pflag.p;
            sb.minphi = red.p + nt; sb.minmarg = red.p + nt + nsb;
            // the pair sums of an accepted step are accumulated there, from the
            // multipliers of the iteration-0 rows (one per pair; the rows of
            // later recursions are added after acceptance)
            sb.clear = lam.p;
            sb.init_row = prow.p;
            sb.init_gam = rgam64.p;
            timed(2, [&] { launch_snsd_pairs(sb, stream); });
            ++tok_seq;
            TailReport rep{nt, red.p, np > 0 ? nsb : 0, red.p + nt, red.p + nt + nsb, nw, work_out.p,
                           red_hd, dbl_hd, tok_d, tok_seq};
            // the violator count (from the check's per-group flag counts) ->
            // int_h[0], then the report; the violators are compacted only
            // when there are some (after the wait, for the augmentation)
            rep.ng = np > 0 ? flag_groups(np) : 0;
            rep.gcount = pcnt.p;
            rep.count = int_d;
            if (rgr[1].final_start) {
                // the polish ran only its start pass: the report checks it
                const RgBufs<double> B64 = rg_bufs<double>(rows_of<double>(), tol);
                PgdCtl c0 = B64.C;
                c0.partials = B64.part;
                launch_report_check(rep, c0, stream);
                rgr[1].final_start = false;
            } else {
                hipLaunchKernelGGL(k_report, dim3(1), dim3(256), 0, stream, rep);
            }
        };
        bool tail_ready = false;  // the tail ran on the final multipliers and was waited for
        if (spec) {
            const RowsT<float> R32 = rows_of<float>();
            const RowsT<double> R64 = rows_of<double>();
            const BodiesT<float> B32 = bodies_of<float>();
            const BodiesT<double> B64 = bodies_of<double>();
            gam_save.ensure(std::max(m, 1));
            for (int attempt = 0;; ++attempt) {
                // the first solve keeps its start: a restart (the graph did
                // not fit its slots) begins from the same one
                const double *g0 = attempt ? gam_save.p : rgam64.p;
                double *keep = attempt ? nullptr : gam_save.p;
                if (precision == 32) {
                    rg_start<float>(R32, dt, tol, g0, keep);
                    // the polish starts from the FP32 solve's final state
                    // (picked on the device, no unpack) and keeps it, in
                    // FP64, in the multipliers
                    const RgBufs<float> Bf = rg_bufs<float>(R32, tol);
                    const StartSrc src{nullptr, {Bf.z0, Bf.z1}, Bf.C.fin, Bf.C.done, (rgr[0].j - 1) & 1};
                    rg_start<double>(R64, dt, tol, nullptr, rgam64.p, &src, true);
                } else {
                    rg_start<double>(R64, dt, tol, g0, keep);
                }
                rg_unpack<double>(R64, B64, tol);
                launch_tail();
                wait_report();
                if ((rgr[0].fresh || rgr[1].fresh) && rg_overflowed()) {
                    if (attempt > 0) throw Error{RELCP_E_DEVICE, "row graph sizing failed"};
                    continue;
                }
                break;
            }
            bool again32 = false, again64 = false;
            if (precision == 32 && lcp_fixed == 0) {
                // an FP32 solve that has not converged within its first chunk
                // is usually a few passes short: a short further chunk, and
                // the polish and the tail again behind it, all waited for
                // together (then chunks twice as long while it has not)
                const RgBufs<float> Bf = rg_bufs<float>(R32, tol);
                const int *done32 = reinterpret_cast<const int *>(pst_h + 1);
                int extra = std::max(4, rgr[0].chunk / 4);
                while (!*done32 && rgr[0].j - 1 < lcp_max_iters) {
                    rg_passes<float>(Bf, R32, std::min(extra, lcp_max_iters - (rgr[0].j - 1)));
                    const StartSrc src{nullptr, {Bf.z0, Bf.z1}, Bf.C.fin, Bf.C.done, (rgr[0].j - 1) & 1};
                    rg_start<double>(R64, dt, tol, nullptr, rgam64.p, &src, true);
                    rg_unpack<double>(R64, B64, tol);
                    launch_tail();
                    wait_report();
                    extra = std::min(64, 2 * extra);
                }
            }
            if (precision == 32) {
                status = rg_finish<float>(R32, B32, tol, it, res, again32);
                if (status == RELCP_OK || status == RELCP_E_LCP_MAXITER) {
                    if (again32) {
                        // the polish started from an unfinished FP32 iterate: again
                        rg_start<double>(R64, dt, tol, rgam64.p, nullptr);
                        rg_unpack<double>(R64, B64, tol);
                        sync();
                    }
                    status = rg_finish<double>(R64, B64, tol, it64, res64, again64);
                }
            } else {
                status = rg_finish<double>(R64, B64, tol, it, res64, again64);
                res = res64;
            }
            if (status == RELCP_OK) {
                if (again32 || again64) {
                    launch_tail();
                    wait_report();
                }
                tail_ready = true;
            }
        } else if (precision == 32) {
            // (the row-graph solve reads the FP64 start and writes the FP64
            // result itself)
            if (!rowgraph_mode()) launch_demote(m, rgam64.p, rgam32.p, stream);
            status = solve<float>(dt, tol, it, res);
            if (status == RELCP_OK || status == RELCP_E_LCP_MAXITER) {
                // FP64 residual of the FP32 iterate, polished in FP64 if needed
                if (!rowgraph_mode()) launch_promote(m, rgam32.p, rgam64.p, stream);
                status = solve<double>(dt, tol, it64, res64);
            }
        } else {
            status = solve<double>(dt, tol, it, res64);
            res = res64;
        }
        iters_total += it + it64;
        if (rec < RELCP_MAX_RECORDED) {
            S.n_contacts[rec] = m;
            S.lcp_iters[rec] = it + it64;
            S.lcp_iters64[rec] = precision == 32 ? it64 : it;
            S.rowgraph_entries[rec] = rowgraph_mode() && rg_valid ? rg_entries : 0;
        }
        S.residual_fp64 = res64;
        S.residual_lowp = res;
        if (status != RELCP_OK) break;
        t_lcp += tm.ms();
        if (!tail_ready) {
            launch_tail();
            wait_report();
        }
        t_narrow += tm.ms();
        int nv = np > 0 ? int_h[0] : 0;
        double maxdisp;
        {
            unsigned long long b = red_h[0];
            std::memcpy(&maxdisp, &b, sizeof(double));
        }
        minphi = np > 0 ? order_key_value(red_h[1]) : 0.0;
        if (rec < RELCP_MAX_RECORDED) {
            S.W[rec] = dbl_h[0];
            S.margin[rec] = np > 0 ? order_key_value(red_h[2]) : 0.0;
        }
        S.max_disp = maxdisp;
        if (!std::isfinite(maxdisp) || !std::isfinite(dbl_h[0])) {
            status = RELCP_E_NAN;
            break;
        }
        if (maxdisp > 0.5 * skin) {
            status = RELCP_E_SKIN;
            break;
        }
        if (nv == 0) break;
        if (rec >= max_rec) {
            if (max_rec == 0) break;  // plain SNSD LCP: accept the first trial
            status = RELCP_E_RECURSION_CAP;
            break;
        }
        // augment: rows generated at C_{n+1}, pulled back (per-row constant)
        ensure_rows(m + nv);
        {
            const int m_old = m;
            compact_flags(pflag.p, np, pcnt.p, sel.p, nullptr, scan_scratch, stream);  // the violators
            // the contact velocities V_n - U_free of the trial (the trial's
            // own arithmetic), which a row-graph trial did not store
            if (rowgraph_mode()) launch_lcp_scatter<double>(0, rows_of<double>(), bodies_of<double>(), PgdCtl{}, 0, stream);
            build_rows(nv, rec + 1, snsdt.p, vc64.p, false, dt);
            rebuild_csr();
            if (resident_mode()) rows_by_packing_append(m_old, nv);
        }
        t_other += tm.ms();
    }
    S.recursions = rec;
    S.lcp_iters_total = iters_total;
    S.n_contacts_final = m;
    if (status == RELCP_OK) {
        S.max_overlap = minphi < 0 ? -minphi : 0.0;
        // accept: C^{k+1} = C_{n+1}; U^{k+1} = V_n
        std::swap(x.p, xt.p);
        std::swap(q.p, qt.p);
        std::swap(geo.p, geot.p);  // the trial's geometry is that of C^{k+1}
        std::swap(u.p, vout.p);  // every trial writes all of vout
        // multiplier sum per pair, for the next warm start (the last trial's
        // SNSD pass set it to the multiplier of the pair's iteration-0 row)
        for (int lv = 1; lv <= rec; ++lv) launch_pair_lambda(m, rrec.p, rpair.p, rgam64.p, lv, lam.p, stream);
        if (!prev_is_list) {
            // the previous-step pairs are the candidate list itself until it is rebuilt
            prev_a.ensure(std::max(np, 1));
            prev_b.ensure(std::max(np, 1));
            if (np > 0) {
                HIP_OK(hipMemcpyAsync(prev_a.p, pa.p, np * sizeof(int), hipMemcpyDeviceToDevice, stream));
                HIP_OK(hipMemcpyAsync(prev_b.p, pb.p, np * sizeof(int), hipMemcpyDeviceToDevice, stream));
            }
            prev_is_list = true;
        }
        std::swap(prev_lam.p, lam.p);
        std::swap(prev_lam.cap, lam.cap);
        vl_used += 2.0 * S.max_disp;
        // keep the multiplier buffer's capacity consistent with ldp
        if ((int)lam.cap < ldp) {
            lam.release();
            lam.ensure(ldp);
        }
        nprev = np;
        m_acc = m;
        m0_last = m0;
        log_valid = log_on;
        hint_ok = true;
        // no wait here: the caller's next call is ordered on the stream
    }
    if (timing) {
        sync();
        collect_timing();
    }
    t_other += tm.ms();
    S.t_narrow = t_narrow;
    S.t_lcp = t_lcp;
    S.t_other = t_other;
    S.n_waits = n_waits;
    S.t_wait = t_wait;
    S.rowgraph_restarts = rg_restarts;
    if (st) *st = S;
    return status;
}

// ===========================================================================
// C ABI
// ===========================================================================
template <typename F>
static int guarded(relcp_ctx *ctx, F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        if (ctx) ctx->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = e.what();
        return RELCP_E_DEVICE;
    }
}

extern "C" {

int relcp_create(const relcp_bodies *bodies, const relcp_shapes *shapes, const relcp_params *params,
                 relcp_ctx **out) {
    if (!out) return RELCP_E_INVALID;
    *out = nullptr;
    relcp_ctx *c = new (std::nothrow) relcp_ctx();
    if (!c) return RELCP_E_OOM;
    try {
        relcp_params P{};
        P.dynamics = RELCP_OVERDAMPED;
        P.precision = 64;
        P.warm_start = RELCP_WS_PREV;
        P.max_recursions = 64;
        P.skin = 0.05;
        if (params) P = *params;
        if (P.dynamics != 0 && P.dynamics != 1) throw Error{RELCP_E_INVALID, "bad dynamics"};
        if (P.precision != 64 && P.precision != 32) throw Error{RELCP_E_INVALID, "precision must be 64 or 32"};
        if (P.warm_start < 0 || P.warm_start > 2) throw Error{RELCP_E_INVALID, "bad warm start"};
        if (P.warm_start == RELCP_WS_LEARNED)
            throw Error{RELCP_E_INVALID, "learned warm start needs a model (relcp_set_warmstart_model)"};
        if (P.max_recursions < 0 || P.max_recursions >= RELCP_MAX_RECORDED)
            throw Error{RELCP_E_INVALID, "max_recursions must be in [0, 64]"};
        if (!(P.skin > 0) || !std::isfinite(P.skin)) throw Error{RELCP_E_INVALID, "skin must be positive"};
        validate(bodies, shapes, &P, P.skin);
        c->dynamics = P.dynamics;
        c->precision = P.precision;
        c->warm_start = P.warm_start;
        c->planar = P.planar ? 1 : 0;
        c->max_rec = P.max_recursions;
        c->lcp_max_iters = P.lcp_max_iters > 0 ? P.lcp_max_iters : 100000;
        c->lcp_fixed = P.lcp_fixed_iters > 0 ? P.lcp_fixed_iters : 0;
        c->skin = P.skin;
        if (P.stream) {
            c->stream = (hipStream_t)P.stream;
        } else {
            HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        c->alloc_host();
        c->upload_bodies(bodies, shapes);
        *out = c;
        return RELCP_OK;
    } catch (const Error &e) {
        delete c;
        return e.code;
    } catch (...) {
        delete c;
        return RELCP_E_DEVICE;
    }
}

void relcp_destroy(relcp_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
}

const char *relcp_last_error(const relcp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int relcp_set_external(relcp_ctx *ctx, const double *f) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        if (!f) {
            ctx->has_fext = false;
            ctx->setup_valid = false;
            return RELCP_OK;
        }
        size_t N = ctx->n;
        std::vector<double> t(6 * N);
        for (size_t i = 0; i < N; ++i)
            for (int k = 0; k < 6; ++k) {
                double v = f[6 * (size_t)ctx->perm[i] + k];
                if (!std::isfinite(v)) throw Error{RELCP_E_INVALID, "non-finite external wrench"};
                t[k * N + i] = v;
            }
        HIP_OK(hipMemcpyAsync(ctx->fext.p, t.data(), 6 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        ctx->sync();
        ctx->has_fext = true;
        ctx->setup_valid = false;
        return RELCP_OK;
    });
}

int relcp_step(relcp_ctx *ctx, double dt, double overlap_tol, double lcp_tol, relcp_step_stats *stats) {
    if (!ctx) return RELCP_E_INVALID;
    if (!(dt > 0) || !(overlap_tol > 0) || !(lcp_tol > 0) || !std::isfinite(dt)) {
        ctx->err = "dt, overlap_tol and lcp_tol must be positive";
        return RELCP_E_INVALID;
    }
    return guarded(ctx, [&]() -> int {
        int rc = ctx->step(dt, overlap_tol, lcp_tol, stats);
        if (rc != RELCP_OK) {
            static const char *names[] = {"ok", "invalid", "out of memory", "device", "LCP iteration cap",
                                          "recursion cap", "skin exceeded", "non-finite value", "capacity"};
            ctx->err = std::string("step failed: ") + names[-rc];
        }
        return rc;
    });
}

static int get_state_impl(const relcp_ctx *cc, double *x, double *q, double *u, double *w, bool device) {
    relcp_ctx *ctx = const_cast<relcp_ctx *>(cc);
    return guarded(ctx, [&]() -> int {
        size_t N = ctx->n;
        if (device) {
            auto conv = [&](const double *src, int c0, int comps, double *dst) {
                if (!dst) return;
                hipLaunchKernelGGL(k_soa_to_aos, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (int)N, comps, src,
                                   (int)N, c0, dst, comps, ctx->perm_d.p);
            };
            conv(ctx->x.p, 0, 3, x);
            conv(ctx->q.p, 0, 4, q);
            conv(ctx->u.p, 0, 3, u);
            conv(ctx->u.p, 3, 3, w);
            ctx->sync();
            return RELCP_OK;
        }
        std::vector<double> t(6 * N);
        auto down = [&](const double *src, int c0, int comps, double *dst) {
            if (!dst) return;
            HIP_OK(hipMemcpyAsync(t.data(), src + c0 * N, comps * N * sizeof(double), hipMemcpyDeviceToHost,
                                  ctx->stream));
            ctx->sync();
            for (size_t i = 0; i < N; ++i)
                for (int k = 0; k < comps; ++k) dst[comps * (size_t)ctx->perm[i] + k] = t[k * N + i];
        };
        down(ctx->x.p, 0, 3, x);
        down(ctx->q.p, 0, 4, q);
        down(ctx->u.p, 0, 3, u);
        down(ctx->u.p, 3, 3, w);
        return RELCP_OK;
    });
}

int relcp_get_state(const relcp_ctx *ctx, double *x, double *q, double *u, double *w) {
    if (!ctx) return RELCP_E_INVALID;
    return get_state_impl(ctx, x, q, u, w, false);
}

int relcp_get_state_device(const relcp_ctx *ctx, double *x, double *q, double *u, double *w) {
    if (!ctx) return RELCP_E_INVALID;
    return get_state_impl(ctx, x, q, u, w, true);
}

int relcp_set_state(relcp_ctx *ctx, const relcp_bodies *bodies, const relcp_shapes *shapes) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        validate(bodies, shapes, nullptr, ctx->skin);
        for (int i = 0; i < bodies->n; ++i) {
            if (ctx->dynamics == RELCP_INERTIAL && shapes->kind[i] != RELCP_ELLIPSOID)
                throw Error{RELCP_E_INVALID, "inertial needs ellipsoids"};
            if (shapes->kind[i] == RELCP_TORUS && (ctx->planar || ctx->warm_start == RELCP_WS_LEARNED))
                throw Error{RELCP_E_INVALID, "tori: not in a monolayer, no learned warm start"};
        }
        ctx->upload_bodies(bodies, shapes);
        return RELCP_OK;
    });
}

int relcp_affine_rescale(relcp_ctx *ctx, double s) {
    if (!ctx) return RELCP_E_INVALID;
    if (!(s > 0) || !std::isfinite(s)) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        for (int pk = 0; pk < ctx->nbatch; ++pk)
            for (int k = 0; k < 3; ++k) {
                double L = ctx->box[3 * pk + k] * s;
                if (L > 0 && L < 2.0 * (ctx->rmax[pk] + ctx->skin))
                    throw Error{RELCP_E_INVALID, "box would become smaller than 2 (R_max + skin)"};
            }
        for (auto &v : ctx->box) v *= s;
        // positions and the device copy of the boxes, stream-ordered (no wait)
        const int nbox = (int)ctx->box.size();
        hipLaunchKernelGGL(k_scale, dim3(nblk(std::max(3LL * ctx->n, (long long)nbox), 256)), dim3(256), 0,
                           ctx->stream, 3 * ctx->n, ctx->x.p, nbox, ctx->boxes.p, s);
        HIP_OK(hipGetLastError());
        // a pair of the list is at most 2 R_max + radius apart: its gap shrinks by at most (1 - s) times that
        double rm = 0.0;
        for (double r : ctx->rmax) rm = std::max(rm, r);
        ctx->vl_used += std::max(0.0, 1.0 - s) * (2.0 * rm + ctx->vl_radius());
        return RELCP_OK;
    });
}

__global__ void k_scale_packings(int n, double *__restrict__ x, const int *__restrict__ body_batch,
                                 const double *__restrict__ s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double f = s[body_batch[i]];
        x[i] *= f;
        x[n + i] *= f;
        x[2 * n + i] *= f;
    }
}

int relcp_affine_rescale_packings(relcp_ctx *ctx, const double *s) {
    if (!ctx || !s) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        for (int pk = 0; pk < ctx->nbatch; ++pk) {
            if (!(s[pk] > 0) || !std::isfinite(s[pk])) throw Error{RELCP_E_INVALID, "scale factors must be positive"};
            for (int k = 0; k < 3; ++k) {
                double L = ctx->box[3 * pk + k] * s[pk];
                if (L > 0 && L < 2.0 * (ctx->rmax[pk] + ctx->skin))
                    throw Error{RELCP_E_INVALID, "box would become smaller than 2 (R_max + skin)"};
            }
        }
        for (int pk = 0; pk < ctx->nbatch; ++pk)
            for (int k = 0; k < 3; ++k) ctx->box[3 * pk + k] *= s[pk];
        DBuf<double> sd;
        sd.ensure(ctx->nbatch);
        HIP_OK(hipMemcpyAsync(sd.p, s, ctx->nbatch * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(hipMemcpyAsync(ctx->boxes.p, ctx->box.data(), ctx->box.size() * sizeof(double),
                              hipMemcpyHostToDevice, ctx->stream));
        hipLaunchKernelGGL(k_scale_packings, dim3(nblk(ctx->n, 256)), dim3(256), 0, ctx->stream, ctx->n, ctx->x.p,
                           ctx->body_batch.p, sd.p);
        ctx->sync();
        sd.release();
        double shrink = 0.0;
        for (int pk = 0; pk < ctx->nbatch; ++pk)
            shrink = std::max(shrink, std::max(0.0, 1.0 - s[pk]) * (2.0 * ctx->rmax[pk] + ctx->vl_radius()));
        ctx->vl_used += shrink;
        return RELCP_OK;
    });
}

// cylinder length l (shape component 1) of every spherocylinder grows by
// dl; `ready` counts those at or past l_div afterwards
__global__ void k_grow(int n, const int *__restrict__ kind, double *__restrict__ p, double dl, double l_div,
                       int *__restrict__ ready) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int r = 0;
    if (i < n && kind[i] == RELCP_SPHEROCYLINDER) {
        const double l = fmax(0.0, p[n + i] + dl);
        p[n + i] = l;
        r = l >= l_div;
    }
    if (ready) {
        for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) r += __shfl_xor(r, o, RELCP_WAVE);
        if ((threadIdx.x & (RELCP_WAVE - 1)) == 0 && r) atomicAdd(ready, r);
    }
}

int relcp_grow(relcp_ctx *ctx, double dl, double l_div, int32_t *n_ready) {
    if (!ctx) return RELCP_E_INVALID;
    if (!std::isfinite(dl) || std::isnan(l_div)) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        const int N = ctx->n;
        DBuf<int> cnt;
        if (n_ready) {
            cnt.ensure(1);
            HIP_OK(hipMemsetAsync(cnt.p, 0, sizeof(int), ctx->stream));
        }
        if (N > 0)
            hipLaunchKernelGGL(k_grow, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, N, ctx->kind.p, ctx->p.p, dl,
                               l_div, n_ready ? cnt.p : nullptr);
        HIP_OK(hipGetLastError());
        // a cap tip moves dl / 2 along the axis: bounding radii grow by dl / 2
        // and the gap of a pair shrinks by at most dl (the kept candidate
        // list accounts for it; a shrink only widens gaps, and the bounding
        // radius bound is kept); mobility and geometry are set up again
        if (dl > 0) {
            for (int pk = 0; pk < ctx->nbatch; ++pk) ctx->rmax[pk] += 0.5 * dl;
            ctx->vl_used += dl;
        }
        ctx->setup_valid = false;
        if (n_ready) {
            int h = 0;
            HIP_OK(hipMemcpyAsync(&h, cnt.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            cnt.release();
            *n_ready = h;
        }
        return RELCP_OK;
    });
}

int relcp_divide(relcp_ctx *ctx, double l_div, const double *jitter, int32_t n_jitter, int32_t *n_divided) {
    if (!ctx || !(l_div > 0) || !std::isfinite(l_div) || n_jitter < 0 || (n_jitter > 0 && !jitter))
        return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        if (ctx->nbatch != 1) throw Error{RELCP_E_INVALID, "division needs a context of one packing"};
        const size_t N = ctx->n;
        std::vector<double> x(3 * N), q(4 * N), u(3 * N), w(3 * N), sp(3 * N), rho(N), t(3 * N);
        std::vector<int> kind(N), kt(N);
        int rc = get_state_impl(ctx, x.data(), q.data(), u.data(), w.data(), false);
        if (rc != RELCP_OK) return rc;
        // shapes, drag and kinds back in the caller's order
        HIP_OK(hipMemcpyAsync(t.data(), ctx->p.p, 3 * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipMemcpyAsync(rho.data(), ctx->rho.p, N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipMemcpyAsync(kt.data(), ctx->kind.p, N * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        std::vector<double> rh(N);
        for (size_t i = 0; i < N; ++i) {
            const size_t c = ctx->perm[i];
            for (int k = 0; k < 3; ++k) sp[3 * c + k] = t[k * N + i];
            rh[c] = rho[i];
            kind[c] = kt[i];
        }
        std::vector<size_t> div;
        for (size_t c = 0; c < N; ++c)
            if (kind[c] == RELCP_SPHEROCYLINDER && sp[3 * c + 1] >= l_div) div.push_back(c);
        if (n_divided) *n_divided = (int32_t)div.size();
        if (div.empty()) return RELCP_OK;
        if ((size_t)n_jitter < 2 * div.size()) throw Error{RELCP_E_INVALID, "two jitter angles per dividing cell"};
        for (size_t c : div)
            if (0.5 * sp[3 * c + 1] - sp[3 * c] < 0.0)
                throw Error{RELCP_E_INVALID, "a dividing cell shorter than its diameter"};
        const size_t M = N + div.size();
        x.resize(3 * M); q.resize(4 * M); u.resize(3 * M); w.resize(3 * M); sp.resize(3 * M); rh.resize(M);
        kind.resize(M);
        for (size_t k = 0; k < div.size(); ++k) {
            const size_t a = div[k], b = N + k;
            const double r = sp[3 * a], l = sp[3 * a + 1];
            const double *qa = &q[4 * a];
            // body x axis (the cell's axis) in the world frame
            const double ax = 1.0 - 2.0 * (qa[2] * qa[2] + qa[3] * qa[3]), ay = 2.0 * (qa[1] * qa[2] + qa[0] * qa[3]),
                         az = 2.0 * (qa[1] * qa[3] - qa[0] * qa[2]);
            // the daughters are the two halves of the parent, tip to tip:
            // total length (l + 2r) / 2 each, centres a quarter of the
            // parent's total length from its centre
            const double h = 0.25 * (l + 2.0 * r);
            const double p0[4] = {qa[0], qa[1], qa[2], qa[3]};
            double xc[3] = {x[3 * a], x[3 * a + 1], x[3 * a + 2]};
            for (int d = 0; d < 2; ++d) {
                const size_t o = d ? b : a;
                const double sgn = d ? -1.0 : 1.0;
                x[3 * o] = xc[0] + sgn * h * ax;
                x[3 * o + 1] = xc[1] + sgn * h * ay;
                x[3 * o + 2] = xc[2] + sgn * h * az;
                // turn about the world z axis by the daughter's jitter angle
                const double th = jitter[2 * k + d], cz = std::cos(0.5 * th), sz = std::sin(0.5 * th);
                q[4 * o] = cz * p0[0] - sz * p0[3];
                q[4 * o + 1] = cz * p0[1] - sz * p0[2];
                q[4 * o + 2] = cz * p0[2] + sz * p0[1];
                q[4 * o + 3] = cz * p0[3] + sz * p0[0];
                const double nq = std::sqrt(q[4 * o] * q[4 * o] + q[4 * o + 1] * q[4 * o + 1] +
                                            q[4 * o + 2] * q[4 * o + 2] + q[4 * o + 3] * q[4 * o + 3]);
                for (int j = 0; j < 4; ++j) q[4 * o + j] /= nq;
                for (int j = 0; j < 3; ++j) {
                    u[3 * o + j] = u[3 * a + j];
                    w[3 * o + j] = w[3 * a + j];
                }
                sp[3 * o] = r;
                sp[3 * o + 1] = 0.5 * l - r;
                sp[3 * o + 2] = 0.0;
                rh[o] = rh[a];
                kind[o] = RELCP_SPHEROCYLINDER;
            }
        }
        const std::vector<double> bx = ctx->box;  // upload_bodies replaces ctx->box
        relcp_bodies B{(int32_t)M, x.data(), q.data(), u.data(), w.data(), 1, nullptr, bx.data()};
        relcp_shapes S{kind.data(), sp.data(), rh.data()};
        validate(&B, &S, nullptr, ctx->skin);
        ctx->upload_bodies(&B, &S);
        return RELCP_OK;
    });
}

int relcp_get_contacts(const relcp_ctx *cc, int32_t *ia, int32_t *ib, int32_t *recursion_added, double *gamma,
                       double *phi_at_discovery, double *normal) {
    relcp_ctx *ctx = const_cast<relcp_ctx *>(cc);
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        size_t M = ctx->m_acc;
        if (M == 0) return RELCP_OK;
        auto cp = [&](void *dst, const void *src, size_t bytes) {
            if (dst) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
        };
        cp(recursion_added, ctx->rrec.p, M * 4);
        cp(gamma, ctx->rgam64.p, M * 8);
        cp(phi_at_discovery, ctx->rphi64.p, M * 8);
        std::vector<double> t;
        if (normal) {
            t.resize(3 * M);
            for (int k = 0; k < 3; ++k) cp(t.data() + k * M, ctx->rn64.p + (size_t)k * ctx->ldr, M * 8);
        }
        std::vector<int> ha(M), hb(M);
        HIP_OK(hipMemcpyAsync(ha.data(), ctx->ria.p, M * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipMemcpyAsync(hb.data(), ctx->rib.p, M * 4, hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        // caller's indices, first body the smaller index, normal from the
        // first body to the second
        for (size_t i = 0; i < M; ++i) {
            int a = ctx->perm[ha[i]], b = ctx->perm[hb[i]];
            double sg = a < b ? 1.0 : -1.0;
            if (ia) ia[i] = a < b ? a : b;
            if (ib) ib[i] = a < b ? b : a;
            if (normal)
                for (int k = 0; k < 3; ++k) normal[3 * i + k] = sg * t[k * M + i];
        }
        return RELCP_OK;
    });
}

int relcp_set_lcp_config(relcp_ctx *ctx, int32_t mode, int32_t block, int32_t lds) {
    if (!ctx) return RELCP_E_INVALID;
    if (mode < 0 || mode > 4 || (block != 256 && block != 512 && block != 1024)) {
        ctx->err = "mode must be 0..4 and block 256, 512 or 1024";
        return RELCP_E_INVALID;
    }
    ctx->lcp_mode = mode;
    ctx->res_block = block;
    ctx->res_lds = lds ? 1 : 0;
    return RELCP_OK;
}

// Time every LCP configuration on the rows of the last accepted step, each
// solve from zero (the step's own multipliers already solve that LCP), and
// keep the fastest; the step's multipliers are restored afterwards.
int relcp_autotune(relcp_ctx *ctx, double dt, double lcp_tol, int32_t reps, int32_t *config, double *ms) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        if (ctx->m_acc <= 0 || ctx->m != ctx->m_acc) throw Error{RELCP_E_INVALID, "autotune needs an accepted step"};
        if (reps < 1) reps = 1;
        const int M = ctx->m;
        DBuf<double> s64;
        DBuf<float> s32;
        s64.ensure(2 * (size_t)M);
        s32.ensure(2 * (size_t)M);
        auto cp = [&](void *dst, const void *src, size_t b) {
            HIP_OK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, ctx->stream));
        };
        cp(s64.p, ctx->rgam64.p, M * 8);
        cp(s64.p + M, ctx->rg64.p, M * 8);
        cp(s32.p, ctx->rgam32.p, M * 4);
        cp(s32.p + M, ctx->rg32.p, M * 4);
        {
            // group the rows by packing (the list is not kept in grid mode)
            std::vector<int> ia(M), bb(ctx->n), order(M);
            HIP_OK(hipMemcpyAsync(ia.data(), ctx->ria.p, M * 4, hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipMemcpyAsync(bb.data(), ctx->body_batch.p, ctx->n * 4, hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            std::vector<int> cnt(ctx->nbatch + 1, 0);
            for (int r = 0; r < M; ++r) cnt[bb[ia[r]] + 1]++;
            for (int k = 0; k < ctx->nbatch; ++k) cnt[k + 1] += cnt[k];
            std::vector<int> pos(cnt.begin(), cnt.end() - 1);
            for (int r = 0; r < M; ++r) order[pos[bb[ia[r]]]++] = r;
            HIP_OK(hipMemcpyAsync(ctx->rlist.p, order.data(), M * 4, hipMemcpyHostToDevice, ctx->stream));
            HIP_OK(hipMemcpyAsync(ctx->roff.p, cnt.data(), (ctx->nbatch + 1) * 4, hipMemcpyHostToDevice,
                                  ctx->stream));
            ctx->sync();
        }
        struct Cfg {
            int mode, block, lds;
        };
        std::vector<Cfg> cfgs = {{1, 256, 0}};
        for (int b : {256, 512, 1024})
            for (int l : {0, 1}) cfgs.push_back({2, b, l});
        cfgs.push_back({3, 256, 0});
        cfgs.push_back({4, 256, 0});
        const int save_mode = ctx->lcp_mode, save_block = ctx->res_block, save_lds = ctx->res_lds;
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        double best = 1e300;
        Cfg bestc = cfgs[0];
        for (const Cfg &c : cfgs) {
            if (c.lds && (size_t)6 * ctx->maxpk * (ctx->precision == 32 ? 4 : 8) > 150 * 1024) continue;
            ctx->lcp_mode = c.mode;
            ctx->res_block = c.block;
            ctx->res_lds = c.lds;
            double tot = 0.0;
            // one untimed solve first (graph instantiation, buffer growth)
            for (int r = -1; r < reps; ++r) {
                // from zero: the last step's multipliers solve this LCP already
                HIP_OK(hipMemsetAsync(ctx->rgam64.p, 0, M * 8, ctx->stream));
                HIP_OK(hipMemsetAsync(ctx->rgam32.p, 0, M * 4, ctx->stream));
                int it = 0;
                double res = 0;
                HIP_OK(hipEventRecord(e0, ctx->stream));
                int rc = ctx->precision == 32 ? ctx->solve<float>(dt, lcp_tol, it, res)
                                              : ctx->solve<double>(dt, lcp_tol, it, res);
                HIP_OK(hipEventRecord(e1, ctx->stream));
                HIP_OK(hipEventSynchronize(e1));
                if (rc != RELCP_OK) {
                    tot = 1e300;
                    break;
                }
                float t = 0.f;
                HIP_OK(hipEventElapsedTime(&t, e0, e1));
                if (r >= 0) tot += t;
            }
            double avg = tot / reps;
            if (ms) ms[&c - &cfgs[0]] = avg;
            if (avg < best) {
                best = avg;
                bestc = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        cp(ctx->rgam64.p, s64.p, M * 8);
        cp(ctx->rg64.p, s64.p + M, M * 8);
        cp(ctx->rgam32.p, s32.p, M * 4);
        cp(ctx->rg32.p, s32.p + M, M * 4);
        ctx->sync();
        s64.release();
        s32.release();
        (void)save_mode; (void)save_block; (void)save_lds;
        ctx->lcp_mode = bestc.mode;
        ctx->res_block = bestc.block;
        ctx->res_lds = bestc.lds;
        if (config) {
            config[0] = bestc.mode;
            config[1] = bestc.block;
            config[2] = bestc.lds;
        }
        return RELCP_OK;
    });
}

int relcp_set_timing(relcp_ctx *ctx, int32_t enable) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        ctx->sync();
        ctx->collect_timing();
        ctx->timing = enable != 0;
        return RELCP_OK;
    });
}

int relcp_get_timing(relcp_ctx *ctx, int32_t *count, double *ms, int32_t reset) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        ctx->sync();
        ctx->collect_timing();
        for (int k = 0; k < relcp_ctx::kClasses; ++k) {
            if (count) count[k] = (int32_t)ctx->t_count[k];
            if (ms) ms[k] = ctx->t_ms[k];
            if (reset) {
                ctx->t_count[k] = 0;
                ctx->t_ms[k] = 0.0;
            }
        }
        return RELCP_OK;
    });
}

// ---------------------------------------------------------------------------
// learned warm start
// ---------------------------------------------------------------------------
int relcp_set_warm_start(relcp_ctx *ctx, int32_t mode) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        if (mode < RELCP_WS_COLD || mode > RELCP_WS_LEARNED) throw Error{RELCP_E_INVALID, "bad warm start"};
        if (mode == RELCP_WS_LEARNED && !ctx->has_model)
            throw Error{RELCP_E_INVALID, "learned warm start needs a model (relcp_set_warmstart_model)"};
        if (mode == RELCP_WS_LEARNED && ctx->has_torus)
            throw Error{RELCP_E_INVALID, "the learned warm start covers ellipsoids and spherocylinders"};
        ctx->warm_start = mode;
        return RELCP_OK;
    });
}

int relcp_set_warmstart_model(relcp_ctx *ctx, const float *params, const float *norm) {
    if (!ctx) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        if (!params || !norm) throw Error{RELCP_E_INVALID, "null model"};
        for (int k = 0; k < MLP_NPARAM; ++k)
            if (!std::isfinite(params[k])) throw Error{RELCP_E_INVALID, "non-finite model weight"};
        for (int k = 0; k < MLP_NORM; ++k)
            if (!std::isfinite(norm[k]) || (k >= 8 && !(norm[k] > 0)))
                throw Error{RELCP_E_INVALID, "feature std and multiplier scale must be positive"};
        ctx->mlp_w.ensure(MLP_NPARAM);
        HIP_OK(hipMemcpyAsync(ctx->mlp_w.p, params, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice,
                              ctx->stream));
        ctx->sync();
        std::memcpy(ctx->mlp_norm, norm, sizeof(ctx->mlp_norm));
        ctx->has_model = true;
        return RELCP_OK;
    });
}

int relcp_enable_contact_log(relcp_ctx *ctx, int32_t on) {
    if (!ctx) return RELCP_E_INVALID;
    ctx->log_on = on != 0;
    if (!ctx->log_on) ctx->log_valid = false;
    return RELCP_OK;
}

int relcp_log_contacts(relcp_ctx *ctx, float *feat, float *gamma, int32_t *ia, int32_t *ib, int32_t cap,
                       int32_t *count) {
    if (!ctx || !count || cap < 0) return RELCP_E_INVALID;
    return guarded(ctx, [&]() -> int {
        const int m0 = ctx->log_valid ? ctx->m0_last : 0;
        *count = m0;
        if (m0 > cap) return RELCP_E_CAPACITY;
        launch_log_rows(m0, ctx->feat.p, ctx->rgam64.p, ctx->rowscale.p, ctx->ria.p, ctx->rib.p, ctx->perm_d.p, feat,
                        gamma, ia, ib, ctx->stream);
        HIP_OK(hipGetLastError());
        ctx->sync();
        return RELCP_OK;
    });
}

size_t relcp_mlp_workspace_bytes(int32_t n) {
    return n < 0 ? 0 : (size_t)mlp_slots(n) * MLP_SLOT * sizeof(float);
}

static bool mlp_norm_ok(const float *norm) {
    if (!norm) return false;
    for (int k = 0; k < MLP_NORM; ++k)
        if (!std::isfinite(norm[k]) || (k >= 8 && !(norm[k] > 0))) return false;
    return true;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

int relcp_mlp_forward(const float *params, const float *norm, int32_t n, const float *feat, const int32_t *idx,
                      float *out, void *stream) {
    if (n < 0 || (n > 0 && (!params || !feat || !out)) || !mlp_norm_ok(norm)) return RELCP_E_INVALID;
    if (n > 0 && !aligned16(params)) return RELCP_E_INVALID;
    try {
        MlpArgs a{};
        a.n = n; a.idx = idx; a.X = feat; a.params = params; a.out32 = out;
        std::memcpy(a.norm, norm, sizeof(a.norm));
        launch_mlp_forward(a, (hipStream_t)stream);
        HIP_OK(hipGetLastError());
        return RELCP_OK;
    } catch (const Error &e) {
        return e.code;
    }
}

int relcp_mlp_grad(const float *params, const float *norm, int32_t n, const float *feat, const float *target,
                   const int32_t *idx, float *grad, float *loss, void *work, size_t work_bytes, void *stream) {
    if (n < 0 || !params || !grad || (n > 0 && (!feat || !target)) || !mlp_norm_ok(norm)) return RELCP_E_INVALID;
    if (n > 0 && (!work || work_bytes < relcp_mlp_workspace_bytes(n) || !aligned16(params))) return RELCP_E_INVALID;
    try {
        MlpArgs a{};
        a.n = n; a.idx = idx; a.X = feat; a.params = params; a.y = target;
        a.scale2 = n > 0 ? 2.0f / (float)n : 0.0f;
        a.partial = (float *)work;
        std::memcpy(a.norm, norm, sizeof(a.norm));
        launch_mlp_grad(a, grad, loss, (hipStream_t)stream);
        HIP_OK(hipGetLastError());
        return RELCP_OK;
    } catch (const Error &e) {
        return e.code;
    }
}

int relcp_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, void *stream) {
    if (!params || !grad || !m || !v || t < 1 || !(lr > 0) || !std::isfinite(lr)) return RELCP_E_INVALID;
    try {
        launch_adam(params, grad, m, v, lr, t, (hipStream_t)stream);
        HIP_OK(hipGetLastError());
        return RELCP_OK;
    } catch (const Error &e) {
        return e.code;
    }
}

// ---------------------------------------------------------------------------
// stand-alone operations
// ---------------------------------------------------------------------------
int relcp_snsd_device(int32_t nb, const double *x, const double *q, const int32_t *kind, const double *p, int32_t m,
                      const int32_t *pa, const int32_t *pb, const double *box, int32_t planar, double *out,
                      void *stream) {
    if (nb <= 0 || m < 0 || !x || !q || !kind || !p || (m > 0 && (!pa || !pb || !out)) || !box)
        return RELCP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    try {
        DBuf<double> geo, Rb, boxes;
        geo.ensure(6 * (size_t)nb);
        Rb.ensure(nb);
        boxes.ensure(3);
        HIP_OK(hipMemcpyAsync(boxes.p, box, 3 * sizeof(double), hipMemcpyHostToDevice, s));
        BodySetupArgs ba{};
        ba.nb = nb; ba.q = q; ba.ldq = nb; ba.kind = kind; ba.p = p; ba.ldp = nb; ba.geo = geo.p; ba.ldg = nb;
        ba.Rb = Rb.p; ba.K = nullptr;
        launch_body_setup(ba, s);
        SnsdArgs sa{};
        sa.m = m; sa.pa = pa; sa.pb = pb; sa.body_batch = nullptr; sa.x = x; sa.ldx = nb; sa.geo = geo.p; sa.ldg = nb;
        sa.kind = kind; sa.p = p; sa.ldp = nb; sa.boxes = boxes.p; sa.planar = planar; sa.hint = nullptr; sa.out = out;
        sa.ldo = m; sa.mode = 0; sa.thresh = 0; sa.eps = 0; sa.flag = nullptr; sa.minphi = nullptr;
        launch_snsd_pairs(sa, s);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
        geo.release(); Rb.release(); boxes.release();
        return RELCP_OK;
    } catch (const Error &e) {
        return e.code;
    }
}

int relcp_broadphase_device(int32_t nb, const double *x, const int32_t *kind, const double *p, const double *box,
                            double skin, int32_t cap, int32_t *pa, int32_t *pb, int32_t *m, void *stream) {
    if (nb <= 0 || !x || !kind || !p || !box || !m || !(skin >= 0)) return RELCP_E_INVALID;
    relcp_ctx c;
    c.stream = (hipStream_t)stream;
    try {
        c.alloc_host();
        c.n = nb;
        c.nbatch = 1;
        c.boff = {0, nb};
        c.box.assign(box, box + 3);
        c.body_batch.ensure(nb);
        HIP_OK(hipMemsetAsync(c.body_batch.p, 0, nb * sizeof(int), c.stream));
        c.Rb.ensure(nb);
        DBuf<double> geo;
        geo.ensure(6 * (size_t)nb);
        DBuf<double> qd;
        qd.ensure(4 * (size_t)nb);
        // bounding radii do not depend on orientation: any unit quaternion
        std::vector<double> qh(4 * (size_t)nb, 0.0);
        for (int i = 0; i < nb; ++i) qh[i] = 1.0;
        HIP_OK(hipMemcpyAsync(qd.p, qh.data(), qh.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
        BodySetupArgs ba{};
        ba.nb = nb; ba.q = qd.p; ba.ldq = nb; ba.kind = kind; ba.p = p; ba.ldp = nb; ba.geo = geo.p; ba.ldg = nb;
        ba.Rb = c.Rb.p; ba.K = nullptr;
        launch_body_setup(ba, c.stream);
        std::vector<double> ph(3 * (size_t)nb);
        std::vector<int> kh(nb);
        HIP_OK(hipMemcpyAsync(ph.data(), p, ph.size() * 8, hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipMemcpyAsync(kh.data(), kind, kh.size() * 4, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        double R = 0;
        for (int i = 0; i < nb; ++i)
            R = std::max(R, kh[i] == 0 ? std::max(ph[i], std::max(ph[nb + i], ph[2 * nb + i]))
                                       : 0.5 * ph[nb + i] + ph[i]);
        c.rmax = {R};
        for (int k = 0; k < 3; ++k)
            if (box[k] > 0 && box[k] < 2.0 * (R + skin)) throw Error{RELCP_E_INVALID, "box too small"};
        c.broadphase(x, skin);
        *m = c.np;
        int k = std::min(c.np, cap);
        if (k > 0 && pa && pb) {
            HIP_OK(hipMemcpyAsync(pa, c.pa.p, k * sizeof(int), hipMemcpyDeviceToDevice, c.stream));
            HIP_OK(hipMemcpyAsync(pb, c.pb.p, k * sizeof(int), hipMemcpyDeviceToDevice, c.stream));
        }
        c.sync();
        geo.release();
        qd.release();
        c.stream = nullptr;
        return RELCP_OK;
    } catch (const Error &e) {
        c.stream = nullptr;
        return e.code;
    }
}

__global__ void k_rows_from_user(int m, int ld, const double *__restrict__ n, const double *__restrict__ ta,
                                 const double *__restrict__ tb, const double *__restrict__ qv,
                                 const int *__restrict__ ia, const int *__restrict__ ib, const double *__restrict__ K,
                                 int ldb, double dt, double *n64, double *ta64, double *tb64, double *qv64,
                                 double *dA64, float *n32, float *ta32, float *tb32, float *qv32, float *dA32) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    d3 nn = mk(n[r], n[m + r], n[2 * m + r]);
    d3 a = mk(ta[r], ta[m + r], ta[2 * m + r]);
    d3 b = mk(tb[r], tb[m + r], tb[2 * m + r]);
    auto quad = [&](int i, d3 t) {
        double tr = nn.x * nn.x * K[i] + nn.y * nn.y * K[ldb + i] + nn.z * nn.z * K[2 * ldb + i];
        sym3 R{K[3 * ldb + i], K[4 * ldb + i], K[5 * ldb + i], K[6 * ldb + i], K[7 * ldb + i], K[8 * ldb + i]};
        return tr + dot(t, mul(R, t));
    };
    double dA = dt * (quad(ia[r], a) + quad(ib[r], b));
    if (!(dA > 0.0)) dA = 1.0;
    double nv[3] = {nn.x, nn.y, nn.z}, av[3] = {a.x, a.y, a.z}, bv[3] = {b.x, b.y, b.z};
    for (int k = 0; k < 3; ++k) {
        n64[k * ld + r] = nv[k];
        ta64[k * ld + r] = av[k];
        tb64[k * ld + r] = bv[k];
        n32[k * ld + r] = (float)nv[k];
        ta32[k * ld + r] = (float)av[k];
        tb32[k * ld + r] = (float)bv[k];
    }
    qv64[r] = qv[r];
    qv32[r] = (float)qv[r];
    dA64[r] = dA;
    dA32[r] = (float)dA;
}

__global__ void k_K_from_user(int nb, const double *__restrict__ kt, const double *__restrict__ Kr, int planar,
                              double *K, float *K32) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double v[9];
    for (int k = 0; k < 3; ++k) v[k] = kt[i];
    for (int k = 0; k < 6; ++k) v[3 + k] = Kr[k * nb + i];
    if (planar) {
        v[2] = 0.0;
        v[3] = v[4] = v[6] = v[7] = v[8] = 0.0;
    }
    for (int k = 0; k < 9; ++k) {
        K[k * nb + i] = v[k];
        K32[k * nb + i] = (float)v[k];
    }
}

int relcp_lcp_solve_device(int32_t nb, int32_t m, const int32_t *ia, const int32_t *ib, const double *n,
                           const double *ta, const double *tb, const double *qv, const double *kt, const double *Kr,
                           double dt, int32_t planar, int32_t precision, int32_t mode, double tol, int32_t max_iters,
                           double *gamma, int32_t *iters, double *residual, void *stream) {
    if (nb <= 0 || m < 0 || !(dt > 0) || (precision != 32 && precision != 64) || !gamma || !kt || !Kr ||
        (mode != 0 && mode != 1 && mode != 3 && mode != 4))
        return RELCP_E_INVALID;
    relcp_ctx c;
    c.stream = (hipStream_t)stream;
    try {
        c.alloc_host();
        c.n = nb;
        c.lcp_mode = mode == 0 ? 4 : mode;
        c.k_from_setup = false;
        c.lcp_max_iters = max_iters > 0 ? max_iters : 100000;
        c.K.ensure(9 * (size_t)nb);
        c.K32.ensure(9 * (size_t)nb);
        c.vc64.ensure(6 * (size_t)nb);
        c.vc32.ensure(6 * (size_t)nb);
        hipLaunchKernelGGL(k_K_from_user, dim3(nblk(nb, 256)), dim3(256), 0, c.stream, nb, kt, Kr, planar, c.K.p,
                           c.K32.p);
        c.ensure_rows(std::max(m, 1));
        c.m = m;
        if (m > 0) {
            HIP_OK(hipMemcpyAsync(c.ria.p, ia, m * 4, hipMemcpyDeviceToDevice, c.stream));
            HIP_OK(hipMemcpyAsync(c.rib.p, ib, m * 4, hipMemcpyDeviceToDevice, c.stream));
            HIP_OK(hipMemcpyAsync(c.rgam64.p, gamma, m * 8, hipMemcpyDeviceToDevice, c.stream));
            hipLaunchKernelGGL(k_rows_from_user, dim3(nblk(m, 256)), dim3(256), 0, c.stream, m, c.ldr, n, ta, tb, qv,
                               ia, ib, c.K.p, nb, dt, c.rn64.p, c.rta64.p, c.rtb64.p, c.rqv64.p, c.rdA64.p, c.rn32.p,
                               c.rta32.p, c.rtb32.p, c.rqv32.p, c.rdA32.p);
        }
        c.rows32_ok = true;
        c.rebuild_csr();
        int it = 0, it64 = 0, rc;
        double res = 0, res64 = 0;
        if (precision == 32) {
            if (!c.rowgraph_mode()) launch_demote(m, c.rgam64.p, c.rgam32.p, c.stream);
            rc = c.solve<float>(dt, tol, it, res);
            if (!c.rowgraph_mode()) launch_promote(m, c.rgam32.p, c.rgam64.p, c.stream);
            if (rc == RELCP_OK || rc == RELCP_E_LCP_MAXITER) rc = c.solve<double>(dt, tol, it64, res64);
        } else {
            rc = c.solve<double>(dt, tol, it, res64);
        }
        if (m > 0) HIP_OK(hipMemcpyAsync(gamma, c.rgam64.p, m * 8, hipMemcpyDeviceToDevice, c.stream));
        c.sync();
        if (iters) *iters = it + it64;
        if (residual) *residual = res64;
        c.stream = nullptr;
        return rc;
    } catch (const Error &e) {
        c.stream = nullptr;
        return e.code;
    }
}

int relcp_exclusive_scan_device(const int32_t *in, int32_t *out, int32_t n, int32_t *total, void *stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return RELCP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    DBuf<int> scratch;
    try {
        exclusive_scan(in, out, n, total, scratch, s);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
    } catch (const Error &e) {
        scratch.release();
        return e.code;
    }
    scratch.release();
    return RELCP_OK;
}

int relcp_compact_flags_device(const int32_t *flags, int32_t n, int32_t *out, int32_t *count, void *stream) {
    if (n < 0 || (n > 0 && (!flags || !out)) || (const void *)flags == (const void *)out) return RELCP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    DBuf<int> scratch;
    try {
        compact_flags(flags, n, nullptr, out, count, scratch, s);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
    } catch (const Error &e) {
        scratch.release();
        return e.code;
    }
    scratch.release();
    return RELCP_OK;
}

}  // extern "C"
