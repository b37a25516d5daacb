// lcp.hip -- contact rows, per-body incidence (CSR) and the matrix-free
// projected-gradient LCP loop on A = dt D^T K D.
//
// Paper: Palmer, Aktulga, Gao (arXiv 2506.14097).  Rows: Eq. collision_ft
// and the rigid wrench form [-n, -(r_a x n), n, (r_b x n)] (proof of Thm.
// is_a_relcp).  LCP of one recursion: Eq. relcp (overdamped) and Eq.
// relcp_inertial; CQP form Eq. cqpp, solved by projected gradient (one of
// the solvers named after Eq. cqpp; the paper does not say which it used).
// Per-row constants of the pulled-back rows: Sec. 3.1 (iteration 1,
// "linearizing and pulling back new constraints").
//
// Iteration (Jacobi-scaled Barzilai-Borwein projected gradient):
//   gamma' = max(0, gamma - alpha g / A_aa)
//   g'     = qv + dt D^T (K D gamma')
//   s = gamma' - gamma, y = g' - g
//   even k: alpha = s^T D s / s^T y ; odd k: alpha = s^T y / y^T D^-1 y
//   (kept when s^T y <= 0, clamped to [1e-10, 1e10]), stop when
//   max_a |min(A_aa gamma_a, g_a)| <= tol.
// Each iteration is two passes: a per-body scatter D gamma' -> K -> vc (no
// atomics: each body walks its incidence list) and a per-row gather
// D^T vc -> g' with the step-size reductions.  The last block of the gather
// finishes the reductions in a fixed order, so the result does not depend
// on block scheduling.
#include <climits>
#include <type_traits>

#include "lcp.h"
#include "report.h"
#include "scatter.h"

namespace relcp {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / RELCP_WAVE;
// candidate-pair groups of kThreads up to which the iteration-0 rows are
// selected and built in one pass (each block sums the groups before it)
constexpr int kSelectGroupsMax = 4096;

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// rows
// ---------------------------------------------------------------------------
// Row m0 + k of pair pr.
__device__ inline void build_row(const RowBuildArgs &A, int k, int pr) {
    int a = A.pa[pr], b = A.pb[pr];
    int r = A.m0 + k;
    const int lp = A.ldp;
    double phi = A.snsd[pr];
    d3 n = mk(A.snsd[1 * lp + pr], A.snsd[2 * lp + pr], A.snsd[3 * lp + pr]);
    d3 ra = mk(A.snsd[4 * lp + pr], A.snsd[5 * lp + pr], A.snsd[6 * lp + pr]);
    d3 rb = mk(A.snsd[7 * lp + pr], A.snsd[8 * lp + pr], A.snsd[9 * lp + pr]);
    d3 ta = cross(ra, n), tb = cross(rb, n);
    const int lb = A.ldb;
    auto rate = [&](const double *V) {  // D_r^T V
        d3 va = mk(V[a], V[lb + a], V[2 * lb + a]), wa = mk(V[3 * lb + a], V[4 * lb + a], V[5 * lb + a]);
        d3 vb = mk(V[b], V[lb + b], V[2 * lb + b]), wb = mk(V[3 * lb + b], V[4 * lb + b], V[5 * lb + b]);
        return -dot(n, va) - dot(ta, wa) + dot(n, vb) + dot(tb, wb);
    };
    // qv = c + dt D^T U_free, with c = Phi at C^k for iteration-0 rows and
    // c = Phi(C_{n+1}) - dt D^T V_n for rows pulled back from a trial, so
    // that for those qv = Phi(C_{n+1}) - dt D^T (V_n - U_free).
    double qv = A.vc ? phi - A.dt * rate(A.vc) : (A.vfree ? phi + A.dt * rate(A.vfree) : phi);
    // A_rr = dt (n.kt_a n + ta.Kr_a ta + n.kt_b n + tb.Kr_b tb)
    auto quad = [&](int i, d3 t) {
        const double *K = A.K;
        double k0, k1, k2;
        sym3 R;
        if (A.kiso) {
            // the same values the nine components hold
            k0 = k1 = k2 = K[i];
            const double kr = K[3 * lb + i];
            R = sym3{kr, kr, kr, 0.0, 0.0, 0.0};
        } else {
            k0 = K[i];
            k1 = K[lb + i];
            k2 = K[2 * lb + i];
            R = sym3{K[3 * lb + i], K[4 * lb + i], K[5 * lb + i], K[6 * lb + i], K[7 * lb + i], K[8 * lb + i]};
        }
        double tr = n.x * n.x * k0 + n.y * n.y * k1 + n.z * n.z * k2;
        return tr + dot(t, mul(R, t));
    };
    double dA = A.dt * (quad(a, ta) + quad(b, tb));
    if (!(dA > 0.0)) dA = 1.0;
    double g0 = 0.0;
    if (A.prev_lam && A.prev_direct) {
        g0 = A.prev_lam[pr];
    } else if (A.prev_lam && A.nprev > 0) {
        int lo = 0, hi = A.nprev - 1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            int pa_ = A.prev_a[mid], pb_ = A.prev_b[mid];
            if (pa_ == a && pb_ == b) {
                g0 = A.prev_lam[mid];
                break;
            }
            if (pa_ < a || (pa_ == a && pb_ < b))
                lo = mid + 1;
            else
                hi = mid - 1;
        }
    }
    const int L = A.ldr;
    A.ia[r] = a;
    A.ib[r] = b;
    A.pair[r] = pr;
    A.rec_out[r] = A.rec;
    double nn[3] = {n.x, n.y, n.z}, tt[3] = {ta.x, ta.y, ta.z}, uu[3] = {tb.x, tb.y, tb.z};
    for (int c = 0; c < 3; ++c) {
        A.n64[c * L + r] = nn[c];
        A.ta64[c * L + r] = tt[c];
        A.tb64[c * L + r] = uu[c];
    }
    if (A.n32) {
        for (int c = 0; c < 3; ++c) {
            A.n32[c * L + r] = (float)nn[c];
            A.ta32[c * L + r] = (float)tt[c];
            A.tb32[c * L + r] = (float)uu[c];
        }
    }
    A.qv64[r] = qv;
    A.qv32[r] = (float)qv;
    A.dA64[r] = dA;
    A.dA32[r] = (float)dA;
    A.gam64[r] = g0;
    if (A.gam32) A.gam32[r] = (float)g0;
    A.phi64[r] = phi;
}

__global__ void k_rows_build(RowBuildArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nsel) return;
    build_row(A, k, A.sel[k]);
}

// The iteration-0 rows straight from the narrowphase's flags, without a
// separate compaction: one thread per candidate pair, one block per group of
// kThreads pairs (the groups whose set flags the narrowphase counted).  A
// pair's row is the number of set flags before it (the counts of the groups
// before the block, then a scan over the block), as the compaction numbers
// them; a selected pair builds its row there.  Also sel (row -> pair), pos
// (pair -> row, or -1) and, from the last block, the row count.
__global__ void __launch_bounds__(kThreads) k_select_rows(RowBuildArgs A, int np, const int *__restrict__ flags,
                                                          const int *__restrict__ gcount, int *__restrict__ sel,
                                                          int *__restrict__ pos, int *__restrict__ total,
                                                          int *__restrict__ total_dev) {
    __shared__ int sh[kWaves];
    __shared__ int goff;
    const int b = blockIdx.x;
    const int p = b * kThreads + threadIdx.x;
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    const int f = p < np && flags[p] ? 1 : 0;
    // set flags of the groups before this one (four loads per thread in
    // flight per round)
    int acc = 0;
    for (int g0 = threadIdx.x; g0 < b; g0 += 4 * kThreads) {
        int v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = g0 + u * kThreads < b ? gcount[g0 + u * kThreads] : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u];
    }
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, RELCP_WAVE);
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kWaves; ++k) t += sh[k];
        goff = t;
    }
    __syncthreads();
    // inclusive scan of the flags over the wave, then over the waves
    int inc = f;
    for (int o = 1; o < RELCP_WAVE; o <<= 1) {
        const int t = __shfl_up(inc, o, RELCP_WAVE);
        if (lane >= o) inc += t;
    }
    if (lane == RELCP_WAVE - 1) sh[w] = inc;
    __syncthreads();
    int woff = 0, btot = 0;
    for (int k = 0; k < kWaves; ++k) {
        woff += k < w ? sh[k] : 0;
        btot += sh[k];
    }
    const int k = goff + woff + inc - f;
    if (b == (int)gridDim.x - 1 && threadIdx.x == 0) {
        if (total_dev) *total_dev = goff + btot;
        *total = goff + btot;
    }
    if (p >= np) return;
    pos[p] = f ? k : -1;
    if (!f) return;
    sel[k] = p;
    build_row(A, k, p);
}


// ---------------------------------------------------------------------------
// incidence lists (CSR by body)
// ---------------------------------------------------------------------------
// Runs of equal keys over consecutive lanes of a wave (the rows of a
// step's first set are sorted by their first body): the lane's run head,
// and the run's length (valid at the head).  Inactive lanes (key -1) form
// runs of their own.
__device__ inline void key_runs(int key, int &head, int &len) {
    const int lane = threadIdx.x & (RELCP_WAVE - 1);
    const int prev = __shfl_up(key, 1, RELCP_WAVE);
    const unsigned long long heads = __ballot(lane == 0 || prev != key);
    head = RELCP_WAVE - 1 - __clzll(heads & ((2ull << lane) - 1ull));
    const unsigned long long above = lane == RELCP_WAVE - 1 ? 0ull : heads & (~0ull << (lane + 1));
    len = (above ? __ffsll((long long)above) - 1 : RELCP_WAVE) - lane;
}

__global__ void k_csr_count(int m, const int *__restrict__ ia, const int *__restrict__ ib, int *__restrict__ cnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = r < m ? ia[r] : -1;
    int head, len;
    key_runs(a, head, len);
    if (r >= m) return;
    // one atomic per run of rows sharing their first body
    if ((threadIdx.x & (RELCP_WAVE - 1)) == head) atomicAdd(cnt + a, len);
    atomicAdd(cnt + ib[r], 1);
}

// Incidence entries of each row at its two bodies.  With rcnt set (the
// row-graph layout), also each row's count of other rows at its two bodies
// (its entries in the row graph) and their sum into *count.
__global__ void __launch_bounds__(256) k_csr_fill(int m, const int *__restrict__ ia, const int *__restrict__ ib,
                                                  const int *__restrict__ off, int *__restrict__ cursor,
                                                  int *__restrict__ ent, int *__restrict__ count,
                                                  int *__restrict__ rcnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    int w = 0;
    const int a = r < m ? ia[r] : -1;
    int head, len;
    key_runs(a, head, len);
    // a run of rows sharing their first body takes consecutive slots there
    // with one atomic (the sort pass orders each body's list afterwards)
    const int lane = threadIdx.x & (RELCP_WAVE - 1);
    int slot = 0;
    if (r < m && lane == head) slot = atomicAdd(cursor + a, len);
    slot = __shfl(slot, head, RELCP_WAVE) + (lane - head);
    if (r < m) {
        const int b = ib[r];
        ent[off[a] + slot] = r << 1;
        ent[off[b] + atomicAdd(cursor + b, 1)] = (r << 1) | 1;
        w = off[a + 1] - off[a] + off[b + 1] - off[b] - 2;  // the row itself at a and at b: the diagonal
        if (rcnt) rcnt[r] = w;
    }
    if (!rcnt) return;
    __shared__ int bsum[4];
    int sum = w;
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, RELCP_WAVE);
    const int wv = threadIdx.x / RELCP_WAVE;
    if (lane == 0) bsum[wv] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = bsum[0] + bsum[1] + bsum[2] + bsum[3];
        if (t) atomicAdd(count, t);
    }
}

// Order each body's list by entry (row index) so summation order is fixed,
// and clear the body's count and cursor for the next build.  Lists of up to
// kSortRegs entries (nearly all) are sorted in registers by odd-even
// transposition, all their loads in flight together; longer ones in place.
// Entries are distinct, so either way gives the one sorted order.
constexpr int kSortRegs = 8;
__global__ void k_csr_sort(int nb, const int *__restrict__ off, int *__restrict__ ent, int *__restrict__ cnt,
                           int *__restrict__ cursor) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    cnt[i] = 0;
    cursor[i] = 0;
    int lo = off[i], hi = off[i + 1];
    if (hi - lo <= kSortRegs) {
        int v[kSortRegs];
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k) v[k] = lo + k < hi ? ent[lo + k] : INT_MAX;
#pragma unroll
        for (int rd = 0; rd < kSortRegs; ++rd)
#pragma unroll
            for (int k = rd & 1; k + 1 < kSortRegs; k += 2) {
                const int a = min(v[k], v[k + 1]), b = max(v[k], v[k + 1]);
                v[k] = a;
                v[k + 1] = b;
            }
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k)
            if (lo + k < hi) ent[lo + k] = v[k];
        return;
    }
    for (int k = lo + 1; k < hi; ++k) {
        int v = ent[k], j = k - 1;
        while (j >= lo && ent[j] > v) {
            ent[j + 1] = ent[j];
            --j;
        }
        ent[j + 1] = v;
    }
}

// ---------------------------------------------------------------------------
// the two passes of one iteration
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RELCP_WAVE);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, RELCP_WAVE));
    return v;
}
// Wave totals through DPP row operations (VALU lane moves, no LDS
// crossbar): quad permutes, row shifts by 4 and 8, then the broadcasts of
// lanes 15 and 31 into the following rows; the total ends in lane 63 and is
// read from there.  Lanes whose source is out of range read 0, the identity
// of the sums and of the max of non-negative values.  A fixed order.
template <int CTRL, int ROWS = 0xf>
__device__ inline double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double lane63(double v) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}
// three sums and the max of non-negative values over the wave (every lane
// gets the results)
__device__ inline void wave_reduce4(double &a, double &b, double &c, double &mx) {
#define RELCP_DPP_STEP(CTRL, ROWS)                \
    a += dpp_move<CTRL, ROWS>(a);                 \
    b += dpp_move<CTRL, ROWS>(b);                 \
    c += dpp_move<CTRL, ROWS>(c);                 \
    mx = fmax(mx, dpp_move<CTRL, ROWS>(mx));
    RELCP_DPP_STEP(0xb1, 0xf)   // quad_perm 1,0,3,2
    RELCP_DPP_STEP(0x4e, 0xf)   // quad_perm 2,3,0,1
    RELCP_DPP_STEP(0x114, 0xf)  // row_shr 4
    RELCP_DPP_STEP(0x118, 0xf)  // row_shr 8
    RELCP_DPP_STEP(0x142, 0xa)  // row_bcast 15 into rows 1 and 3
    RELCP_DPP_STEP(0x143, 0xc)  // row_bcast 31 into rows 2 and 3
#undef RELCP_DPP_STEP
    a = lane63(a);
    b = lane63(b);
    c = lane63(c);
    mx = lane63(mx);
}

// Block reduction of 3 sums and 1 max in a fixed order over NW waves; the
// result is valid in thread 0.
template <int NW>
__device__ inline void block_reduce4n(double &a, double &b, double &c, double &mx, double (*sh)[NW]) {
    wave_reduce4(a, b, c, mx);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    if (lane == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
        sh[3][w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0.0;
        mx = 0.0;
        for (int k = 0; k < NW; ++k) {
            a += sh[0][k];
            b += sh[1][k];
            c += sh[2][k];
            mx = fmax(mx, sh[3][k]);
        }
    }
    __syncthreads();
}

// TRAIL: a barrier after thread 0's reads of sh, before sh is written
// again; left out where a later barrier comes first or sh is not used again.
template <bool TRAIL = true>
__device__ inline void block_reduce4(double &a, double &b, double &c, double &mx, double (*sh)[kWaves]) {
    wave_reduce4(a, b, c, mx);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    if (lane == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
        sh[3][w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0.0;
        mx = 0.0;
        for (int k = 0; k < kWaves; ++k) {
            a += sh[0][k];
            b += sh[1][k];
            c += sh[2][k];
            mx = fmax(mx, sh[3][k]);
        }
    }
    if (TRAIL) __syncthreads();
}

// State after one gather: iteration count, residual, convergence and the
// Barzilai-Borwein step (BB1 after even iterations, BB2 after odd ones).
// An FP32 solve (stall > 0) whose residual has not halved for `stall`
// iterations stops as stalled: its rounding floor is above the tolerance,
// and the FP64 polish that follows it continues from its last iterate.
__device__ inline PgdState pgd_next(const PgdState &s, double ss, double sy, double yy, double res, double tol,
                                    int stall = 0) {
    PgdState n = s;
    const int k = s.iter;
    n.iter = k + 1;
    n.res = res;
    n.ss = ss;
    n.sy = sy;
    n.yy = yy;
    n.conv = (res <= tol) ? 1 : 0;
    if (!(res >= 0.5 * s.best)) {
        n.best = res;
        n.best_iter = n.iter;
    }
    if (stall > 0 && !n.conv && n.iter - n.best_iter >= stall) n.conv = 2;
    if (sy > 0.0) {
        double a = (k % 2 == 0) ? ss / sy : sy / yy;
        n.alpha = a < 1e-10 ? 1e-10 : (a > 1e10 ? 1e10 : a);
    }
    return n;
}

// Reduce the gather partials (same fixed order in every block) and advance
// the state; thread 0 of every block ends with the new state in `out`.
__device__ inline void reduce_partials(const PgdCtl &C, int par, PgdState *out, double (*sh)[kWaves]) {
    double ss = 0.0, sy = 0.0, yy = 0.0, res = 0.0;
    // thread t adds partials t, t + kThreads, ... in that order; the loads of
    // kU of them are issued before their adds
    constexpr int kU = 8;
    for (int k0 = threadIdx.x; k0 < C.nbg; k0 += kU * kThreads) {
        double4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int k = k0 + u * kThreads;
            v[u] = k < C.nbg ? *reinterpret_cast<const double4 *>(C.partials + 4 * k) : double4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (k0 + u * kThreads < C.nbg) {
                ss += v[u].x;
                sy += v[u].y;
                yy += v[u].z;
                res = fmax(res, v[u].w);
            }
        }
    }
    block_reduce4<false>(ss, sy, yy, res, sh);
    if (threadIdx.x == 0) *out = pgd_next(C.S[par ^ 1], ss, sy, yy, res, C.tol, C.stall);
    __syncthreads();
}

// The previous pass's partial sums held in registers: loaded at the start
// of a pass (their latency overlaps the row's own loads) and reduced later
// in the order reduce_partials uses (thread t: partials t, t + kThreads,
// ...), so the state is the same bit for bit.  For passes over at most
// kPartRegs * kThreads blocks.
constexpr int kPartRegs = 4;
struct PartialRegs {
    double4 v[kPartRegs];
};
__device__ inline void load_partials(const PgdCtl &C, PartialRegs &pr) {
    // every lane loads (a lane past the last block re-reads that block's
    // sums, which reduce_loaded skips): no branch, so no wait before the
    // row's own loads go out
    const int last = C.nbg > 0 ? C.nbg - 1 : 0;
#pragma unroll
    for (int u = 0; u < kPartRegs; ++u) {
        const int k = min((int)threadIdx.x + u * kThreads, last);
        pr.v[u] = *reinterpret_cast<const double4 *>(C.partials + 4 * k);
    }
}
// this thread's share of the loaded partial sums, in reduce_partials' order
__device__ inline void loaded_sums(const PgdCtl &C, const PartialRegs &pr, double &ss, double &sy, double &yy,
                                   double &res) {
    ss = sy = yy = res = 0.0;
#pragma unroll
    for (int u = 0; u < kPartRegs; ++u) {
        if ((int)threadIdx.x + u * kThreads < C.nbg) {
            ss += pr.v[u].x;
            sy += pr.v[u].y;
            yy += pr.v[u].z;
            res = fmax(res, pr.v[u].w);
        }
    }
}
__device__ inline void reduce_loaded(const PgdCtl &C, int par, const PartialRegs &pr, PgdState *out,
                                     double (*sh)[kWaves]) {
    double ss, sy, yy, res;
    loaded_sums(C, pr, ss, sy, yy, res);
    block_reduce4<false>(ss, sy, yy, res, sh);
    if (threadIdx.x == 0) *out = pgd_next(C.S[par ^ 1], ss, sy, yy, res, C.tol, C.stall);
    __syncthreads();
}

// the control block of a new solve (states before iteration 0, not done)
__device__ inline void pgd_reset(const PgdCtl &C) {
    PgdState s{};
    s.alpha = 1.0;
    s.iter = -1;
    s.best = __builtin_huge_val();
    s.best_iter = -1;
    C.S[0] = s;
    C.S[1] = s;
    *C.fin = s;
    *C.done = 0;
    if (C.fin_h) *C.fin_h = s;
    if (C.done_h) *C.done_h = 0;
}

__global__ void k_pgd_init(PgdCtl C) {
    if (threadIdx.x == 0 && blockIdx.x == 0) pgd_reset(C);
}

// Row c: gamma' (MODE 0: max(0, gamma); MODE 1: projected step), then
// g' = qv + dt D_c^T V, the step-size sums and the scaled natural residual.
template <typename T, int MODE, class VS>
__device__ inline void gather_row(const RowsT<T> &R, int c, T al, T dtT, const VS &V, double &ss, double &sy,
                                  double &yy, double &res) {
    const int L = R.ld;
    T gm = R.gam[c], gold = R.g[c], dA = R.dA[c];
    T gv = MODE == 1 ? project(gm, gold, dA, al) : clamp0(gm);
    int a = R.ia[c], b = R.ib[c];
    T nx = R.n[c], ny = R.n[L + c], nz = R.n[2 * L + c];
    T rate = -(nx * V(0, a) + ny * V(1, a) + nz * V(2, a)) -
             (R.ta[c] * V(3, a) + R.ta[L + c] * V(4, a) + R.ta[2 * L + c] * V(5, a)) +
             (nx * V(0, b) + ny * V(1, b) + nz * V(2, b)) +
             (R.tb[c] * V(3, b) + R.tb[L + c] * V(4, b) + R.tb[2 * L + c] * V(5, b));
    T gn = R.qv[c] + dtT * rate;
    T dg = dA * gv;
    res = fmax(res, fabs((double)(dg < gn ? dg : gn)));
    if (MODE == 1) {
        double s = (double)gv - (double)gm, y = (double)gn - (double)gold;
        ss += (double)dA * s * s;
        sy += s * y;
        yy += y * y / (double)dA;
    }
    R.gam[c] = gv;
    R.g[c] = gn;
}

// Grid mode, MODE 0: V = K D max(0, gamma) (start of a solve).
// MODE 1: reduce the previous gather, advance the state (S[par^1] ->
// S[par]); stop if converged; else V = K D gamma' with gamma' the projected
// step.  The projection is recomputed per incident row, bit-identical to
// the gather's.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_scatter(RowsT<T> R, BodiesT<T> B, PgdCtl C, int par) {
    __shared__ double sh[4][kWaves];
    __shared__ PgdState ns;
    T al = T(0);
    if (MODE == 1) {
        if (*C.done) return;
        reduce_partials(C, par, &ns, sh);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            C.S[par] = ns;
            if (ns.conv) {
                *C.fin = ns;
                *C.done = 1;
                if (C.fin_h) *C.fin_h = ns;
                if (C.done_h) *C.done_h = 1;
            }
        }
        if (ns.conv) return;
        al = (T)ns.alpha;
    }
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B.nb) return;
    scatter_body<T, MODE>(R, B, i, al, VGlobal<T>{B.vc, B.ld});
}

// Grid mode, MODE 0: g = qv + dt D^T V at max(0, gamma); MODE 1: the same at
// the projected step, plus the step-size sums.  Each block writes its
// partial sums (s^T D s, s^T y, y^T D^-1 y, max residual) for the next
// scatter.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_gather(RowsT<T> R, BodiesT<T> B, double dt, PgdCtl C, int par) {
    if (MODE == 1 && *C.done) return;
    __shared__ double sh[4][kWaves];
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    double ss = 0.0, sy = 0.0, yy = 0.0, res = 0.0;
    if (c < R.m) {
        const T al = MODE == 1 ? (T)C.S[par].alpha : T(0);
        gather_row<T, MODE>(R, c, al, (T)dt, VGlobal<T>{B.vc, B.ld}, ss, sy, yy, res);
    }
    block_reduce4(ss, sy, yy, res, sh);
    if (threadIdx.x == 0) {
        double *p = C.partials + 4 * blockIdx.x;
        p[0] = ss;
        p[1] = sy;
        p[2] = yy;
        p[3] = res;
    }
}

// Resident mode: one workgroup owns one packing (bodies [boff[p],
// boff[p+1]), rows rlist[roff[p] .. roff[p+1])) and runs its whole solve:
// the same two passes per iteration separated by workgroup barriers, with
// the packing's own step length and convergence.  With LDSV the packing's
// velocities live in LDS during the solve and are written back at the end.
template <typename T, int BS, bool LDSV>
__global__ void __launch_bounds__(BS) k_lcp_resident(RowsT<T> R, BodiesT<T> B, const int *__restrict__ boff,
                                                     const int *__restrict__ roff, const int *__restrict__ rlist,
                                                     double dt, double tol, int cap, PgdState *__restrict__ out,
                                                     int lds_ld, int stall) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double sh[4][BS / RELCP_WAVE];
    __shared__ PgdState st;
    const int p = blockIdx.x;
    const int b0 = boff[p], b1 = boff[p + 1], r0 = roff[p], r1 = roff[p + 1];
    const T dtT = (T)dt;
    auto run = [&](const auto &V) {
        for (int i = b0 + threadIdx.x; i < b1; i += BS) scatter_body<T, 0>(R, B, i, T(0), V);
        __syncthreads();
        double ss = 0.0, sy = 0.0, yy = 0.0, res = 0.0;
        for (int k = r0 + threadIdx.x; k < r1; k += BS) gather_row<T, 0>(R, rlist[k], T(0), dtT, V, ss, sy, yy, res);
        block_reduce4n<BS / RELCP_WAVE>(ss, sy, yy, res, sh);
        if (threadIdx.x == 0) {
            PgdState s0{};
            s0.alpha = 1.0;
            s0.iter = -1;
            s0.best = __builtin_huge_val();
            s0.best_iter = -1;
            st = pgd_next(s0, ss, sy, yy, res, tol);
        }
        __syncthreads();
        while (!st.conv && st.iter < cap) {
            const T al = (T)st.alpha;
            for (int i = b0 + threadIdx.x; i < b1; i += BS) scatter_body<T, 1>(R, B, i, al, V);
            __syncthreads();
            ss = sy = yy = res = 0.0;
            for (int k = r0 + threadIdx.x; k < r1; k += BS)
                gather_row<T, 1>(R, rlist[k], al, dtT, V, ss, sy, yy, res);
            block_reduce4n<BS / RELCP_WAVE>(ss, sy, yy, res, sh);
            if (threadIdx.x == 0) st = pgd_next(st, ss, sy, yy, res, tol, stall);
            __syncthreads();
        }
    };
    if (LDSV) {
        VLocal<T> V{reinterpret_cast<T *>(smem_raw), lds_ld, b0};
        run(V);
        for (int i = b0 + threadIdx.x; i < b1; i += BS)
            for (int k = 0; k < 6; ++k) B.vc[k * B.ld + i] = V(k, i);
    } else {
        run(VGlobal<T>{B.vc, B.ld});
    }
    if (threadIdx.x == 0) out[p] = st;
}

// rows grouped by packing: count the rows of each packing in [m0, m1)
// Rows per packing.  Rows arrive grouped by packing, so the lanes of a wave
// mostly share one counter: each round, the lanes holding the packing of the
// lowest pending lane add their count in one atomic (usually one or two
// rounds per wave instead of 64 contended atomics).
__global__ void k_rows_per_packing(int m0, int m1, const int *__restrict__ ia, const int *__restrict__ body_batch,
                                   int *__restrict__ cnt) {
    const int r = m0 + blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (RELCP_WAVE - 1);
    const int p = r < m1 ? body_batch[ia[r]] : -1;
    unsigned long long pending = __ballot(p >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int key = __shfl(p, leader, RELCP_WAVE);
        const unsigned long long same = __ballot(p == key) & pending;
        if (lane == leader) atomicAdd(cnt + key, __popcll(same));
        pending &= ~same;
    }
}

// New row list after appending rows [m_old, m_old + nv) (themselves grouped
// by packing): old position t of packing p moves to t + E[p]; the k-th new
// row goes to roff_old[p + 1] + k, where E = exclusive scan of the new
// rows' per-packing counts.
__global__ void k_rlist_merge(int m_old, int nv, const int *__restrict__ rlist_old, const int *__restrict__ ia,
                              const int *__restrict__ body_batch, const int *__restrict__ roff_old,
                              const int *__restrict__ E, int *__restrict__ rlist_new) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m_old) {
        int r = rlist_old[t];
        rlist_new[t + E[body_batch[ia[r]]]] = r;
    } else if (t < m_old + nv) {
        int k = t - m_old;
        int r = m_old + k;
        rlist_new[roff_old[body_batch[ia[r]] + 1] + k] = r;
    }
}

__global__ void k_add_arrays(int n, const int *__restrict__ a, const int *__restrict__ b, int *__restrict__ c) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = a[i] + b[i];
}

__global__ void k_iota(int n, int *__restrict__ v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

// Advance the state from the last gather without another scatter (end of a
// solve that hit its iteration cap, or a fixed-iteration run).
__global__ void __launch_bounds__(kThreads) k_pgd_finalize(PgdCtl C, int par) {
    __shared__ double sh[4][kWaves];
    __shared__ PgdState ns;
    if (*C.done) return;
    reduce_partials(C, par, &ns, sh);
    if (threadIdx.x == 0) {
        C.S[par] = ns;
        *C.fin = ns;
        if (C.fin_h) *C.fin_h = ns;
        if (ns.conv) {
            *C.done = 1;
            if (C.done_h) *C.done_h = 1;
        }
    }
}

// The reduction of the last pass's partial sums into the new state, in one
// block and in the order every block of an iteration pass uses (so the
// iterates are the same either way), for passes over many blocks: there,
// every block re-reading all partial sums would cost reads quadratic in the
// block count.  Stops the solve (done) on convergence.
__global__ void __launch_bounds__(kThreads) k_pgd_reduce(PgdCtl C, int par) {
    __shared__ double sh[4][kWaves];
    __shared__ PgdState ns;
    if (*C.done) return;
    reduce_partials(C, par, &ns, sh);
    if (threadIdx.x == 0) {
        C.S[par] = ns;
        if (ns.conv) {
            *C.fin = ns;
            *C.done = 1;
            if (C.fin_h) *C.fin_h = ns;
            if (C.done_h) *C.done_h = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// row-graph LCP: A = dt D^T K D assembled over rows, one pass per iteration
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_rowgraph_counts(int m, const int *__restrict__ ia,
                                                              const int *__restrict__ ib, const int *__restrict__ off,
                                                              int *__restrict__ count, int *__restrict__ rcnt) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    int w = 0;
    if (r < m) {
        const int a = ia[r], b = ib[r];
        w = off[a + 1] - off[a] + off[b + 1] - off[b] - 2;  // the row itself at a and at b: the diagonal
        rcnt[r] = w;
    }
    if (!count) return;
    __shared__ int bsum[kWaves];
    int sum = w;
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, RELCP_WAVE);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), wv = threadIdx.x / RELCP_WAVE;
    if (lane == 0) bsum[wv] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kWaves; ++k) t += bsum[k];
        if (t) atomicAdd(count, t);
    }
}

// Entries of the row graph, one thread per incidence entry in CSR order
// (entry e of body c: row r, side): the thread forms its own column of D at
// c, s (n_r, tau_r), shares it and its entry through LDS with the other
// entries of c in its block, and writes row r's entries at c: for every other entry j of c,
// in incidence order, column r_j and value dt J_j . K_c J_e (so row r holds
// its entries at body a, then those at body b).  The slots past a row's
// entries are not written: the passes read a row's entries only (its count
// from the count pass).  A row with more entries than the stride is left
// out (its count raises *need, and the overflow is reported).  A column of
// an entry outside the block (a body that straddles two blocks) is formed
// again from the rows.  The diagonal A_rr is not stored: a pass takes it
// from the rows' A_aa.
__device__ inline void column_of(const RowGraphFill &A, int en, double J[6]) {
    const int L = A.ldr, j = en >> 1;
    const double s = (en & 1) ? 1.0 : -1.0;
    const double *t = (en & 1) ? A.tb : A.ta;
    J[0] = s * A.n[j];
    J[1] = s * A.n[L + j];
    J[2] = s * A.n[2 * L + j];
    J[3] = s * t[j];
    J[4] = s * t[L + j];
    J[5] = s * t[2 * L + j];
}

__global__ void __launch_bounds__(kThreads) k_rowgraph_fill_entries(RowGraphFill A) {
    __shared__ double shJ[6][kThreads];
    __shared__ int shE[kThreads];
    __shared__ int shs[kWaves];
    const int E0 = blockIdx.x * kThreads;
    const int e = E0 + threadIdx.x;
    // a slot past a list's length holds -1 (lists with lengths)
    const int en = e < A.nslots ? A.ent[e] : -1;
    const bool act = en >= 0;
    int r = 0, side = 0, c = 0, other = 0;
    double J[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        r = en >> 1;
        side = en & 1;
        const int a = A.ia[r], b = A.ib[r];
        c = side ? b : a;
        other = side ? a : b;
        column_of(A, en, J);
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) shJ[t][threadIdx.x] = J[t];
    shE[threadIdx.x] = en;
    if (A.lcnt && blockIdx.x == 0) {
        // the entry count: the list filter's block sums, added up here
        int acc = 0;
        for (int k = threadIdx.x; k < A.nbsums; k += kThreads) acc += A.bsums[k];
        for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, RELCP_WAVE);
        if ((threadIdx.x & (RELCP_WAVE - 1)) == 0) shs[threadIdx.x / RELCP_WAVE] = acc;
    }
    __syncthreads();
    if (A.lcnt && blockIdx.x == 0 && threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kWaves; ++k) t += shs[k];
        A.report[1] = t;
    }
    if (!act) return;
    const int lane = r & (RELCP_WAVE - 1), sl = r / RELCP_WAVE;
    const int S = A.stride;
    const size_t b0 = (size_t)sl * S;
    if (!A.lcnt && r == 0 && side == 0) {
        // the count pass is complete: report and clear its counter
        A.report[1] = *A.count;
        *A.count = 0;
    }
    const int j0 = A.off[c], j1 = A.lcnt ? j0 + A.lcnt[c] : A.off[c + 1];
    // the row's entries: its other rows at c and at the other body (formed
    // here from the lists' lengths, and stored once, by the side-b entry)
    int cnt;
    if (A.lcnt) {
        cnt = (j1 - j0 - 1) + (A.lcnt[other] - 1);
        if (side) A.rcnt[r] = cnt;
    } else {
        cnt = A.rcnt[r];
    }
    // a row that does not fit is left out by both of its entries' threads
    // side b: after the slots of body a's other rows (the row's count less
    // those at b)
    int k = side ? cnt - (j1 - j0 - 1) : 0;
    if (cnt > S || (size_t)RELCP_WAVE * (b0 + S) > A.cap) {
        atomicMax(A.need, cnt);
        A.report[2] = 1;
        return;
    }
    int *__restrict__ col = A.col;
    double *__restrict__ v64 = A.val64;
    float *__restrict__ v32 = A.val32;
    const int lb = A.ldb;
    const double sr = side ? 1.0 : -1.0;
    // K_c applied to this row's column (sign included)
    const double *K = A.K;
    const d3 nr = mk(sr * J[0], sr * J[1], sr * J[2]);
    const d3 ur = mk(sr * J[3], sr * J[4], sr * J[5]);
    double k0, k1, k2;
    sym3 Kr;
    if (A.kiso) {
        // the same values the nine components hold
        k0 = k1 = k2 = K[c];
        const double kr = K[3 * lb + c];
        Kr = sym3{kr, kr, kr, 0.0, 0.0, 0.0};
    } else {
        k0 = K[c];
        k1 = K[lb + c];
        k2 = K[2 * lb + c];
        Kr = sym3{K[3 * lb + c], K[4 * lb + c], K[5 * lb + c], K[6 * lb + c], K[7 * lb + c], K[8 * lb + c]};
    }
    const d3 Kn = mk(sr * k0 * nr.x, sr * k1 * nr.y, sr * k2 * nr.z);
    const d3 Ku = sr * mul(Kr, ur);
    for (int j = j0; j < j1; ++j) {
        if (j == e) continue;
        double Jj[6];
        int cj;
        if (j >= E0 && j < E0 + kThreads) {
#pragma unroll
            for (int t = 0; t < 6; ++t) Jj[t] = shJ[t][j - E0];
            cj = shE[j - E0] >> 1;
        } else {
            const int ej = A.ent[j];
            column_of(A, ej, Jj);
            cj = ej >> 1;
        }
        const double v =
            A.dt * (Jj[0] * Kn.x + Jj[1] * Kn.y + Jj[2] * Kn.z + Jj[3] * Ku.x + Jj[4] * Ku.y + Jj[5] * Ku.z);
        const size_t at = (size_t)RELCP_WAVE * (b0 + (size_t)k) + lane;
        col[at] = cj;
        v64[at] = v;
        v32[at] = (float)v;
        ++k;
    }
}

// max(0, gamma - alpha h); the same rounding wherever a row's step is formed
__device__ inline double step_h(double gm, double h, double al) {
    const double v = __dsub_rn(gm, __dmul_rn(al, h));
    return v > 0.0 ? v : 0.0;
}
__device__ inline float step_h(float gm, float h, float al) {
    const float v = __fsub_rn(gm, __fmul_rn(al, h));
    return v > 0.0f ? v : 0.0f;
}

// One row of a row-graph pass, split so that everything that does not
// depend on the step length (the row's own state, up to KP matrix entries
// and the previous state of the rows they point at) is loaded before the
// reduction that yields the step length.
constexpr int kPre = 16;

// The start values of a solve as its start pass reads them (see StartSrc):
// an FP64 array, or the final state of an FP32 solve; a compile-time choice,
// so the start pass's loads carry no branch.
struct StartF64 {
    const double *g;
    __device__ double operator[](int j) const { return g[j]; }
    __device__ static StartF64 from(const StartSrc &S) { return StartF64{S.gam64}; }
};
struct StartF32 {
    const RowStep<float> *z;
    __device__ double operator[](int j) const { return (double)z[j].gam; }
    __device__ static StartF32 from(const StartSrc &S) {
        const bool odd = (S.done && !*S.done) ? (S.last_par & 1) : (S.fin->iter & 1);
        return StartF32{S.z[odd ? 1 : 0]};
    }
};

template <typename T>
struct RowPre {
    int cnt;  // this row's entries (<= the stride)
    const int *col;
    const T *val;
    T gm, hm, gold, dA, q;
    int cj[kPre];
    T vj[kPre], gj[kPre], hj[kPre];
};

// Stage A of a row's loads: the row's own state; nothing here waits on
// another load of the pass.
template <typename T, int MODE, class SV>
__device__ inline void row_preload_a(const RowGraphT<T> &G, const T *__restrict__ qv, const T *__restrict__ dA0,
                                     const SV &gam0, const RowStep<T> *__restrict__ zin,
                                     const T *__restrict__ gin, int r, RowPre<T> &P) {
    P.cnt = G.rcnt[r];
    P.dA = dA0[r];
    P.q = qv[r];
    if (MODE == 1) {
        const RowStep<T> z = zin[r];
        P.gm = z.gam;
        P.hm = z.h;
        P.gold = gin[r];
    } else {
        P.gm = (T)gam0[r];
        P.hm = T(0);
        P.gold = T(0);
    }
}

// Stage B: the first kPre entries of the row and the states of the rows
// they point at (two dependent loads).  The slice's slots are at a fixed
// offset (the stride is a launch argument, the same in every lane).
template <typename T, int MODE, class SV>
__device__ inline void row_preload_b(const RowGraphT<T> &G, const SV &gam0, const RowStep<T> *__restrict__ zin, int r,
                                     RowPre<T> &P) {
    const int lane = r & (RELCP_WAVE - 1);
    const int S = G.stride;
    const size_t b0 = (size_t)(r / RELCP_WAVE) * S;
    // a row that did not fit, or a slice past the allocation: no entries
    // (the caller sees the overflow report, re-sizes and starts over)
    if (P.cnt > S || (size_t)RELCP_WAVE * (b0 + S) > G.cap) P.cnt = 0;
    P.col = G.col + (size_t)RELCP_WAVE * b0 + lane;
    P.val = G.val + (size_t)RELCP_WAVE * b0 + lane;
    // slots past the row's entries are not read (zero value, zero neighbour
    // state); past the stride no lane has any (a uniform branch)
    const int kp = S < kPre ? S : kPre;
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        if (k < kp && k < P.cnt) {
            P.cj[k] = P.col[RELCP_WAVE * k];
            P.vj[k] = P.val[RELCP_WAVE * k];
        } else {
            P.cj[k] = r;
            P.vj[k] = T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        if (k < kp && k < P.cnt) {
            if (MODE == 1) {
                const RowStep<T> z = zin[P.cj[k]];
                P.gj[k] = z.gam;
                P.hj[k] = z.h;
            } else {
                P.gj[k] = (T)gam0[P.cj[k]];
                P.hj[k] = T(0);
            }
        } else {
            P.gj[k] = T(0);
            P.hj[k] = T(0);
        }
    }
}

template <typename T, int MODE, class SV>
__device__ inline void row_preload(const RowGraphT<T> &G, const T *__restrict__ qv, const T *__restrict__ dA0,
                                   const SV &gam0, const RowStep<T> *__restrict__ zin,
                                   const T *__restrict__ gin, int r, RowPre<T> &P) {
    row_preload_a<T, MODE, SV>(G, qv, dA0, gam0, zin, gin, r, P);
    row_preload_b<T, MODE, SV>(G, gam0, zin, r, P);
}

// projected steps, g' = qv + A gamma', the row's new state and its share
// of the step-size sums (s^T D s, s^T y, y^T D^-1 y) and residual
// (gv_out, gn_out: the new gamma and g also returned)
template <typename T, int MODE, class SV>
__device__ inline void row_finish(const RowPre<T> &P, T al, const RowStep<T> *__restrict__ zin,
                                  const SV &gam0, RowStep<T> *__restrict__ zout, T *__restrict__ gout,
                                  int r, double &ss, double &sy, double &yy, double &res, T *gv_out = nullptr,
                                  T *gn_out = nullptr) {
    // the diagonal first (A_rr, not stored in the graph), then the entries
    const T gv = MODE == 1 ? step_h(P.gm, P.hm, al) : clamp0(P.gm);
    T acc = P.dA * gv;
#pragma unroll
    for (int k = 0; k < kPre; ++k) acc += P.vj[k] * (MODE == 1 ? step_h(P.gj[k], P.hj[k], al) : clamp0(P.gj[k]));
    for (int k = kPre; k < P.cnt; ++k) {
        const int j = P.col[RELCP_WAVE * k];
        const T v = P.val[RELCP_WAVE * k];
        if (MODE == 1) {
            const RowStep<T> z = zin[j];
            acc += v * step_h(z.gam, z.h, al);
        } else {
            acc += v * clamp0((T)gam0[j]);
        }
    }
    const T gn = P.q + acc;
    zout[r] = RowStep<T>{gv, gn / P.dA};
    gout[r] = gn;
    if (gv_out) *gv_out = gv;
    if (gn_out) *gn_out = gn;
    const T dg = P.dA * gv;
    res = fmax(res, fabs((double)(dg < gn ? dg : gn)));
    if (MODE == 1) {
        const double sd = (double)gv - (double)P.gm, yd = (double)gn - (double)P.gold;
        ss += (double)P.dA * sd * sd;
        sy += sd * yd;
        yy += yd * yd / (double)P.dA;
    }
}

// One pass per launch (chunked mode): every block first reduces the
// previous pass's partial sums (fixed order) into the new state and step
// length, overlapped with the row's loads.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads)
    k_spmv(RowGraphT<T> G, const T *__restrict__ qv, const T *__restrict__ dA0, StartSrc start,
           const RowStep<T> *__restrict__ zin, const T *__restrict__ gin, RowStep<T> *__restrict__ zout,
           T *__restrict__ gout, PgdCtl C, double *__restrict__ pout, int par, double *__restrict__ save) {
    __shared__ double sh[4][kWaves];
    __shared__ PgdState ns;
    // MODE 3: a start from the final state of an FP32 solve (StartF32)
    constexpr bool START = MODE == 0 || MODE == 3;
    constexpr int RM = START ? 0 : 1;  // row arithmetic: start or iteration
    using SV = typename std::conditional<MODE == 3, StartF32, StartF64>::type;
    if (START && blockIdx.x == 0 && threadIdx.x == 0) pgd_reset(C);
    const int lb = xcd_block(blockIdx.x, gridDim.x);  // logical block: a contiguous row range per XCD
    const int r = lb * kThreads + threadIdx.x;
    const bool act = r < G.m;
    SV gam0{};
    if (START) gam0 = SV::from(start);
    // loads that depend on no other load of the pass go out first: the last
    // pass's partial sums, the row's own state and the done flag; a pass after convergence leaves once the flag is in
    // Lanes past the last row load the last row (their results are never
    // written), so the loads need no branch and nothing waits for them
    // before they are used.
    PartialRegs pr;
    if (MODE == 1) load_partials(C, pr);
    const int done = START ? 0 : __builtin_amdgcn_readfirstlane(*C.done);
    const int rl = act ? r : G.m - 1;
    RowPre<T> P;
    if (G.m > 0) row_preload_a<T, RM, SV>(G, qv, dA0, gam0, zin, gin, rl, P);
    if (done) return;
    if (G.m > 0) row_preload_b<T, RM, SV>(G, gam0, zin, rl, P);
    if (START && save && act) save[r] = gam0[r];  // the start, kept for a restart
    T al = T(0);
    if (MODE == 2) {
        // the state was advanced by k_pgd_reduce
        if (threadIdx.x == 0) ns = C.S[par];
        __syncthreads();
        al = (T)ns.alpha;
    }
    if (MODE == 1) {
        reduce_loaded(C, par, pr, &ns, sh);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            C.S[par] = ns;
            if (ns.conv) {
                *C.fin = ns;
                *C.done = 1;
                if (C.fin_h) *C.fin_h = ns;
                if (C.done_h) *C.done_h = 1;
            }
        }
        if (ns.conv) return;
        al = (T)ns.alpha;
    }
    double ss = 0.0, sy = 0.0, yy = 0.0, res = 0.0;
    T gv = T(0), gn = T(0);
    if (act) row_finish<T, RM, SV>(P, al, zin, gam0, zout, gout, r, ss, sy, yy, res, &gv, &gn);
    // (sh is used again only by the final start's work sums)
    block_reduce4<MODE == 3>(ss, sy, yy, res, sh);
    if (threadIdx.x == 0) {
        double *p = pout + 4 * lb;
        p[0] = ss;
        p[1] = sy;
        p[2] = yy;
        p[3] = res;
    }
    if (MODE == 3 && start.g_final) {
        // what the unpack of a solve that converges here would write: gamma,
        // g and the work's partial sums (the unpack's arithmetic, over the
        // same 256 rows per block)
        double w = 0.0, z0s = 0.0, z1s = 0.0, z2s = 0.0;
        if (act) {
            save[r] = (double)gv;
            start.g_final[r] = (double)gn;
            w = (double)gv * ((double)gn - (double)P.q);
        }
        block_reduce4<false>(w, z0s, z1s, z2s, sh);
        if (threadIdx.x == 0) start.work_final[lb] = w;
    }
}

// The tail report after checking a solve of which only the start pass ran
// (see launch_report_check).
__global__ void __launch_bounds__(kThreads) k_report_check(TailReport R, PgdCtl C) {
    __shared__ double sh[4][kWaves];
    // the report's loads, the partial sums' and the state before them go
    // out together; the two reductions share one barrier (the partial sums'
    // in the order reduce_loaded uses, so the state is the same bit for bit)
    TailRegs tr;
    tail_preload(R, tr);
    PartialRegs pr;
    load_partials(C, pr);
    const PgdState prev = C.S[0];
    double ss, sy, yy, res;
    loaded_sums(C, pr, ss, sy, yy, res);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    tail_report(
        R, tr,
        [&] {
            wave_reduce4(ss, sy, yy, res);
            if (lane == 0) {
                sh[0][w] = ss;
                sh[1][w] = sy;
                sh[2][w] = yy;
                sh[3][w] = res;
            }
        },
        [&] {
            double a = 0.0, b = 0.0, c = 0.0, mx = 0.0;
            for (int k = 0; k < kWaves; ++k) {
                a += sh[0][k];
                b += sh[1][k];
                c += sh[2][k];
                mx = fmax(mx, sh[3][k]);
            }
            const PgdState ns = pgd_next(prev, a, b, c, mx, C.tol, C.stall);
            C.S[1] = ns;
            if (ns.conv) {
                *C.fin = ns;
                *C.done = 1;
                if (C.fin_h) *C.fin_h = ns;
                if (C.done_h) *C.done_h = 1;
            }
        });
}

// A pass whose parameters live in device memory (LcpDev), so that the
// same launch can be recorded once in a graph and replayed for every solve.
// The grid covers a row capacity; blocks past the current row count leave
// at once.  A pass that finds the solve converged, or the iteration cap
// reached, records the final state and stops the later passes.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_spmv_dev(const LcpDev<T> *__restrict__ D, int par) {
    __shared__ double sh[4][kWaves];
    __shared__ PgdState ns;
    const LcpDev<T> &d = *D;
    if (*d.done) return;
    const int nbg = d.nbg;
    if ((int)blockIdx.x >= nbg) return;
    const RowGraphT<T> G{d.m, d.stride, d.col, d.val, d.slots, d.rcnt};
    const int lb = xcd_block(blockIdx.x, nbg);  // the same order as the per-pass launch over nbg blocks
    const int r = lb * kThreads + threadIdx.x;
    const bool act = r < d.m;
    RowPre<T> P;
    if (act) row_preload<T, 1, StartF64>(G, d.qv, d.dA, StartF64{nullptr}, d.z[par ^ 1], d.g[par ^ 1], r, P);
    PgdCtl C{d.S, d.fin, d.done, d.part[par ^ 1], nbg, d.tol, d.fin_h, d.done_h, d.stall};
    reduce_partials(C, par, &ns, sh);
    const bool stop = ns.conv || ns.iter >= d.cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.S[par] = ns;
        if (stop) {
            // done stops the passes; the host mirror done_h reports convergence
            // only (a capped solve is seen from fin_h->iter)
            *d.fin = ns;
            *d.done = 1;
            if (d.fin_h) *d.fin_h = ns;
            if (d.done_h && ns.conv) *d.done_h = 1;
        }
    }
    if (stop) return;
    double ss = 0.0, sy = 0.0, yy = 0.0, res = 0.0;
    if (act)
        row_finish<T, 1, StartF64>(P, (T)ns.alpha, d.z[par ^ 1], StartF64{nullptr}, d.z[par], d.g[par], r, ss, sy,
                                   yy, res);
    block_reduce4(ss, sy, yy, res, sh);
    if (threadIdx.x == 0) {
        double *p = d.part[par] + 4 * lb;
        p[0] = ss;
        p[1] = sy;
        p[2] = yy;
        p[3] = res;
    }
}

// the parameters of the next solve, copied in stream order
template <typename T>
__global__ void k_set_lcpdev(LcpDev<T> *D, LcpDev<T> v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *D = v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
    k_rowstate_unpack(int m, const RowStep<T> *__restrict__ z0, const RowStep<T> *__restrict__ z1,
                      const T *__restrict__ g0, const T *__restrict__ g1, const PgdState *__restrict__ fin,
                      const int *__restrict__ done, int last_par, T *__restrict__ gam, T *__restrict__ g,
                      double *__restrict__ gam64, const T *__restrict__ qv, double *__restrict__ work) {
    __shared__ double sh[4][kWaves];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double w = 0.0, z0s = 0.0, z1s = 0.0, z2s = 0.0;
    if (r < m) {
        // a finished solve: the state of its final iterate; else that of the last pass launched
        const bool odd = (done && !*done) ? (last_par & 1) : (fin->iter & 1);
        const T v = (odd ? z1 : z0)[r].gam;
        const T gv = (odd ? g1 : g0)[r];
        gam[r] = v;
        g[r] = gv;
        if (gam64) gam64[r] = (double)v;
        if (work) w = (double)v * ((double)gv - (double)qv[r]);
    }
    if (work) {
        // the work partials of this block, as k_work forms them
        block_reduce4<false>(w, z0s, z1s, z2s, sh);
        if (threadIdx.x == 0) work[blockIdx.x] = w;
    }
}

__global__ void k_promote(int m, const float *__restrict__ a, double *__restrict__ b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) b[i] = (double)a[i];
}
__global__ void k_demote(int m, const double *__restrict__ a, float *__restrict__ b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) b[i] = (float)a[i];
}

// per-block sums of gamma (g - qv) into partials[block] (summed in a fixed
// order by the caller's report)
__global__ void __launch_bounds__(kThreads) k_work(int m, const double *__restrict__ gam, const double *__restrict__ g,
                                                   const double *__restrict__ qv, double *__restrict__ partials) {
    __shared__ double sh[4][kWaves];
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    double w = 0.0, z0 = 0.0, z1 = 0.0, z2 = 0.0;
    if (c < m) w = gam[c] * (g[c] - qv[c]);
    block_reduce4<false>(w, z0, z1, z2, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = w;
}

__global__ void k_pair_lambda(int m, const int *__restrict__ rec, const int *__restrict__ pair,
                              const double *__restrict__ gam, int level, double *__restrict__ lam) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m && rec[r] == level) lam[pair[r]] += gam[r];
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int lcp_partials_needed(int m) { return 4 * (nblk(m > 0 ? m : 1, kThreads) + 1); }

void launch_rows_build(const RowBuildArgs &a, hipStream_t s) {
    if (a.nsel <= 0) return;
    hipLaunchKernelGGL(k_rows_build, dim3(nblk(a.nsel, 256)), dim3(256), 0, s, a);
}

int select_rows_max_pairs() { return kSelectGroupsMax * kThreads; }

void launch_select_rows(const RowBuildArgs &a, int np, const int *flags, const int *gcount, int *sel, int *pos,
                        int *total, hipStream_t s, int *total_dev) {
    if (np <= 0 || np > select_rows_max_pairs()) return;
    hipLaunchKernelGGL(k_select_rows, dim3(nblk(np, kThreads)), dim3(kThreads), 0, s, a, np, flags, gcount, sel, pos,
                       total, total_dev);
}


void launch_csr(int nb, int m, const int *ia, const int *ib, int *cnt, int *off, int *cursor, int *ent,
                bool cleared, DBuf<int> &scan_scratch, hipStream_t s, const CsrRowGraphOut *rg) {
    // cnt and cursor are adjacent (cursor = cnt + nb + 1): one clear, unless
    // the last build's sort pass left them at zero
    if (!cleared) HIP_OK(hipMemsetAsync(cnt, 0, sizeof(int) * 2 * (nb + 1), s));
    if (m > 0) hipLaunchKernelGGL(k_csr_count, dim3(nblk(m, 256)), dim3(256), 0, s, m, ia, ib, cnt);
    exclusive_scan(cnt, off, nb + 1, nullptr, scan_scratch, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_csr_fill, dim3(nblk(m, 256)), dim3(256), 0, s, m, ia, ib, off, cursor, ent,
                           rg ? rg->count : nullptr, rg ? rg->rcnt : nullptr);
        hipLaunchKernelGGL(k_csr_sort, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, off, ent, cnt, cursor);
    }
}

template <typename T>
void launch_lcp_scatter(int mode, const RowsT<T> &r, const BodiesT<T> &b, const PgdCtl &C, int par, hipStream_t s) {
    int nbk = nblk(b.nb > 0 ? b.nb : 1, kThreads);
    if (mode == 0)
        launch_k(k_scatter<T, 0>, dim3(nbk), dim3(kThreads), 0, s, r, b, C, par);
    else
        launch_k(k_scatter<T, 1>, dim3(nbk), dim3(kThreads), 0, s, r, b, C, par);
}

template <typename T>
void launch_lcp_gather(int mode, const RowsT<T> &r, const BodiesT<T> &b, double dt, const PgdCtl &C, int par,
                       hipStream_t s) {
    int nbk = nblk(r.m > 0 ? r.m : 1, kThreads);
    if (mode == 0)
        launch_k(k_gather<T, 0>, dim3(nbk), dim3(kThreads), 0, s, r, b, dt, C, par);
    else
        launch_k(k_gather<T, 1>, dim3(nbk), dim3(kThreads), 0, s, r, b, dt, C, par);
}

int lcp_gather_blocks(int m) { return nblk(m > 0 ? m : 1, kThreads); }

template <typename T, int BS, bool LDSV>
static int launch_res(const ResidentArgs<T> &a, hipStream_t s) {
    size_t lds = LDSV ? (size_t)6 * a.lds_ld * sizeof(T) : 0;
    auto fn = k_lcp_resident<T, BS, LDSV>;
    if (lds > 0) {
        if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return -1;
    }
    launch_k(fn, dim3(a.npk), dim3(BS), lds, s, a.R, a.B, a.boff, a.roff, a.rlist, a.dt, a.tol, a.cap, a.out,
             a.lds_ld, a.stall);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_lcp_resident(const ResidentArgs<T> &a, int block, bool lds, hipStream_t s) {
    if (a.npk <= 0) return 0;
    switch (block) {
        case 256: return lds ? launch_res<T, 256, true>(a, s) : launch_res<T, 256, false>(a, s);
        case 512: return lds ? launch_res<T, 512, true>(a, s) : launch_res<T, 512, false>(a, s);
        default: return lds ? launch_res<T, 1024, true>(a, s) : launch_res<T, 1024, false>(a, s);
    }
}
template int launch_lcp_resident<double>(const ResidentArgs<double> &, int, bool, hipStream_t);
template int launch_lcp_resident<float>(const ResidentArgs<float> &, int, bool, hipStream_t);

void launch_rows_per_packing(int m0, int m1, const int *ia, const int *body_batch, int *cnt, hipStream_t s) {
    if (m1 > m0) hipLaunchKernelGGL(k_rows_per_packing, dim3(nblk(m1 - m0, 256)), dim3(256), 0, s, m0, m1, ia,
                                    body_batch, cnt);
}
void launch_rlist_merge(int m_old, int nv, const int *rlist_old, const int *ia, const int *body_batch,
                        const int *roff_old, const int *E, int *rlist_new, hipStream_t s) {
    if (m_old + nv > 0)
        hipLaunchKernelGGL(k_rlist_merge, dim3(nblk(m_old + nv, 256)), dim3(256), 0, s, m_old, nv, rlist_old, ia,
                           body_batch, roff_old, E, rlist_new);
}
void launch_add_arrays(int n, const int *a, const int *b, int *c, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_add_arrays, dim3(nblk(n, 256)), dim3(256), 0, s, n, a, b, c);
}
void launch_iota(int n, int *v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_iota, dim3(nblk(n, 256)), dim3(256), 0, s, n, v);
}

void launch_pgd_init(const PgdCtl &C, hipStream_t s) {
    hipLaunchKernelGGL(k_pgd_init, dim3(1), dim3(64), 0, s, C);
}

void launch_pgd_finalize(const PgdCtl &C, int par, hipStream_t s) {
    hipLaunchKernelGGL(k_pgd_finalize, dim3(1), dim3(kThreads), 0, s, C, par);
}

int rowgraph_slices(int m) { return (m + RELCP_WAVE - 1) / RELCP_WAVE; }

void launch_rowgraph_counts(int m, const int *ia, const int *ib, const int *off, int *count, int *rcnt,
                            hipStream_t s) {
    launch_k(k_rowgraph_counts, dim3(nblk(m > 0 ? m : 1, kThreads)), dim3(kThreads), 0, s, m, ia, ib, off, count,
             rcnt);
}


void launch_rowgraph_fill(const RowGraphFill &a, hipStream_t s) {
    if (a.m > 0 && a.nslots > 0)
        launch_k(k_rowgraph_fill_entries, dim3(nblk(a.nslots, kThreads)), dim3(kThreads), 0, s, a);
}

template <typename T>
void launch_lcp_spmv(int mode, const RowGraphT<T> &G, const T *qv, const T *dA, const StartSrc &gam0,
                     const RowStep<T> *zin, const T *gin, RowStep<T> *zout, T *gout, const PgdCtl &C, double *pout,
                     int par, hipStream_t s, double *save) {
    const int nb = nblk(G.m > 0 ? G.m : 1, kThreads);
    if (mode == 0 && gam0.gam64) {
        launch_k(k_spmv<T, 0>, dim3(nb), dim3(kThreads), 0, s, G, qv, dA, gam0, zin, gin, zout, gout, C, pout, par,
                 save);
    } else if (mode == 0) {
        launch_k(k_spmv<T, 3>, dim3(nb), dim3(kThreads), 0, s, G, qv, dA, gam0, zin, gin, zout, gout, C, pout, par,
                 save);
    } else if (mode == 2) {
        hipLaunchKernelGGL(k_pgd_reduce, dim3(1), dim3(kThreads), 0, s, C, par);
        launch_k(k_spmv<T, 2>, dim3(nb), dim3(kThreads), 0, s, G, qv, dA, gam0, zin, gin, zout, gout, C, pout, par,
                 (double *)nullptr);
    } else
        launch_k(k_spmv<T, 1>, dim3(nb), dim3(kThreads), 0, s, G, qv, dA, gam0, zin, gin, zout, gout, C, pout, par,
                 (double *)nullptr);
}

template <typename T>
void launch_set_lcpdev(LcpDev<T> *D, const LcpDev<T> &v, hipStream_t s) {
    hipLaunchKernelGGL((k_set_lcpdev<T>), dim3(1), dim3(64), 0, s, D, v);
}

template <typename T>
void launch_spmv_dev(const LcpDev<T> *D, int grid_rows, int par, hipStream_t s) {
    hipLaunchKernelGGL((k_spmv_dev<T>), dim3(nblk(grid_rows > 0 ? grid_rows : 1, kThreads)), dim3(kThreads), 0, s, D,
                       par);
}

template <typename T>
int make_spmv_graph(const LcpDev<T> *D, int grid_rows, int k, hipGraphExec_t *out) {
    *out = nullptr;
    if (k <= 0 || (k & 1)) return -1;
    hipGraph_t g = nullptr;
    if (hipGraphCreate(&g, 0) != hipSuccess) return -1;
    const LcpDev<T> *dp = D;
    hipGraphNode_t prev = nullptr;
    int rc = 0;
    for (int t = 0; t < k && rc == 0; ++t) {
        int par = (t & 1) ? 0 : 1;  // the passes of a chunk start at an odd iteration
        void *args[] = {(void *)&dp, (void *)&par};
        hipKernelNodeParams p{};
        p.func = reinterpret_cast<void *>(&k_spmv_dev<T>);
        p.gridDim = dim3(nblk(grid_rows > 0 ? grid_rows : 1, kThreads));
        p.blockDim = dim3(kThreads);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        if (hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess) rc = -1;
        prev = node;
    }
    if (rc == 0 && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) {
        *out = nullptr;
        rc = -1;
    }
    (void)hipGraphDestroy(g);
    return rc;
}

template <typename T>
void launch_rowstate_unpack(int m, const RowStep<T> *z0, const RowStep<T> *z1, const T *g0, const T *g1,
                            const PgdState *fin, const int *done, int last_par, T *gam, T *g, double *gam64,
                            hipStream_t s, const T *qv, double *work) {
    if (m > 0 || work)
        hipLaunchKernelGGL((k_rowstate_unpack<T>), dim3(work_blocks(m)), dim3(kThreads), 0, s, m, z0, z1, g0, g1,
                           fin, done, last_par, gam, g, gam64, qv, work);
}

bool unpack_can_check(int m) { return work_blocks(m) <= kPartRegs * kThreads; }

void launch_report_check(const TailReport &R, const PgdCtl &C, hipStream_t s) {
    hipLaunchKernelGGL(k_report_check, dim3(1), dim3(kThreads), 0, s, R, C);
}

#define RELCP_INST(T)                                                                                              \
    template void launch_lcp_scatter<T>(int, const RowsT<T> &, const BodiesT<T> &, const PgdCtl &, int,           \
                                        hipStream_t);                                                             \
    template void launch_lcp_gather<T>(int, const RowsT<T> &, const BodiesT<T> &, double, const PgdCtl &, int,    \
                                       hipStream_t);                                                              \
    template void launch_lcp_spmv<T>(int, const RowGraphT<T> &, const T *, const T *, const StartSrc &,           \
                                     const RowStep<T> *, const T *, RowStep<T> *, T *, const PgdCtl &, double *,  \
                                     int, hipStream_t, double *);                                                 \
    template void launch_rowstate_unpack<T>(int, const RowStep<T> *, const RowStep<T> *, const T *, const T *,    \
                                            const PgdState *, const int *, int, T *, T *, double *, hipStream_t,  \
                                            const T *, double *);                                                 \
    template void launch_set_lcpdev<T>(LcpDev<T> *, const LcpDev<T> &, hipStream_t);                               \
    template void launch_spmv_dev<T>(const LcpDev<T> *, int, int, hipStream_t);                                    \
    template int make_spmv_graph<T>(const LcpDev<T> *, int, int, hipGraphExec_t *);
RELCP_INST(double)
RELCP_INST(float)
#undef RELCP_INST

void launch_promote(int m, const float *g32, double *g64, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_promote, dim3(nblk(m, 256)), dim3(256), 0, s, m, g32, g64);
}
void launch_demote(int m, const double *g64, float *g32, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_demote, dim3(nblk(m, 256)), dim3(256), 0, s, m, g64, g32);
}

int work_blocks(int m) { return nblk(m > 0 ? m : 1, kThreads); }

void launch_work(int m, const double *gam, const double *g, const double *qv, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_work, dim3(work_blocks(m)), dim3(kThreads), 0, s, m, gam, g, qv, partials);
}

void launch_pair_lambda(int m, const int *rec, const int *pair, const double *gam, int level, double *lam,
                        hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_pair_lambda, dim3(nblk(m, 256)), dim3(256), 0, s, m, rec, pair, gam, level, lam);
}

}  // namespace relcp
