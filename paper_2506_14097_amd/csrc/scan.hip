// scan.hip -- exclusive prefix sums (CSR offsets, cell lists, slice bases)
// and stream compaction of flagged items.
//
// A scan of at most kSmall items runs in one block of 1024 threads.  A
// larger one takes two passes over tiles of 2048 items (256 threads x 8
// items): the tile totals, then the tile scans, each block adding the sum of
// the totals of the tiles before its own (it sums them itself while there are
// at most kDirect tiles, 16 loads per thread; past that the totals are
// scanned first, by the same routine).  Within a tile: wave scans through
// cross-lane shuffles, wave totals through LDS.  Every sum is over integers, so the order does not
// change the result.
#include "common.h"
#include "report.h"
#include "../../include/relcp.h"

#include <mutex>

namespace relcp {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kSmallThreads = 1024;
constexpr int kSmall = kSmallThreads * kItems;
constexpr int kDirect = 4096;  // tiles (groups) whose offsets a block sums by itself

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (RELCP_WAVE - 1);
#pragma unroll
    for (int o = 1; o < RELCP_WAVE; o <<= 1) {
        int t = __shfl_up(v, o, RELCP_WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline int wave_total(int v) {
#pragma unroll
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RELCP_WAVE);
    return v;
}

// sum of v over the block (every thread gets it); sh holds one int per wave
template <int NT>
__device__ inline int block_total(int v, int *sh) {
    v = wave_total(v);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int k = 0; k < NT / RELCP_WAVE; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// Exclusive scan of the kItems values of each thread of an NT-thread block,
// offset by `base`: on return v[k] holds the exclusive prefix of item k and
// the block total is returned.
template <int NT>
__device__ inline int block_scan_items(int (&v)[kItems], int base, int *wsum) {
    int acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) acc += v[k];
    const int inc = wave_incl_scan(acc);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    if (lane == RELCP_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int woff = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < NT / RELCP_WAVE; ++j) {
        woff += j < w ? wsum[j] : 0;
        tot += wsum[j];
    }
    int run = base + woff + inc - acc;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int x = v[k];
        v[k] = run;
        run += x;
    }
    return tot;
}

__global__ void __launch_bounds__(kSmallThreads) k_scan_small(const int *__restrict__ in, int *__restrict__ out,
                                                              int n, int *__restrict__ total) {
    __shared__ int wsum[kSmallThreads / RELCP_WAVE];
    const int base = threadIdx.x * kItems;
    int v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = base + k < n ? in[base + k] : 0;
    const int tot = block_scan_items<kSmallThreads>(v, 0, wsum);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) out[base + k] = v[k];
    if (total && threadIdx.x == 0) *total = tot;
}

__global__ void __launch_bounds__(kThreads) k_tile_sums(const int *__restrict__ in, int n, int *__restrict__ sums) {
    __shared__ int sh[kThreads / RELCP_WAVE];
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) acc += base + k < n ? in[base + k] : 0;
    const int t = block_total<kThreads>(acc, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

// The offset of tile b: offs[b] when the totals are already scanned, else
// the sum of sums[0 .. b) (every thread of the block gets it).
__device__ inline int tile_offset(const int *sums, const int *offs, int b, int *sh) {
    if (offs) return offs[b];
    int acc = 0;
    for (int k = threadIdx.x; k < b; k += kThreads) acc += sums[k];
    return block_total<kThreads>(acc, sh);
}

__global__ void __launch_bounds__(kThreads) k_scan_apply(const int *__restrict__ in, int *__restrict__ out, int n,
                                                         const int *__restrict__ sums, const int *__restrict__ offs,
                                                         int *__restrict__ total) {
    __shared__ int sh[kThreads / RELCP_WAVE];
    __shared__ int wsum[kThreads / RELCP_WAVE];
    const int b = blockIdx.x;
    const int off = tile_offset(sums, offs, b, sh);
    const long long base = (long long)b * kTile + (long long)threadIdx.x * kItems;
    int v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = base + k < n ? in[base + k] : 0;
    const int tot = block_scan_items<kThreads>(v, off, wsum);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) out[base + k] = v[k];
    if (total && b == (int)gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

// Flag counts per 256 items (for callers whose flags come without them).
__global__ void __launch_bounds__(kThreads) k_count_flags(const int *__restrict__ flags, int n,
                                                          int *__restrict__ bcount) {
    __shared__ int sh[kThreads / RELCP_WAVE];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int f = i < n && flags[i] ? 1 : 0;
    const int t = block_total<kThreads>(f, sh);
    if (threadIdx.x == 0) bcount[blockIdx.x] = t;
}

// Compaction of tile b (2048 flags = 8 count groups of 256): its offset is
// the number of set flags in the groups before it.
__global__ void __launch_bounds__(kThreads) k_compact_tiles(const int *__restrict__ flags, int n,
                                                            const int *__restrict__ bcount,
                                                            const int *__restrict__ boffs, int *__restrict__ out,
                                                            int *__restrict__ total, TailReport rep,
                                                            int *__restrict__ pos) {
    __shared__ int sh[kThreads / RELCP_WAVE];
    __shared__ int wsum[kThreads / RELCP_WAVE];
    const int b = blockIdx.x;
    const int g0 = b * (kTile / kThreads);  // first count group of the tile
    const int off = tile_offset(bcount, boffs, g0, sh);
    const long long base = (long long)b * kTile + (long long)threadIdx.x * kItems;
    int v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = base + k < n && flags[base + k] ? 1 : 0;
    int set[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) set[k] = v[k];
    const int tot = block_scan_items<kThreads>(v, off, wsum);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (set[k]) out[v[k]] = (int)(base + k);
    if (pos) {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (base + k < n) pos[base + k] = set[k] ? v[k] : -1;
    }
    if (b != (int)gridDim.x - 1) return;
    if (total && threadIdx.x == 0) *total = off + tot;
    // the count is stored (thread 0 before its fence): the tail report, whose
    // inputs all come from earlier launches, goes last
    if (rep.red_h) tail_report(rep);
}

}  // namespace

int flag_groups(int n) { return (n + kThreads - 1) / kThreads; }

// scratch use of a scan of n items: the tile totals, then (past kDirect
// tiles) their scan and the scratch of that scan
static size_t scan_scratch_need(long long n) {
    if (n <= kSmall) return 0;
    const long long nt = (n + kTile - 1) / kTile;
    size_t need = (size_t)nt;
    if (nt > kDirect) need += (size_t)nt + scan_scratch_need(nt);
    return need;
}

static void scan_into(const int *in, int *out, int n, int *total_dev, int *scratch, hipStream_t s) {
    if (n <= kSmall) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallThreads), 0, s, in, out, n, total_dev);
        return;
    }
    const int nt = (n + kTile - 1) / kTile;
    int *sums = scratch;
    hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kThreads), 0, s, in, n, sums);
    int *offs = nullptr;
    if (nt > kDirect) {
        offs = scratch + nt;
        scan_into(sums, offs, nt, nullptr, scratch + 2 * (size_t)nt, s);
    }
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kThreads), 0, s, in, out, n, sums, offs, total_dev);
}

void exclusive_scan(const int *in, int *out, int n, int *total_dev, DBuf<int> &scratch, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) HIP_OK(hipMemsetAsync(total_dev, 0, sizeof(int), s));
        return;
    }
    scratch.ensure(scan_scratch_need(n) + 2);
    scan_into(in, out, n, total_dev, scratch.p, s);
}

// ---------------------------------------------------------------------------
// the scan without allocation: tile totals in a file-scope device array
// ---------------------------------------------------------------------------
// Scratch of relcp_exclusive_scan_device_noalloc: one int per tile of a scan
// of up to RELCP_NOALLOC_SCAN_MAX items (kDirect tiles: the totals are summed
// by each block, never scanned themselves, so no further scratch).  Each GPU
// holds its own copy until the process ends.
constexpr int kNoAllocTiles = kDirect;
static_assert((long long)kNoAllocTiles * kTile == RELCP_NOALLOC_SCAN_MAX, "scratch bound");
static __device__ __align__(256) int scratch[kNoAllocTiles];

namespace {
__global__ void k_set_zero(int *p) { *p = 0; }

// The array's device address on the current device, looked up once per
// device (host code must never pass the array's own name to a kernel).
constexpr int kMaxDevices = 64;
int *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_ptr(int **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RELCP_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RELCP_E_DEVICE;
        g_scratch_ptr[dev] = static_cast<int *>(p);
    }
    *out = g_scratch_ptr[dev];
    return RELCP_OK;
}
}  // namespace

bool compact_flags(const int *flags, int n, const int *bcount, int *out, int *total_dev, DBuf<int> &scratch,
                   hipStream_t s, const TailReport *rep, int *pos) {
    if (n <= 0) {
        if (total_dev) HIP_OK(hipMemsetAsync(total_dev, 0, sizeof(int), s));
        return false;
    }
    const int ng = flag_groups(n);
    const int nt = (n + kTile - 1) / kTile;
    size_t need = 2;
    int *cnt = nullptr;
    if (!bcount) need += (size_t)ng;
    if (ng > kDirect) need += (size_t)ng + scan_scratch_need(ng);
    scratch.ensure(need);
    int *p = scratch.p;
    if (!bcount) {
        cnt = p;
        p += ng;
        hipLaunchKernelGGL(k_count_flags, dim3(ng), dim3(kThreads), 0, s, flags, n, cnt);
        bcount = cnt;
    }
    int *boffs = nullptr;
    if (ng > kDirect) {
        boffs = p;
        scan_into(bcount, boffs, ng, nullptr, p + ng, s);
    }
    TailReport none{};
    hipLaunchKernelGGL(k_compact_tiles, dim3(nt), dim3(kThreads), 0, s, flags, n, bcount, boffs, out, total_dev,
                       rep ? *rep : none, pos);
    return rep != nullptr;
}

// ---------------------------------------------------------------------------
// filtered incidence lists
// ---------------------------------------------------------------------------
namespace {
// The kept entries of item i's list (pos of the entry's index >= 0), up to
// kFiltU entries per round with all their loads in flight.
constexpr int kFiltU = 4;
template <bool WRITE>
__device__ inline int filter_list(const int *__restrict__ boff, const int *__restrict__ bent,
                                  const int *__restrict__ pos, int i, int *__restrict__ ent, int at) {
    const int j0 = boff[i], j1 = boff[i + 1];
    int c = 0;
    for (int j = j0; j < j1; j += kFiltU) {
        int e[kFiltU], q[kFiltU];
#pragma unroll
        for (int u = 0; u < kFiltU; ++u) e[u] = j + u < j1 ? bent[j + u] : -1;
#pragma unroll
        for (int u = 0; u < kFiltU; ++u) q[u] = e[u] >= 0 ? pos[e[u] >> 1] : -1;
#pragma unroll
        for (int u = 0; u < kFiltU; ++u) {
            if (q[u] < 0) continue;
            if (WRITE) ent[at + c] = (q[u] << 1) | (e[u] & 1);
            ++c;
        }
    }
    return c;
}

// One item per thread, in place in the unfiltered lists' slots: item i's
// kept entries, renumbered, in its own order at boff[i] .. boff[i] + c - 1,
// then -1 up to boff[i + 1]; cnt[i] = c, and per block of kThreads items the
// sum of c (c - 1) (ordered pairs of kept entries of one item) in bsums.
// No count pass and no scan: the offsets are the unfiltered lists'.
__global__ void __launch_bounds__(kThreads) k_filter_gapped(int n, const int *__restrict__ boff,
                                                            const int *__restrict__ bent, const int *__restrict__ pos,
                                                            int *__restrict__ cnt, int *__restrict__ ent,
                                                            int *__restrict__ bsums) {
    __shared__ int sh[kThreads / RELCP_WAVE];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    int c = 0;
    if (i < n) {
        const int j0 = boff[i], j1 = boff[i + 1];
        c = filter_list<true>(boff, bent, pos, i, ent, j0);
        for (int j = j0 + c; j < j1; ++j) ent[j] = -1;
        cnt[i] = c;
    }
    const int tp = block_total<kThreads>(c * (c - 1), sh);
    if (threadIdx.x == 0) bsums[blockIdx.x] = tp;
}

}  // namespace

int filter_blocks(int n) { return (n + kThreads - 1) / kThreads; }

void filter_lists(int n, const int *boff, const int *bent, const int *pos, int *cnt, int *ent, int *bsums,
                  hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_filter_gapped, dim3(filter_blocks(n)), dim3(kThreads), 0, s, n, boff, bent, pos, cnt, ent,
                       bsums);
}

}  // namespace relcp

extern "C" int relcp_exclusive_scan_device_noalloc(const int32_t *in, int32_t *out, int32_t n, int32_t *total,
                                                   void *stream) {
    using namespace relcp;
    if (n < 0 || (n > 0 && (!in || !out))) return RELCP_E_INVALID;
    if (n > RELCP_NOALLOC_SCAN_MAX) return RELCP_E_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    int *tiles = nullptr;
    const int rc = scratch_ptr(&tiles);
    if (rc != RELCP_OK) return rc;
    if (n == 0) {
        if (total) hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, s, total);
    } else {
        // at most kDirect tiles: scan_into uses `tiles` for their totals only
        scan_into(in, out, n, total, tiles, s);
    }
    return hipGetLastError() == hipSuccess ? RELCP_OK : RELCP_E_DEVICE;
}
