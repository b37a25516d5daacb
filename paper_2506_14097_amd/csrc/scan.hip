// scan.hip -- exclusive prefix sums for compaction, CSR offsets and cells.
//
// Three passes: per-block scans of 2048 items (256 threads x 8 items, wave
// scans through DPP shuffles, block totals through LDS), a recursive scan of
// the block totals, and an add-back pass.
#include "common.h"

namespace relcp {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (RELCP_WAVE - 1);
#pragma unroll
    for (int o = 1; o < RELCP_WAVE; o <<= 1) {
        int t = __shfl_up(v, o, RELCP_WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

__global__ void __launch_bounds__(kThreads) k_scan_tiles(const int *__restrict__ in, int *__restrict__ out, int n,
                                                         int *__restrict__ tile_sums) {
    __shared__ int wsum[kThreads / RELCP_WAVE];
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
    int v[kItems];
    int acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        long long i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        acc += v[k];
    }
    int inc = wave_incl_scan(acc);
    const int lane = threadIdx.x & (RELCP_WAVE - 1), w = threadIdx.x / RELCP_WAVE;
    if (lane == RELCP_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int woff = 0;
    for (int j = 0; j < w; ++j) woff += wsum[j];
    int run = woff + inc - acc;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        long long i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kThreads - 1) tile_sums[blockIdx.x] = woff + inc;
}

__global__ void __launch_bounds__(kThreads) k_scan_add(int *__restrict__ out, int n, const int *__restrict__ offs) {
    const long long base = (long long)blockIdx.x * kTile;
    const int add = offs[blockIdx.x];
    for (int k = threadIdx.x; k < kTile; k += kThreads) {
        long long i = base + k;
        if (i < n) out[i] += add;
    }
}

// Scan of one level; the total of the whole input ends in `total` (the top
// level is a single tile whose block sum is the total).
void scan_rec(const int *in, int *out, int n, int *scratch, int *total, hipStream_t s) {
    int nt = (n + kTile - 1) / kTile;
    if (nt == 1) {
        int *sums = total ? total : scratch;
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kThreads), 0, s, in, out, n, sums);
        return;
    }
    int *sums = scratch;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kThreads), 0, s, in, out, n, sums);
    scan_rec(sums, sums, nt, scratch + nt, total, s);
    hipLaunchKernelGGL(k_scan_add, dim3(nt), dim3(kThreads), 0, s, out, n, sums);
}

}  // namespace

void exclusive_scan(const int *in, int *out, int n, int *total_dev, DBuf<int> &scratch, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) HIP_OK(hipMemsetAsync(total_dev, 0, sizeof(int), s));
        return;
    }
    size_t need = 1;
    for (long long m = n; m > 1; m = (m + kTile - 1) / kTile) need += (m + kTile - 1) / kTile;
    scratch.ensure(need + 2);
    scan_rec(in, out, n, scratch.p, total_dev, s);
}

}  // namespace relcp
