// report.h -- the fixed-order reduction of one recursion's tail results
// (largest displacement key of the trial, smallest Phi and margin keys of
// the overlap check, the work gamma^T A gamma) into host-mapped memory,
// then a token written last after a system-scope fence: the host polls the
// token.  Run by one workgroup of 256 threads, either the report kernel
// (which also adds up the violator count from the overlap check's per-group
// flag counts) or the last workgroup of a compaction of the violators.
#pragma once

#include "common.h"

namespace relcp {

struct TailReport {
    int nt;                            // trial blocks
    const unsigned long long *disp;    // their displacement keys
    int ns;                            // overlap-check blocks (0: none)
    const unsigned long long *phi, *marg;
    int nw;                            // work partial sums
    const double *work;
    unsigned long long *red_h;         // host-mapped: [0] displacement, [1] Phi, [2] margin keys
    double *work_h;                    // host-mapped: the work
    int *tok;                          // host-mapped token (or null)
    int seq;
    // the overlap check's flag counts per group of 256 pairs (ng groups),
    // summed into *count (the violator count), or gcount null
    int ng = 0;
    const int *gcount = nullptr;
    int *count = nullptr;
};

__device__ inline unsigned long long u64_max(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
__device__ inline unsigned long long u64_min(unsigned long long a, unsigned long long b) { return a < b ? a : b; }

// Strided per-thread sums, then a fixed shuffle tree and the four waves in
// order, so the work sum is the same on every run.  All 256 threads of the
// workgroup call it.  Thread t takes items t, t + 256, ... of each array in
// that order, kTailU of each array per round with all their loads issued
// before any use; the first round's loads can be issued early
// (tail_preload), so that their latency overlaps other work of the caller.
constexpr int kTailU = 4;
struct TailRegs {
    unsigned long long vd[kTailU], vp[kTailU], vq[kTailU];
    double vw[kTailU];
    int vc[kTailU];
};
__device__ inline void tail_load(const TailReport &R, int k0, TailRegs &v) {
    const int ng = R.gcount ? R.ng : 0;
#pragma unroll
    for (int u = 0; u < kTailU; ++u) {
        const int k = k0 + u * 256;
        v.vd[u] = k < R.nt ? R.disp[k] : 0ull;
        v.vp[u] = k < R.ns ? R.phi[k] : ~0ull;
        v.vq[u] = k < R.ns ? R.marg[k] : ~0ull;
        v.vw[u] = k < R.nw ? R.work[k] : 0.0;
        v.vc[u] = k < ng ? R.gcount[k] : 0;
    }
}
__device__ inline void tail_preload(const TailReport &R, TailRegs &v) { tail_load(R, threadIdx.x, v); }

// pre: run by every thread just before the barrier (a caller's own wave
// results into LDS); post: run by thread 0 just after it, before the
// report's writes (the caller's own block result), so that both share the
// report's one barrier.
struct NoHook {
    __device__ void operator()() const {}
};
template <class Pre = NoHook, class Post = NoHook>
__device__ inline void tail_report(const TailReport &R, const TailRegs &first, const Pre &pre = Pre{},
                                   const Post &post = Post{}) {
    __shared__ unsigned long long s0[4], s1[4], s2[4];
    __shared__ double s3[4];
    unsigned long long d = 0ull, p = ~0ull, q = ~0ull;
    double w = 0.0;
    int c = 0;
    const int ng = R.gcount ? R.ng : 0;
    const int nmax = max(max(R.nt, R.ns), max(R.nw, ng));
    TailRegs v = first;
    for (int k0 = threadIdx.x; k0 < nmax; k0 += kTailU * 256) {
        if (k0 != (int)threadIdx.x) tail_load(R, k0, v);
#pragma unroll
        for (int u = 0; u < kTailU; ++u) {
            const int k = k0 + u * 256;
            d = u64_max(d, v.vd[u]);
            p = u64_min(p, v.vp[u]);
            q = u64_min(q, v.vq[u]);
            if (k < R.nw) w += v.vw[u];
            c += v.vc[u];
        }
    }
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) {
        d = u64_max(d, __shfl_xor(d, o, RELCP_WAVE));
        p = u64_min(p, __shfl_xor(p, o, RELCP_WAVE));
        q = u64_min(q, __shfl_xor(q, o, RELCP_WAVE));
        w += __shfl_xor(w, o, RELCP_WAVE);
        c += __shfl_xor(c, o, RELCP_WAVE);
    }
    __shared__ int s4[4];
    const int lane = threadIdx.x & (RELCP_WAVE - 1), wv = threadIdx.x / RELCP_WAVE;
    if (lane == 0) {
        s0[wv] = d;
        s1[wv] = p;
        s2[wv] = q;
        s3[wv] = w;
        s4[wv] = c;
    }
    pre();
    __syncthreads();
    if (threadIdx.x == 0) {
        post();
        for (int k = 1; k < 4; ++k) {
            d = u64_max(d, s0[k]);
            p = u64_min(p, s1[k]);
            q = u64_min(q, s2[k]);
            w += s3[k];
            c += s4[k];
        }
        if (R.gcount) *R.count = c;
        R.red_h[0] = d;
        R.red_h[1] = p;
        R.red_h[2] = q;
        R.work_h[0] = w;
        if (R.tok) {
            // everything the host reads after this recursion is written: the
            // token goes last, after a system-scope fence
            __threadfence_system();
            *(volatile int *)R.tok = R.seq;
        }
    }
}

__device__ inline void tail_report(const TailReport &R) {
    TailRegs v;
    tail_preload(R, v);
    tail_report(R, v);
}

}  // namespace relcp
