// common.h -- internal declarations of librelcp (gfx950).
//
// Layout: every per-body and per-contact quantity is structure-of-arrays
// (component k of item i at ptr[k * ld + i]) so that a wavefront of 64 lanes
// reads 64 consecutive values of one component.  Symmetric 3x3 matrices are
// stored as 6 components (xx, yy, zz, xy, xz, yz).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <string>
#include <vector>

#define RELCP_WAVE 64

namespace relcp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};

#define HIP_OK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess)                                                                         \
            throw ::relcp::Error{-3, std::string(#expr) + ": " + hipGetErrorString(_e)};              \
    } while (0)

// ---------------------------------------------------------------------------
// XCD-aware block order.  The dispatcher hands workgroup b of a launch to
// XCD b % 8 (each XCD has its own L2); xcd_block maps it to a logical block
// so that each XCD runs one contiguous range of the nb logical blocks, and
// reads of nearby items (the rows a row couples to) hit that XCD's L2.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nb) {
    const int x = b % kXcds, i = b / kXcds;
    const int q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------
// kernel timing: when an event pair is armed, the next launch made through
// launch_k takes it as the dispatch's own start and end timestamps (the
// kernel's execution, without the host's enqueue time), then disarms it
// ---------------------------------------------------------------------------
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchEvents &armed_launch_events() {
    static thread_local LaunchEvents e;
    return e;
}
template <typename K, typename... Args>
inline void launch_k(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args &&...args) {
    LaunchEvents &e = armed_launch_events();
    if (e.start) {
        const LaunchEvents t = e;
        e = LaunchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, std::forward<Args>(args)...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, std::forward<Args>(args)...);
    }
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;  // elements
    void ensure(size_t n) {
        if (n <= cap) return;
        size_t nc = cap ? cap : 256;
        while (nc < n) nc *= 2;
        if (p) HIP_OK(hipFree(p));
        p = nullptr;
        cap = 0;
        if (hipMalloc(&p, nc * sizeof(T)) != hipSuccess) {
            p = nullptr;
            throw Error{-2, "device allocation failed"};
        }
        cap = nc;
    }
    // grow keeping the first `keep` elements of each of `comps` components
    // laid out with leading dimension cap
    void grow_soa(size_t n, int comps, size_t keep, hipStream_t s) {
        if (n * comps <= cap) return;
        size_t oldld = cap / (comps ? comps : 1);
        size_t nld = oldld ? oldld : 256;
        while (nld < n) nld *= 2;
        T *np_ = nullptr;
        if (hipMalloc(&np_, nld * comps * sizeof(T)) != hipSuccess) throw Error{-2, "device allocation failed"};
        if (p && keep) {
            for (int k = 0; k < comps; ++k)
                HIP_OK(hipMemcpyAsync(np_ + k * nld, p + k * oldld, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
        }
        HIP_OK(hipStreamSynchronize(s));
        if (p) HIP_OK(hipFree(p));
        p = np_;
        cap = nld * comps;
    }
    size_t ld(int comps) const { return cap / comps; }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// ---------------------------------------------------------------------------
// small device vector helpers (FP64 geometry)
// ---------------------------------------------------------------------------
struct d3 {
    double x, y, z;
};
__host__ __device__ inline d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__host__ __device__ inline d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ inline d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline d3 operator*(double s, d3 a) { return d3{s * a.x, s * a.y, s * a.z}; }
__host__ __device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline d3 cross(d3 a, d3 b) {
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline double len(d3 a) { return sqrt(dot(a, a)); }

struct sym3 {
    double xx, yy, zz, xy, xz, yz;
};
__host__ __device__ inline d3 mul(const sym3 &S, d3 v) {
    return d3{S.xx * v.x + S.xy * v.y + S.xz * v.z, S.xy * v.x + S.yy * v.y + S.yz * v.z,
              S.xz * v.x + S.yz * v.y + S.zz * v.z};
}

// rotation matrix columns of a unit quaternion [s, w]
__host__ __device__ inline void quat_axes(double s, double x, double y, double z, d3 &c0, d3 &c1, d3 &c2) {
    c0 = d3{1 - 2 * (y * y + z * z), 2 * (x * y + s * z), 2 * (x * z - s * y)};
    c1 = d3{2 * (x * y - s * z), 1 - 2 * (x * x + z * z), 2 * (y * z + s * x)};
    c2 = d3{2 * (x * z + s * y), 2 * (y * z - s * x), 1 - 2 * (x * x + y * y)};
}

// ---------------------------------------------------------------------------
// per-packing broadphase grid
// ---------------------------------------------------------------------------
struct PackGrid {
    int nc[3];
    int periodic[3];
    double cs[3];      // cell size
    double org[3];     // origin (open directions)
    double box[3];     // periodic edge (0 = open)
    long long cell_off;
};

// ---------------------------------------------------------------------------
// LCP iteration state (device, one per solve)
// ---------------------------------------------------------------------------
struct PgdState {
    double alpha;     // current step (Jacobi-scaled variables)
    double res;       // scaled natural residual of the current iterate
    double ss, sy, yy;
    int iter;         // iterations taken
    int conv;         // 1 once res <= tol; 2: stalled (an FP32 solve whose residual stopped falling)
    unsigned ticket;  // last-block counter
    int best_iter;    // iteration at which `best` was set
    double best;      // residual of the last iterate that at least halved the one before it
};

// ---------------------------------------------------------------------------
// host launchers (each defined in the .hip file that owns the kernels)
// ---------------------------------------------------------------------------
// scan.hip: exclusive prefix sum of n ints (out may alias in); the total is
// written to total_dev[0] when total_dev is not null.  scratch grows as needed.
void exclusive_scan(const int *in, int *out, int n, int *total_dev, DBuf<int> &scratch, hipStream_t s);
// scan.hip: out[j] = index of the j-th set flag (increasing), the count to
// total_dev[0] when not null.  bcount: the set flags of each group of 256
// (flag_groups(n) entries, written by the flags' producer), or null to count
// them here.  out must not alias flags.  rep (optional): a tail report
// (report.h) that the compaction's last workgroup writes after the count;
// returns whether it was written (false when n <= 0: nothing was launched).
// pos (optional, n entries): item i's index in out, or -1 for an unset flag.
struct TailReport;
int flag_groups(int n);
bool compact_flags(const int *flags, int n, const int *bcount, int *out, int *total_dev, DBuf<int> &scratch,
                   hipStream_t s, const TailReport *rep = nullptr, int *pos = nullptr);
// scan.hip: lists of n items (boff, bent: entries (j << 1) | side, as the
// incidence lists) keeping the entries whose j has pos[j] >= 0, renumbered
// (pos[j] << 1) | side, each list in its own order and in place of the
// unfiltered one: item i's kept entries at boff[i] .. boff[i] + cnt[i] - 1 of
// ent, then -1 up to boff[i + 1] (ent has boff[n] slots).  bsums
// (filter_blocks(n) ints) <- per block of items the sum of c (c - 1), c the
// kept count (summed by the row graph's assembly).
int filter_blocks(int n);
void filter_lists(int n, const int *boff, const int *bent, const int *pos, int *cnt, int *ent, int *bsums,
                  hipStream_t s);

}  // namespace relcp
