// mlp.hip -- learned warm start of the LCP: per-row features, a small MLP
// (8 -> 128 -> 128 -> 1, exact GELU) correcting the previous-step multiplier,
// on the matrix cores
// (bf16 operands, fp32 accumulation), its backward pass and Adam.
//
// The paper leaves the start of the LCP iteration open: the projected
// gradient solve of the constrained quadratic program (Eq. cqpp) converges
// from any nonnegative start, so a better start only saves iterations.  The
// previous-step multiplier of the pair remains the fallback and a feature.
//
// Matrix-core layout (v_mfma_f32_32x32x8bf16_1k, one wave; checked on the
// device): lane l holds A[l % 32][4 (l / 32) + e] and B[4 (l / 32) + e][l % 32]
// for e = 0..3, and accumulator r holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Hence accumulators 4s..4s+3 of a 32x32 tile D are, lane by lane, the A
// operand of D^T for k-chunk s: products with a transposed activation need
// no trip through LDS.
#include "mlp.h"

#include <algorithm>
#include <cmath>

namespace relcp {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int HID = 128;
constexpr int NF = 8;
constexpr int LDP = HID + 4;  // padded LDS row (bf16): rows start 2 banks apart
constexpr int OW1 = 0, OB1 = 1024, OW2 = 1152, OB2 = 17536, OW3 = 17664, OB3 = 17792;

// round to nearest even (hardware v_cvt_pk_bf16_f32)
__device__ inline short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }

// Standard normal CDF and density for the exact GELU, x Phi(x), and its
// derivative Phi(x) + x phi(x).  erfc(u) = t P(t) exp(-u^2), t = 1/(1 + p u),
// with the five-term polynomial of Abramowitz & Stegun 7.1.26 (absolute
// error below 1.5e-7); taking Phi(x) = erfc(|x|/sqrt 2)/2 for x < 0 and one
// minus it otherwise avoids cancellation.  Branch free: one reciprocal, one
// exponential, a handful of fma.
__device__ inline void normal_cdf_pdf(float x, float &cdf, float &pdf) {
    const float u = fabsf(x) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
    const float P = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                             0.254829592f);
    const float e = __expf(-0.5f * x * x);
    const float q = 0.5f * P * e;
    cdf = x < 0.0f ? q : 1.0f - q;
    pdf = 0.39894228040143268f * e;
}
__device__ inline float gelu(float x) {
    float c, d;
    normal_cdf_pdf(x, c, d);
    return x * c;
}
__device__ inline float gelu_prime(float x) {
    float c, d;
    normal_cdf_pdf(x, c, d);
    return fmaf(x, d, c);
}

__device__ inline f32x16 mfma(bf16x4 a, bf16x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline bf16x4 ld4(const short *p) { return *reinterpret_cast<const bf16x4 *>(p); }
// row of the accumulator register r in lane half kh
__device__ inline int crow(int r, int kh) { return 8 * (r >> 2) + 4 * kh + (r & 3); }

template <bool TRAIN, int NW>
struct MlpLds {
    short W2[HID * LDP];  // [j][k], bf16
    short W1[HID * NF];   // [j][f], bf16
    float b1[HID], b2[HID], w3[HID];
    short H1[NW][32 * LDP];  // per wave [i][j], bf16; backward: dZ2 (bf16) once dW2 is done
    short X[NW][32 * NF];    // per wave standardised inputs, bf16
};

// One tile of 32 rows per wave, NW waves per block, tiles walked in
// block-uniform rounds.  Inference: y0 = max(0, x_2 + scale z) (x_2 = raw
// feature 2, the previous-step multiplier), times rowscale when given.
// TRAIN: forward, then the backward pass of the batch loss
// mean((z - (y - x_2) / scale)^2), writing the tile's gradient contribution
// to its own slot of `partial` (summed later in a fixed order, so results do
// not depend on scheduling).
template <bool TRAIN, int NW>
__global__ void __launch_bounds__(NW * 64) k_mlp(MlpArgs A) {
    __shared__ MlpLds<TRAIN, NW> S;
    {
        // weights to LDS in bf16: all loads of a thread in flight at once
        // (params is 16-byte aligned; W1 and W2 start at multiples of 4)
        constexpr int N2 = HID * HID / 4 / (NW * 64), N1 = HID * NF / 4 / (NW * 64);
        static_assert(N2 * NW * 64 * 4 == HID * HID && N1 * NW * 64 * 4 == HID * NF, "staging split");
        const float4 *P4 = reinterpret_cast<const float4 *>(A.params);
        float4 v2[N2], v1[N1];
#pragma unroll
        for (int i = 0; i < N2; ++i) v2[i] = P4[OW2 / 4 + threadIdx.x + i * NW * 64];
#pragma unroll
        for (int i = 0; i < N1; ++i) v1[i] = P4[OW1 / 4 + threadIdx.x + i * NW * 64];
#pragma unroll
        for (int i = 0; i < N2; ++i) {
            const int k = 4 * (threadIdx.x + i * NW * 64);  // 4 consecutive entries of one row
            short *d = &S.W2[(k >> 7) * LDP + (k & 127)];
            d[0] = to_bf16(v2[i].x);
            d[1] = to_bf16(v2[i].y);
            d[2] = to_bf16(v2[i].z);
            d[3] = to_bf16(v2[i].w);
        }
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            short *d = &S.W1[4 * (threadIdx.x + i * NW * 64)];
            d[0] = to_bf16(v1[i].x);
            d[1] = to_bf16(v1[i].y);
            d[2] = to_bf16(v1[i].z);
            d[3] = to_bf16(v1[i].w);
        }
    }
    for (int k = threadIdx.x; k < HID; k += NW * 64) {
        S.b1[k] = A.params[OB1 + k];
        S.b2[k] = A.params[OB2 + k];
        S.w3[k] = A.params[OW3 + k];
    }
    __syncthreads();
    const float b3 = A.params[OB3];
    const float scale = A.norm[2 * NF];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lo = l & 31, kh = l >> 5;
    const int ntiles = (A.n + 31) / 32;
    for (int base = blockIdx.x * NW; base < ntiles; base += gridDim.x * NW) {
        const int tile = base + w;
        const bool live = tile < ntiles;
        const int row0 = tile * 32;
        // ---- inputs: lane holds row lo, features 4 kh .. 4 kh + 3
        bf16x4 a1;
        {
            const int row = row0 + lo;
            const bool ok = live && row < A.n;
            const int gi = ok ? (A.idx ? A.idx[row] : row) : 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int f = 4 * kh + e;
                const float xv = ok ? (A.X[(size_t)gi * NF + f] - A.norm[f]) / A.norm[NF + f] : 0.0f;
                a1[e] = to_bf16(xv);
                S.X[w][lo * NF + f] = a1[e];
            }
        }
        // ---- layer 1 (K = 8: one product per 32 columns)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x4 b = ld4(&S.W1[(nt * 32 + lo) * NF + 4 * kh]);
            f32x16 c = {0};
            c = mfma(a1, b, c);
            const int j = nt * 32 + lo;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = crow(r, kh);
                const float z = c[r] + S.b1[j];
                S.H1[w][i * LDP + j] = to_bf16(gelu(z));
            }
        }
        __syncthreads();
        // ---- layer 2: Z2 = H1 W2^T + b2, kept in registers (c2)
        f32x16 c2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) c2[nt] = f32x16{0};
#pragma unroll 2
        for (int s = 0; s < HID / 8; ++s) {
            const bf16x4 a = ld4(&S.H1[w][lo * LDP + 8 * s + 4 * kh]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) c2[nt] = mfma(a, ld4(&S.W2[(nt * 32 + lo) * LDP + 8 * s + 4 * kh]), c2[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float bj = S.b2[nt * 32 + lo];
#pragma unroll
            for (int r = 0; r < 16; ++r) c2[nt][r] += bj;
        }
        // ---- layer 3: each half-wave sums its 32 columns with xor shuffles;
        // every lane ends with the outputs of its 16 rows
        // (training keeps H2 and overwrites c2 with GELU'(Z2))
        float zr[16];
        float h2[TRAIN ? 4 : 1][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float p = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float t = c2[nt][r];
                float cdf, pdf;
                normal_cdf_pdf(t, cdf, pdf);
                const float h = t * cdf;
                p += h * S.w3[nt * 32 + lo];
                if constexpr (TRAIN) {
                    h2[nt][r] = h;
                    c2[nt][r] = fmaf(t, pdf, cdf);
                }
            }
#pragma unroll
            for (int off = 1; off < 32; off <<= 1) p += __shfl_xor(p, off, 64);
            zr[r] = p + b3;
        }
        if constexpr (!TRAIN) {
            if (lo == 0 && live) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = row0 + crow(r, kh);
                    if (row < A.n) {
                        const int gi = A.idx ? A.idx[row] : row;
                        const float y0 = fmaxf(0.0f, fmaf(scale, zr[r], A.X[(size_t)gi * NF + 2]));
                        const double rs = A.rowscale ? A.rowscale[gi] : 1.0;
                        if (A.out32) A.out32[gi] = (float)(y0 * rs);
                        if (A.out64) A.out64[gi] = (double)y0 * rs;
                        if (A.zout) A.zout[gi] = zr[r];
                    }
                }
            }
            __syncthreads();
        } else {
            // ================= backward =================
            float dz[16];
            float lsum = 0.0f, dzsum = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + crow(r, kh);
                dz[r] = 0.0f;
                if (live && row < A.n) {
                    const int gi = A.idx ? A.idx[row] : row;
                    const float d = zr[r] - (A.y[gi] - A.X[(size_t)gi * NF + 2]) / scale;
                    dz[r] = A.scale2 * d;
                    lsum += d * d;
                    dzsum += dz[r];
                }
            }
            float *P = A.partial + (size_t)(live ? tile : 0) * MLP_SLOT;
            dzsum += __shfl_xor(dzsum, 32, 64);
            lsum += __shfl_xor(lsum, 32, 64);
            if (live && l == 0) {
                P[OB3] = dzsum;
                P[MLP_SLOT - 1] = lsum;
            }
            // w3 gradient (sum over rows of dz H2), dZ2 = (dz w3^T) * GELU'(Z2)
            // in place in c2, b2 gradient; each lane sums its 16 rows, then
            // the other half-wave's
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float w3j = S.w3[nt * 32 + lo];
                float s3 = 0.0f, s2 = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    s3 += dz[r] * h2[nt][r];
                    const float d = dz[r] * w3j * c2[nt][r];
                    c2[nt][r] = d;
                    s2 += d;
                }
                s3 += __shfl_xor(s3, 32, 64);
                s2 += __shfl_xor(s2, 32, 64);
                if (live && kh == 0) {
                    P[OW3 + nt * 32 + lo] = s3;
                    P[OB2 + nt * 32 + lo] = s2;
                }
            }
            // dZ2 in bf16, held as the A operands of dZ2^T (k-chunk s = rows 8s..8s+7)
            bf16x4 at[4][4];
#pragma unroll
            for (int jt = 0; jt < 4; ++jt)
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int e = 0; e < 4; ++e) at[jt][s][e] = to_bf16(c2[jt][4 * s + e]);
            // dW2[j][k] = sum_i dZ2[i][j] H1[i][k]
            float *P2 = P + OW2 + 4 * kh * HID + lo;
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) {
#pragma unroll 1
                for (int kt = 0; kt < 4; ++kt) {
                    f32x16 acc = {0};
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        bf16x4 b;
#pragma unroll
                        for (int e = 0; e < 4; ++e) b[e] = S.H1[w][(8 * s + 4 * kh + e) * LDP + kt * 32 + lo];
                        acc = mfma(at[jt][s], b, acc);
                    }
                    if (live) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) P2[(jt * 32 + 8 * (r >> 2) + (r & 3)) * HID + kt * 32] = acc[r];
                    }
                }
            }
            // H1 is no longer needed: its LDS tile takes dZ2 (bf16)
            __syncthreads();
#pragma unroll
            for (int jt = 0; jt < 4; ++jt)
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int e = 0; e < 4; ++e) S.H1[w][(8 * s + 4 * kh + e) * LDP + jt * 32 + lo] = at[jt][s][e];
            __syncthreads();
            // dH1 = dZ2 W2, dZ1 = dH1 * GELU'(Z1) (Z1 recomputed: one product
            // per 32 columns), then the b1 and W1 gradients
#pragma unroll 1
            for (int kt = 0; kt < 4; ++kt) {
                f32x16 acc = {0};
#pragma unroll 2
                for (int s = 0; s < HID / 8; ++s) {
                    bf16x4 b;
#pragma unroll
                    for (int e = 0; e < 4; ++e) b[e] = S.W2[(8 * s + 4 * kh + e) * LDP + kt * 32 + lo];
                    acc = mfma(ld4(&S.H1[w][lo * LDP + 8 * s + 4 * kh]), b, acc);
                }
                const int kc = kt * 32 + lo;
                f32x16 z1 = {0};
                z1 = mfma(a1, ld4(&S.W1[kc * NF + 4 * kh]), z1);
                const float b1k = S.b1[kc];
                float s1 = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc[r] *= gelu_prime(z1[r] + b1k);
                    s1 += acc[r];
                }
                s1 += __shfl_xor(s1, 32, 64);
                if (live && kh == 0) P[OB1 + kc] = s1;
                // dW1[j][f] = sum_i dZ1[i][j] X[i][f]  (the 8 features padded to 32 columns)
                f32x16 acc1 = {0};
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    bf16x4 a, b;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        a[e] = to_bf16(acc[4 * s + e]);
                        b[e] = lo < NF ? S.X[w][(8 * s + 4 * kh + e) * NF + lo] : (short)0;
                    }
                    acc1 = mfma(a, b, acc1);
                }
                if (live && lo < NF) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) P[OW1 + (kt * 32 + crow(r, kh)) * NF + lo] = acc1[r];
                }
            }
            __syncthreads();
        }
    }
}

// grad[p] = (sum over slots of partial[slot][p]) in slot order; the loss
// slot entry gives the mean loss.
__global__ void k_mlp_reduce(const float *__restrict__ partial, int nslots, float inv_n, float *__restrict__ grad,
                             float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NPARAM) return;
    const int src = p < MLP_NPARAM ? p : MLP_SLOT - 1;
    float s = 0.0f;
    for (int k = 0; k < nslots; ++k) s += partial[(size_t)k * MLP_SLOT + src];
    if (p < MLP_NPARAM)
        grad[p] = s;
    else if (loss)
        *loss = s * inv_n;
}

__global__ void k_zero(int n, float *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0.0f;
}

// Adam with the bias corrections folded into the step and epsilon
// (c1 = 1 - b1 and c2 = 1 - b2 rounded from double: 1 - 0.999f in fp32
// would be 1.3e-5 off)
__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr_t, float b1, float c1, float b2, float c2, float eps_t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + c1 * gi;
    const float vi = b2 * v[i] + c2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
}

// ---------------------------------------------------------------------------
// features of the iteration-0 rows
// ---------------------------------------------------------------------------
__device__ inline double mean_semiaxis(int kind, double a, double b, double c) {
    // spherocylinder: radius a, cylinder length b -> semi-extents a, a, b/2 + a
    return kind == 0 ? (a + b + c) / 3.0 : (3.0 * a + 0.5 * b) / 3.0;
}
__device__ inline double semiaxis_ratio(int kind, double a, double b, double c) {
    return kind == 0 ? fmin(a, fmin(b, c)) / fmax(a, fmax(b, c)) : a / (0.5 * b + a);
}

__global__ void k_features(FeatureArgs A) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.m0) return;
    const int a = A.ia[r], b = A.ib[r];
    const int L = A.ldr, lb = A.ldb;
    const d3 n = mk(A.n[r], A.n[L + r], A.n[2 * L + r]);
    const double *p = A.p;
    const int ka = A.kind[a], kb = A.kind[b];
    const double abar = 0.5 * (mean_semiaxis(ka, p[a], p[lb + a], p[2 * lb + a]) +
                               mean_semiaxis(kb, p[b], p[lb + b], p[2 * lb + b]));
    double rate = 0.0;
    if (A.u) {
        const double *U = A.u;
        const d3 ta = mk(A.ta[r], A.ta[L + r], A.ta[2 * L + r]);
        const d3 tb = mk(A.tb[r], A.tb[L + r], A.tb[2 * L + r]);
        rate = -(dot(n, mk(U[a], U[lb + a], U[2 * lb + a])) + dot(ta, mk(U[3 * lb + a], U[4 * lb + a], U[5 * lb + a]))) +
               dot(n, mk(U[b], U[lb + b], U[2 * lb + b])) + dot(tb, mk(U[3 * lb + b], U[4 * lb + b], U[5 * lb + b]));
    }
    const int ea0 = A.off[a], ea1 = A.lcnt ? ea0 + A.lcnt[a] : A.off[a + 1];
    const int eb0 = A.off[b], eb1 = A.lcnt ? eb0 + A.lcnt[b] : A.off[b + 1];
    double ca = ea1 - ea0, cb = eb1 - eb0;
    double ra = semiaxis_ratio(ka, p[a], p[lb + a], p[2 * lb + a]);
    double rb = semiaxis_ratio(kb, p[b], p[lb + b], p[2 * lb + b]);
    // overlap load of the other rows at a and at b
    double load = 0.0;
    for (int k = ea0; k < ea1; ++k) {
        const int o = A.ent[k] >> 1;
        if (o != r) load += fmax(0.0, -A.phi[o]);
    }
    for (int k = eb0; k < eb1; ++k) {
        const int o = A.ent[k] >> 1;
        if (o != r) load += fmax(0.0, -A.phi[o]);
    }
    if (A.perm[a] > A.perm[b]) {  // orient by caller index
        double t = ca; ca = cb; cb = t;
        t = ra; ra = rb; rb = t;
    }
    const double rs = abar / A.dA[r];
    A.rowscale[r] = rs;
    float *f = A.feat + (size_t)r * NF;
    f[0] = (float)(A.phi[r] / abar);
    f[1] = (float)(A.dt * rate / abar);
    f[2] = (float)(A.lam[r] / rs);
    f[3] = (float)ca;
    f[4] = (float)cb;
    f[5] = (float)ra;
    f[6] = (float)rb;
    f[7] = (float)(load / abar);
}

__global__ void k_log_rows(int m0, const float *__restrict__ feat, const double *__restrict__ gam,
                           const double *__restrict__ rowscale, const int *__restrict__ ia,
                           const int *__restrict__ ib, const int *__restrict__ perm, float *__restrict__ of,
                           float *__restrict__ og, int *__restrict__ oa, int *__restrict__ ob) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m0) return;
    if (of)
        for (int k = 0; k < NF; ++k) of[(size_t)r * NF + k] = feat[(size_t)r * NF + k];
    if (og) og[r] = (float)(gam[r] / rowscale[r]);
    const int pa = perm[ia[r]], pb = perm[ib[r]];
    if (oa) oa[r] = pa < pb ? pa : pb;
    if (ob) ob[r] = pa < pb ? pb : pa;
}

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_features(const FeatureArgs &a, hipStream_t s) {
    if (a.m0 > 0) launch_k(k_features, dim3(nblk(a.m0, 256)), dim3(256), 0, s, a);
}

void launch_mlp_forward(const MlpArgs &a, hipStream_t s) {
    if (a.n <= 0) return;
    constexpr int NW = 4;
    const int tiles = (a.n + 31) / 32;
    // persistent: two resident blocks per CU (73 KB of LDS each), weights
    // staged once per block
    const int blocks = std::min(nblk(tiles, NW), 512);
    launch_k(k_mlp<false, NW>, dim3(blocks), dim3(NW * 64), 0, s, a);
}

int mlp_slots(int n) { return std::max(1, (n + 31) / 32); }

void launch_mlp_grad(const MlpArgs &a, float *grad, float *loss, hipStream_t s) {
    constexpr int NW = 4;
    const int tiles = (a.n + 31) / 32;
    if (tiles > 0) {
        launch_k(k_mlp<true, NW>, dim3(nblk(tiles, NW)), dim3(NW * 64), 0, s, a);
        hipLaunchKernelGGL(k_mlp_reduce, dim3(nblk(MLP_NPARAM + 1, 256)), dim3(256), 0, s, a.partial, tiles,
                           1.0f / (float)a.n, grad, loss);
    } else {
        hipLaunchKernelGGL(k_zero, dim3(nblk(MLP_NPARAM, 256)), dim3(256), 0, s, MLP_NPARAM, grad);
        if (loss) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, 1, loss);
    }
}

void launch_adam(float *p, const float *g, float *m, float *v, float lr, int t, hipStream_t s) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    // p -= lr (m / k1) / (sqrt(v / k2) + eps) = lr_t m / (sqrt(v) + eps sqrt(k2)),
    // k1 = 1 - b1^t, k2 = 1 - b2^t (bias corrections)
    const double k1 = 1.0 - std::pow(b1, t), k2 = 1.0 - std::pow(b2, t);
    const float lr_t = (float)(lr * std::sqrt(k2) / k1);
    const float eps_t = (float)(eps * std::sqrt(k2));
    hipLaunchKernelGGL(k_adam, dim3(nblk(MLP_NPARAM, 256)), dim3(256), 0, s, MLP_NPARAM, p, g, m, v, lr_t, (float)b1,
                       (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), eps_t);
}

void launch_log_rows(int m0, const float *feat, const double *gam, const double *rowscale, const int *ia,
                     const int *ib, const int *perm, float *out_feat, float *out_gam, int *out_ia, int *out_ib,
                     hipStream_t s) {
    if (m0 > 0)
        hipLaunchKernelGGL(k_log_rows, dim3(nblk(m0, 256)), dim3(256), 0, s, m0, feat, gam, rowscale, ia, ib, perm,
                           out_feat, out_gam, out_ia, out_ib);
}

}  // namespace relcp
