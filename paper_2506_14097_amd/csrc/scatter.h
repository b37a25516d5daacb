// scatter.h -- the per-body half of the LCP operator, V_i = K_i (D gamma)_i,
// shared by the LCP passes (lcp.hip) and the trial integration
// (geometry.hip), which forms the contact velocities itself.
#pragma once

#include "lcp.h"

namespace relcp {

// The projection must round identically in the scatter and the gather.
__device__ inline double project(double gm, double g, double dA, double al) {
    double v = __dsub_rn(gm, __ddiv_rn(__dmul_rn(al, g), dA));
    return v > 0.0 ? v : 0.0;
}
__device__ inline float project(float gm, float g, float dA, float al) {
    float v = __fsub_rn(gm, __fdiv_rn(__fmul_rn(al, g), dA));
    return v > 0.0f ? v : 0.0f;
}
template <typename T>
__device__ inline T clamp0(T v) {
    return v > T(0) ? v : T(0);
}

// Velocity storage of the LCP loop: the global array (ld, body index) or a
// packing's slice staged in LDS (ld = packing size, index minus first body).
template <typename T>
struct VGlobal {
    T *v;
    int ld;
    __device__ T &operator()(int comp, int i) const { return v[comp * ld + i]; }
};
template <typename T>
struct VLocal {
    T *v;
    int ld, b0;
    __device__ T &operator()(int comp, int i) const { return v[comp * ld + (i - b0)]; }
};

// V_i = K_i (D gamma)_i over the incident rows of body i, walking its
// incidence list in a fixed order.  MODE 0 uses max(0, gamma); MODE 1 the
// projected step with step length al.  Four rows per round so that all their
// loads are in flight together (a body has 2-3 rows on average).
template <typename T, int MODE, class VS>
__device__ inline void scatter_body(const RowsT<T> &R, const BodiesT<T> &B, int i, T al, const VS &V) {
    T f0 = 0, f1 = 0, f2 = 0, t0 = 0, t1 = 0, t2 = 0;
    const int e0 = B.off[i], e1 = B.lcnt ? e0 + B.lcnt[i] : B.off[i + 1];
    const int L = R.ld;
    constexpr int U = 4;
    for (int e = e0; e < e1; e += U) {
        int cc[U], sd[U];
        T gm[U], gg[U], da[U], n0[U], n1[U], n2[U], u0[U], u1[U], u2[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            int en = (e + k < e1) ? B.ent[e + k] : -1;
            cc[k] = en >= 0 ? (en >> 1) : -1;
            sd[k] = en & 1;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (cc[k] < 0) continue;
            const int c = cc[k];
            const T *tau = sd[k] ? R.tb : R.ta;
            gm[k] = R.gam[c];
            if (MODE == 1) {
                gg[k] = R.g[c];
                da[k] = R.dA[c];
            }
            n0[k] = R.n[c];
            n1[k] = R.n[L + c];
            n2[k] = R.n[2 * L + c];
            u0[k] = tau[c];
            u1[k] = tau[L + c];
            u2[k] = tau[2 * L + c];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (cc[k] < 0) continue;
            T gv = MODE == 1 ? project(gm[k], gg[k], da[k], al) : clamp0(gm[k]);
            T sg = sd[k] ? gv : -gv;
            f0 += sg * n0[k];
            f1 += sg * n1[k];
            f2 += sg * n2[k];
            t0 += sg * u0[k];
            t1 += sg * u1[k];
            t2 += sg * u2[k];
        }
    }
    const int lb = B.ld;
    const T *K = B.K;
    T k0, k1, k2, kxx, kyy, kzz, kxy, kxz, kyz;
    if (B.kiso) {
        // the same values the nine components hold
        k0 = k1 = k2 = K[i];
        kxx = kyy = kzz = K[3 * lb + i];
        kxy = kxz = kyz = T(0);
    } else {
        k0 = K[i];
        k1 = K[lb + i];
        k2 = K[2 * lb + i];
        kxx = K[3 * lb + i];
        kyy = K[4 * lb + i];
        kzz = K[5 * lb + i];
        kxy = K[6 * lb + i];
        kxz = K[7 * lb + i];
        kyz = K[8 * lb + i];
    }
    V(0, i) = k0 * f0;
    V(1, i) = k1 * f1;
    V(2, i) = k2 * f2;
    V(3, i) = kxx * t0 + kxy * t1 + kxz * t2;
    V(4, i) = kxy * t0 + kyy * t1 + kyz * t2;
    V(5, i) = kxz * t0 + kyz * t1 + kzz * t2;
}

// Velocity storage in registers (a body's own six values).
template <typename T>
struct VRegs {
    T *r;
    __device__ T &operator()(int comp, int) const { return r[comp]; }
};

}  // namespace relcp
