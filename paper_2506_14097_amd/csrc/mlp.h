// mlp.h -- launch arguments of the learned warm start kernels (mlp.hip).
#pragma once

#include "common.h"

namespace relcp {

constexpr int MLP_NPARAM = 17793;  // W1 128x8, b1, W2 128x128, b2, w3, b3
constexpr int MLP_SLOT = 17800;    // floats per gradient slot (last = loss sum)
constexpr int MLP_NORM = 17;       // mean (8), std (8), correction scale

// Features of the iteration-0 rows, written oriented so that body a has the
// smaller caller index (perm: internal -> caller).  Multipliers enter in
// length units, A_aa gamma / abar (the row's own displacement per unit
// multiplier times the multiplier), so that the mobility is applied exactly
// and the network sees dimensionless numbers:
//   0 Phi_0 / abar            abar = mean of the two bodies' mean semi-extents
//   1 dt D^T U_prev / abar     previous-step velocity along the row
//   2 A_aa lambda_prev / abar  previous-step multiplier of the pair
//   3, 4 rows of A_0 incident to a, to b
//   5, 6 min / max semi-extent of a, of b
//   7 sum over the other rows of A_0 at a or b of max(0, -Phi_0) / abar
//     (the overlap load of the neighbourhood)
// rowscale[r] = abar / A_aa converts the network's output back.
struct FeatureArgs {
    int m0, ldr;
    const int *ia, *ib;
    const double *n, *ta, *tb, *phi, *lam, *dA;  // rows (SoA, ld = ldr)
    int ldb;
    const int *kind;
    const double *p, *u;        // bodies (SoA, ld = ldb); u may be null
    const int *off, *ent;       // incidence lists of A_0 (entry = row << 1 | side)
    const int *lcnt;            // their lengths (as BodiesT::lcnt), or null for CSR
    const int *perm;
    double dt;
    float *feat;                // [m0][8]
    double *rowscale;           // [m0]
};

struct MlpArgs {
    int n;
    const int *idx;       // optional gather: row k uses entry idx[k]
    const float *X;       // raw features [.][8]
    const float *params;  // fp32 master weights
    float norm[MLP_NORM];
    // inference outputs (indexed like X; any may be null), each
    // max(0, X[2] + scale z), times rowscale[row] when given
    const double *rowscale;
    float *out32;
    double *out64;
    float *zout;
    // training
    const float *y;  // targets (converged multipliers, features' units; indexed like X)
    float scale2;    // 2 / n
    float *partial;  // one MLP_SLOT slot per 32-row tile
};

void launch_features(const FeatureArgs &a, hipStream_t s);
void launch_mlp_forward(const MlpArgs &a, hipStream_t s);
int mlp_slots(int n);
// gradient of the mean loss into grad[MLP_NPARAM], the mean loss into *loss
void launch_mlp_grad(const MlpArgs &a, float *grad, float *loss, hipStream_t s);
void launch_adam(float *p, const float *g, float *m, float *v, float lr, int t, hipStream_t s);
// copy out the rows of A_0: features, final multipliers, caller pair indices
// (targets in the features' units: gamma / rowscale)
void launch_log_rows(int m0, const float *feat, const double *gam, const double *rowscale, const int *ia,
                     const int *ib, const int *perm, float *out_feat, float *out_gam, int *out_ia, int *out_ib,
                     hipStream_t s);

}  // namespace relcp
