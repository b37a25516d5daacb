// geometry.h -- launch arguments of the geometry kernels (geometry.hip).
#pragma once

#include "common.h"
#include "lcp.h"

namespace relcp {

struct SnsdArgs {
    int m;                       // pairs
    const int *pa, *pb;          // pair bodies
    const int *body_batch;       // packing of each body (null: one packing)
    const double *x;             // positions, 3 comps
    int ldx;
    const double *geo;           // Sigma (6 comps) or axis (first 3 comps)
    int ldg;
    const int *kind;
    const double *p;             // shape parameters, 3 comps
    int ldp;
    const double *boxes;         // 3 per packing (device)
    int planar;
    const double *hint;          // previous normals (3 comps, ld = ldo) or null
    double *out;                 // 10 comps: Phi, n, r_a, r_b
    int ldo;
    int mode;                    // 0: flag = Phi <= thresh;  1: flag = Phi < -eps
    double thresh, eps;
    // bounding radii or null: a pair whose bounding spheres are more than
    // thresh (mode 0) or 0 (mode 1) apart cannot be flagged and skips the
    // Newton solve; it reports the sphere gap (a lower bound of Phi) and
    // the centre-to-centre normal
    const double *Rb;
    int *flag;                   // per pair, or null
    int *bcount;                 // set flags per block of 256 pairs (snsd_blocks(m) slots), or null
    double *clear;               // per pair, set to 0 (a per-pair accumulator for later), or null
    // with clear: per pair a row (or -1) whose init_gam value clear starts
    // from instead of 0, or null
    const int *init_row;
    const double *init_gam;
    // per-block order keys of min Phi and min |Phi + eps| (snsd_blocks(m)
    // slots each), or null
    unsigned long long *minphi;
    unsigned long long *minmarg;
    // 2: every body is a torus, so the launch may use the kernel built for
    // tori alone (no ellipsoid or spherocylinder code to share registers
    // with); anything else: the kernel for every kind
    int only_kind = -1;
};

struct BodySetupArgs {
    int nb;
    const double *q;
    int ldq;
    const int *kind;
    const double *p;
    int ldp;
    const double *rho_xi;
    const double *u;  // 6 comps (inertial U^k) or null
    int ldu;
    const double *fext;  // 6 comps or null
    int ldf;
    int dynamics, planar;
    double dt;
    double *geo;
    int ldg;
    double *Rb;
    double *K;  // 9 comps (or null: geometry only)
    int ldk;
    float *K32;
    double *vfree;  // 6 comps
    int ldv;
};

void launch_body_setup(const BodySetupArgs &a, hipStream_t s);
int snsd_blocks(int m);
// maxdisp: trial_blocks(nb) slots, each the bits of its block's largest
// surface-point displacement bound
int trial_blocks(int nb);
// R, Bd (or null): the FP64 rows with their multipliers and the incidence
// lists; then the contact velocities vc = K D max(0, gamma) are formed here
// (and stored to Bd->vc unless it is null) instead of read from vc.  vfree
// null: U_free is zero (not read).
void launch_trial(int nb, const double *x, int ldx, const double *q, int ldq, const double *vfree, const double *vc,
                  int ldv, double dt, const int *kind, const double *p, int ldp, const double *Rb, double *xt,
                  double *qt, double *geo, int ldg, double *vout, unsigned long long *maxdisp, hipStream_t s,
                  const RowsT<double> *R = nullptr, const BodiesT<double> *Bd = nullptr);
void launch_snsd_pairs(const SnsdArgs &a, hipStream_t s);
void launch_cell_assign(int nb, const double *x, int ldx, const int *body_batch, const PackGrid *grids,
                        int *body_cell, int *cell_count, hipStream_t s);
void launch_cell_fill(int nb, const int *body_cell, const int *cell_start, int *cursor, int *items, hipStream_t s);
// Shapes for the candidate search's second test (all null: bounding spheres
// only): Sigma (6 comps) or axis (3), kind, shape parameters (3 comps).
struct PairShapes {
    const double *geo;
    int ldg;
    const int *kind;
    const double *p;
    int ldp;
};
// Candidate pairs: bounding spheres within skin; with shapes also the support
// gap along the centre line within skin (it bounds Phi from below, so a pair
// beyond it is farther than skin apart).
void launch_pairs(bool fill, int nb, const double *x, int ldx, const double *Rb, const int *body_batch,
                  const PackGrid *grids, const int *body_cell, const int *cell_start, const int *cell_count,
                  const int *items, double skin, int *pair_count, const int *pair_off, int *pa, int *pb, int cap,
                  hipStream_t s, const PairShapes *shapes = nullptr);

// host helpers of the order keys used by the min reductions
inline unsigned long long order_key_host(double v) {
    unsigned long long b;
    static_assert(sizeof(b) == sizeof(v), "");
    __builtin_memcpy(&b, &v, sizeof(v));
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
inline double order_key_value(unsigned long long k) {
    unsigned long long b = (k & 0x8000000000000000ull) ? (k & ~0x8000000000000000ull) : ~k;
    double v;
    __builtin_memcpy(&v, &b, sizeof(v));
    return v;
}

}  // namespace relcp
