/*
 * relcp_oracle.c -- plain FP64 CPU oracle for one ReLCP time-step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library, and the
 * GPU library never loads it.
 *
 * Paper: Palmer, Aktulga, Gao, "Smooth-Rigid-Body Contact as a ReLCP: a
 * recursively generated linear complementarity problem" (arXiv 2506.14097).
 * Every function names the passage it follows (section / equation /
 * algorithm).  Where the paper is silent the reading used is stated in the
 * comment; the GPU library takes the same readings.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA
 * contraction, so the arithmetic is exactly the order written here; OpenMP
 * only shares independent pairs among threads).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_OOM (-2)
#define ORC_E_LCP_MAXITER (-4)
#define ORC_E_RECURSION_CAP (-5)
#define ORC_E_SKIN (-6)
#define ORC_E_CAPACITY (-8)

#define ORC_MAXREC 64

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void matvec3(const double M[9], const double v[3], double out[3]) {
    for (int i = 0; i < 3; ++i)
        out[i] = M[3 * i + 0] * v[0] + M[3 * i + 1] * v[1] + M[3 * i + 2] * v[2];
}

/* Rotation matrix (row-major) of a unit quaternion q = [s, w] with scalar
 * part first (Sec. 2.1.1, nonsmooth generalized dynamics).  Column j is the
 * world direction of body axis j. */
void orc_quat_to_R(const double q[4], double R[9]) {
    double s = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - s * z);     R[2] = 2 * (x * z + s * y);
    R[3] = 2 * (x * y + s * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - s * x);
    R[6] = 2 * (x * z - s * y);     R[7] = 2 * (y * z + s * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Hamilton product a (x) b of scalar-first quaternions. */
static void quat_mul(const double a[4], const double b[4], double c[4]) {
    c[0] = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    c[1] = a[0] * b[1] + b[0] * a[1] + (a[2] * b[3] - a[3] * b[2]);
    c[2] = a[0] * b[2] + b[0] * a[2] + (a[3] * b[1] - a[1] * b[3]);
    c[3] = a[0] * b[3] + b[0] * a[3] + (a[1] * b[2] - a[2] * b[1]);
}

/* Configuration update C (+) dt*U for one body (Sec. 2.1.2, Eq. law_inertia /
 * Eq. law_overdamped: C^{k+1} = C^k + dt G^k U).  Reading: the orientation
 * is advanced by the exponential map of the world-frame rotation vector
 * theta = dt*omega, q' = exp(theta) (x) q, then renormalised; this agrees with
 * the linear map G^k to first order in dt, which is the order the paper
 * keeps.  Positions are exactly x + dt*u. */
void orc_integrate_body(const double x[3], const double q[4], const double v[6], double dt,
                        double xo[3], double qo[4]) {
    for (int i = 0; i < 3; ++i) xo[i] = x[i] + dt * v[i];
    double th[3] = {dt * v[3], dt * v[4], dt * v[5]};
    double a = norm3(th);
    double e[4];
    if (a < 1e-8) {
        /* series of cos(a/2) and sin(a/2)/a */
        e[0] = 1.0 - a * a / 8.0;
        double k = 0.5 * (1.0 - a * a / 24.0);
        e[1] = k * th[0]; e[2] = k * th[1]; e[3] = k * th[2];
    } else {
        e[0] = cos(0.5 * a);
        double k = sin(0.5 * a) / a;
        e[1] = k * th[0]; e[2] = k * th[1]; e[3] = k * th[2];
    }
    double r[4];
    quat_mul(e, q, r);
    double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int i = 0; i < 4; ++i) qo[i] = r[i] / nr;
}

/* ------------------------------------------------------------------------ */
/* Shared-normal signed distance (SNSD) of two ellipsoids                    */
/* ------------------------------------------------------------------------ */
/* Shape matrix Sigma = R diag(e^2) R^T of an ellipsoid with semiaxes e; its
 * support function is h(n) = sqrt(n^T Sigma n). */
void orc_ellipsoid_sigma(const double q[4], const double e[3], double S[9]) {
    double R[9];
    orc_quat_to_R(q, R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[3 * i + k] * (e[k] * e[k]) * R[3 * j + k];
            S[3 * i + j] = acc;
        }
}

/* Support gap f(n) = n.d - h_a(n) - h_b(n) for centre offset d = x_b - x_a. */
static double ell_gap(const double n[3], const double d[3], const double Sa[9], const double Sb[9]) {
    double sa[3], sb[3];
    matvec3(Sa, n, sa);
    matvec3(Sb, n, sb);
    return dot3(n, d) - sqrt(dot3(n, sa)) - sqrt(dot3(n, sb));
}

static void tangent_basis(const double n[3], double e1[3], double e2[3]) {
    double a[3] = {1.0, 0.0, 0.0};
    if (fabs(n[0]) > 0.9) { a[0] = 0.0; a[1] = 1.0; }
    double an = dot3(a, n);
    for (int i = 0; i < 3; ++i) e1[i] = a[i] - an * n[i];
    double l = norm3(e1);
    for (int i = 0; i < 3; ++i) e1[i] /= l;
    cross3(n, e1, e2);
}

/* Riemannian Newton ascent of f on the unit sphere, from n (updated in
 * place).  Gradient of f is p_b - p_a; stationarity on the sphere is the
 * shared-normal condition p_b - p_a = Phi n (Lemma uniform interior tangent
 * ball).  Returns the final f. */
static double ell_newton(double n[3], const double d[3], const double Sa[9], const double Sb[9],
                         int maxit) {
    double F = ell_gap(n, d, Sa, Sb);
    for (int it = 0; it < maxit; ++it) {
        double sa[3], sb[3];
        matvec3(Sa, n, sa);
        matvec3(Sb, n, sb);
        double ha = sqrt(dot3(n, sa)), hb = sqrt(dot3(n, sb));
        double E[3];
        for (int i = 0; i < 3; ++i) E[i] = d[i] - sa[i] / ha - sb[i] / hb;
        double nE = dot3(n, E);
        double e1[3], e2[3];
        tangent_basis(n, e1, e2);
        double g1 = dot3(e1, E), g2 = dot3(e2, E);
        double scale = norm3(d) + ha + hb;
        if (sqrt(g1 * g1 + g2 * g2) <= 1e-14 * scale) break;
        /* Euclidean Hessian of f: -(Sa/ha - sa sa^T/ha^3) - (same for b) */
        double H[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                H[3 * i + j] = -(Sa[3 * i + j] / ha - sa[i] * sa[j] / (ha * ha * ha))
                               - (Sb[3 * i + j] / hb - sb[i] * sb[j] / (hb * hb * hb));
        double He1[3], He2[3];
        matvec3(H, e1, He1);
        matvec3(H, e2, He2);
        double h11 = dot3(e1, He1) - nE, h12 = dot3(e1, He2), h22 = dot3(e2, He2) - nE;
        double det = h11 * h22 - h12 * h12;
        double v1, v2;
        if (h11 < 0.0 && det > 0.0) {
            /* Newton: v = -H^{-1} g */
            v1 = -(h22 * g1 - h12 * g2) / det;
            v2 = -(-h12 * g1 + h11 * g2) / det;
        } else {
            /* not locally concave: gradient ascent, step bounded by 0.5 rad */
            double curv = fabs(h11) + fabs(h22) + 2.0 * fabs(h12) + 1e-300;
            double gn = sqrt(g1 * g1 + g2 * g2);
            double t = 1.0 / curv;
            if (t * gn > 0.5) t = 0.5 / gn;
            v1 = t * g1;
            v2 = t * g2;
        }
        double vn = sqrt(v1 * v1 + v2 * v2);
        if (vn > 0.5) { v1 *= 0.5 / vn; v2 *= 0.5 / vn; }
        double t = 1.0, Fn = F, nn[3];
        int ok = 0;
        for (int ls = 0; ls < 40; ++ls) {
            for (int i = 0; i < 3; ++i) nn[i] = n[i] + t * (v1 * e1[i] + v2 * e2[i]);
            double l = norm3(nn);
            for (int i = 0; i < 3; ++i) nn[i] /= l;
            Fn = ell_gap(nn, d, Sa, Sb);
            if (Fn >= F - 1e-15 * scale) { ok = 1; break; }
            t *= 0.5;
        }
        if (!ok) break;
        for (int i = 0; i < 3; ++i) n[i] = nn[i];
        F = Fn;
        if (t * sqrt(v1 * v1 + v2 * v2) < 1e-15) break;
    }
    return F;
}

/* SNSD of two ellipsoids (Sec. 2.1.4 proxy surfaces, Fig. surface
 * representation (a); ellipsoid test in Sec. 5.2).  Reading: the shared-
 * normal pair is the one that maximises the support gap
 *     Phi = max_{|n|=1}  n.d - h_a(n) - h_b(n),
 * which is the Euclidean distance when separated and minus the minimum
 * translation depth when overlapping (signed distance of d to the boundary of
 * A (+) (-B)).  The paper cites a common-normal method for this; the result
 * is defined by the maximisation, so any correct maximiser is acceptable.
 * Oracle method: the best `nsamp` Fibonacci-sphere directions seed Riemannian
 * Newton runs and the best converged value wins.
 * out = [Phi, n(3), r_a(3), r_b(3)] with r_a = p_a - x_a, r_b = p_b - x_b,
 * n pointing from a towards b. */
void orc_snsd_ellipsoid(const double d[3], const double qa[4], const double ea[3], const double qb[4],
                        const double eb[3], int nsamp, double out[10]) {
    double Sa[9], Sb[9];
    orc_ellipsoid_sigma(qa, ea, Sa);
    orc_ellipsoid_sigma(qb, eb, Sb);
    if (nsamp < 8) nsamp = 8;
    enum { TOP = 8 };
    double topF[TOP];
    double topn[TOP][3];
    for (int k = 0; k < TOP; ++k) topF[k] = -INFINITY;
    const double golden = M_PI * (3.0 - sqrt(5.0));
    for (int i = 0; i < nsamp; ++i) {
        double z = 1.0 - (2.0 * i + 1.0) / nsamp;
        double r = sqrt(fmax(0.0, 1.0 - z * z));
        double ph = golden * i;
        double n[3] = {r * cos(ph), r * sin(ph), z};
        double F = ell_gap(n, d, Sa, Sb);
        /* keep the TOP best samples (insertion into a sorted list) */
        if (F > topF[TOP - 1]) {
            int k = TOP - 1;
            while (k > 0 && topF[k - 1] < F) {
                topF[k] = topF[k - 1];
                memcpy(topn[k], topn[k - 1], sizeof(topn[k]));
                --k;
            }
            topF[k] = F;
            topn[k][0] = n[0]; topn[k][1] = n[1]; topn[k][2] = n[2];
        }
    }
    /* centre direction as an extra seed */
    double best = -INFINITY, bn[3] = {1, 0, 0};
    double dn = norm3(d);
    for (int k = 0; k <= TOP; ++k) {
        double n[3];
        if (k < TOP) {
            n[0] = topn[k][0]; n[1] = topn[k][1]; n[2] = topn[k][2];
        } else {
            if (dn == 0.0) continue;
            n[0] = d[0] / dn; n[1] = d[1] / dn; n[2] = d[2] / dn;
        }
        double F = ell_newton(n, d, Sa, Sb, 100);
        if (F > best) { best = F; bn[0] = n[0]; bn[1] = n[1]; bn[2] = n[2]; }
    }
    double sa[3], sb[3];
    matvec3(Sa, bn, sa);
    matvec3(Sb, bn, sb);
    double ha = sqrt(dot3(bn, sa)), hb = sqrt(dot3(bn, sb));
    out[0] = best;
    for (int i = 0; i < 3; ++i) {
        out[1 + i] = bn[i];
        out[4 + i] = sa[i] / ha;  /* p_a - x_a: support point of A in direction n */
        out[7 + i] = -sb[i] / hb; /* p_b - x_b: support point of B in direction -n */
    }
}

/* ------------------------------------------------------------------------ */
/* SNSD of two spherocylinders (Sec. 5.3): closest points of the two axis   */
/* segments, minus the cap radii.                                            */
/* ------------------------------------------------------------------------ */
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Squared distance |d + u t_b - s t_a|^2 between segment points. */
static double seg_dist2(const double d[3], const double ta[3], const double tb[3], double s, double u) {
    double w[3];
    for (int i = 0; i < 3; ++i) w[i] = d[i] + u * tb[i] - s * ta[i];
    return dot3(w, w);
}

/* Axis segments A: x_a + s t_a, s in [-ha, ha];  B: x_b + u t_b, u in
 * [-hb, hb].  d = x_b - x_a.  The closest pair minimises a convex quadratic
 * over a rectangle: it is the interior stationary point if that lies inside,
 * else the best of the four edge minimisers.  Readings for the cases with no
 * unique closest pair (the paper allows any deterministic selection rule):
 *  - parallel axes (|t_a x t_b|^2 < 1e-12): s = midpoint of the overlap of B's
 *    projection onto A with [-ha, ha] (or the nearer end of A when they do
 *    not overlap), u = the clamped projection of that point onto B;
 *  - touching axes (|q - p| < 1e-12): n = t_a x t_b normalised, signed so
 *    that n.d >= 0; with parallel axes as well, n = the part of d normal to
 *    t_a, else the in-plane normal of t_a; in a monolayer (planar) the normal
 *    must stay in the plane, so there it is the in-plane normal of t_a,
 *    signed so that n.d >= 0.                                                */
void orc_snsd_spherocyl(const double d[3], const double ta[3], double la, double ra, const double tb[3],
                        double lb, double rb, int planar, double out[10]) {
    double ha = 0.5 * la, hb = 0.5 * lb;
    double c[3];
    cross3(ta, tb, c);
    double s, u;
    if (dot3(c, c) < 1e-12) {
        /* projection of B's end points onto A's axis: t_a.(d -/+ hb t_b) */
        double p0 = dot3(ta, d) - hb * dot3(ta, tb), p1 = dot3(ta, d) + hb * dot3(ta, tb);
        double lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        double olo = lo > -ha ? lo : -ha, ohi = hi < ha ? hi : ha;
        if (olo <= ohi) s = 0.5 * (olo + ohi);
        else s = (hi < -ha) ? -ha : ha;
        /* point on B closest to x_a + s t_a */
        double w[3];
        for (int i = 0; i < 3; ++i) w[i] = s * ta[i] - d[i];
        u = clampd(dot3(tb, w), -hb, hb);
    } else {
        double b = dot3(ta, tb), ea = dot3(ta, d), eb = dot3(tb, d);
        /* stationary point: s - b u = ea,  b s - u = eb */
        double den = 1.0 - b * b;
        double s0 = (ea - b * eb) / den;
        double u0 = (b * ea - eb) / den;
        double best = INFINITY;
        s = 0.0; u = 0.0;
        if (s0 >= -ha && s0 <= ha && u0 >= -hb && u0 <= hb) {
            best = seg_dist2(d, ta, tb, s0, u0);
            s = s0; u = u0;
        }
        /* the four edges, each a clamped 1-D minimisation */
        double sv[2] = {-ha, ha}, uv[2] = {-hb, hb};
        for (int k = 0; k < 2; ++k) {
            double ss = sv[k];
            double uu = clampd(ss * b - eb, -hb, hb); /* argmin_u |d + u tb - ss ta| */
            double v = seg_dist2(d, ta, tb, ss, uu);
            if (v < best) { best = v; s = ss; u = uu; }
        }
        for (int k = 0; k < 2; ++k) {
            double uu = uv[k];
            double ss = clampd(ea + uu * b, -ha, ha); /* argmin_s |d + uu tb - s ta| */
            double v = seg_dist2(d, ta, tb, ss, uu);
            if (v < best) { best = v; s = ss; u = uu; }
        }
    }
    double p[3], q[3], w[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = s * ta[i];          /* relative to x_a */
        q[i] = d[i] + u * tb[i];   /* relative to x_a */
        w[i] = q[i] - p[i];
    }
    double dist = norm3(w);
    double n[3];
    if (dist >= 1e-12) {
        for (int i = 0; i < 3; ++i) n[i] = w[i] / dist;
    } else {
        double cl = norm3(c);
        if (planar) {
            n[0] = -ta[1]; n[1] = ta[0]; n[2] = 0.0;
            double l = norm3(n);
            for (int i = 0; i < 3; ++i) n[i] /= l;
        } else if (cl * cl >= 1e-12) {
            for (int i = 0; i < 3; ++i) n[i] = c[i] / cl;
        } else {
            double dt = dot3(d, ta);
            for (int i = 0; i < 3; ++i) n[i] = d[i] - dt * ta[i];
            double l = norm3(n);
            if (l < 1e-12) { n[0] = -ta[1]; n[1] = ta[0]; n[2] = 0.0; l = norm3(n); }
            if (l < 1e-12) { n[0] = 0.0; n[1] = -ta[2]; n[2] = ta[1]; l = norm3(n); }
            for (int i = 0; i < 3; ++i) n[i] /= l;
        }
        if (dot3(n, d) < 0.0) for (int i = 0; i < 3; ++i) n[i] = -n[i];
    }
    out[0] = dist - ra - rb;
    for (int i = 0; i < 3; ++i) {
        out[1 + i] = n[i];
        out[4 + i] = p[i] + ra * n[i];              /* p_a - x_a */
        out[7 + i] = (q[i] - d[i]) - rb * n[i];     /* p_b - x_b */
    }
}

/* ------------------------------------------------------------------------ */
/* SNSD of two tori (Sec. 6, non-convex rings): the distance between the two */
/* centre circles, minus the two minor radii.  The paper minimises the       */
/* distance over the two circle angles; here the minimum over both angles is */
/* written as the minimum over the angle of circle a of the distance from    */
/* that point to circle b, which has a closed form, so only a 1-D search is  */
/* left: the circle of a is sampled at ORC_TORUS_NS equal steps, and each of */
/* the ORC_TORUS_K smallest sampled local minima is refined by golden-       */
/* section search inside its two neighbouring steps.                          */
/* Readings (the paper asks only for a deterministic selection rule where    */
/* the closest pair is not unique): the smallest refined value wins, the     */
/* earlier sample on ties; where the centre circles meet (distance below     */
/* 1e-12), n = t_a x t_b (tangents of the two circles there), or, with       */
/* parallel tangents, the axis of a; n is signed so that n.d >= 0.            */
/* ------------------------------------------------------------------------ */
#define ORC_TORUS_NS 4096
#define ORC_TORUS_K 8

/* Unit vectors u, v completing the unit axis e to a right-handed frame. */
static void plane_basis(const double e[3], double u[3], double v[3]) {
    double ax = fabs(e[0]), ay = fabs(e[1]), az = fabs(e[2]);
    double c[3] = {0.0, 0.0, 0.0};
    if (ax <= ay && ax <= az) c[0] = 1.0;
    else if (ay <= az) c[1] = 1.0;
    else c[2] = 1.0;
    cross3(e, c, u);
    double l = norm3(u);
    for (int i = 0; i < 3; ++i) u[i] /= l;
    cross3(e, u, v);
}

/* Closest point q of the circle (centre c, unit axis e, radius R) to the
 * point y; returns |y - q|^2 = h^2 + (rho - R)^2 with h the height of y over
 * the circle's plane and rho its distance from the axis.  On the axis every
 * point of the circle is closest; q is then taken along `fallback`. */
static double circle_closest(const double y[3], const double c[3], const double e[3], double R,
                             const double fallback[3], double q[3]) {
    double w[3], up[3];
    for (int i = 0; i < 3; ++i) w[i] = y[i] - c[i];
    double h = dot3(w, e);
    for (int i = 0; i < 3; ++i) up[i] = w[i] - h * e[i];
    double rho = norm3(up);
    if (q) {
        if (rho > 0.0) for (int i = 0; i < 3; ++i) q[i] = c[i] + R * up[i] / rho;
        else for (int i = 0; i < 3; ++i) q[i] = c[i] + R * fallback[i];
    }
    return h * h + (rho - R) * (rho - R);
}

typedef struct {
    double d[3], ea[3], ua[3], va[3], eb[3], ub[3];
    double Ra, Rb;
} torus_pair;

/* Point of circle a at angle t (relative to x_a) and its squared distance to
 * circle b (centre d). */
static void ring_point(const torus_pair *T, double t, double y[3]) {
    double ct = cos(t), st = sin(t);
    for (int i = 0; i < 3; ++i) y[i] = T->Ra * (ct * T->ua[i] + st * T->va[i]);
}
static double ring_gap2(const torus_pair *T, double t) {
    double y[3];
    ring_point(T, t, y);
    return circle_closest(y, T->d, T->eb, T->Rb, T->ub, NULL);
}

/* Derivative of ring_gap2 at t: by the envelope theorem it is
 * 2 (y - q).y'(t), q the closest point of circle b to y = ring_point(t). */
static double ring_gap2_dt(const torus_pair *T, double t) {
    double y[3], q[3], dy[3];
    ring_point(T, t, y);
    circle_closest(y, T->d, T->eb, T->Rb, T->ub, q);
    double ct = cos(t), st = sin(t);
    for (int i = 0; i < 3; ++i) dy[i] = T->Ra * (-st * T->ua[i] + ct * T->va[i]);
    double acc = 0.0;
    for (int i = 0; i < 3; ++i) acc += (y[i] - q[i]) * dy[i];
    return 2.0 * acc;
}

/* Golden-section search for the minimum of ring_gap2 on [lo, hi], then, as
 * golden section locates a minimum only to about the square root of the
 * rounding unit, bisection on the sign of the derivative in a small bracket
 * around it where the derivative goes from negative to positive (values
 * alone cannot tell points that close apart). */
static double golden_min(const torus_pair *T, double lo, double hi, double *tmin) {
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    double f1 = ring_gap2(T, x1), f2 = ring_gap2(T, x2);
    for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        if (f1 <= f2) {
            hi = x2; x2 = x1; f2 = f1;
            x1 = hi - g * (hi - lo); f1 = ring_gap2(T, x1);
        } else {
            lo = x1; x1 = x2; f1 = f2;
            x2 = lo + g * (hi - lo); f2 = ring_gap2(T, x2);
        }
    }
    double t = f1 <= f2 ? x1 : x2, ft = f1 <= f2 ? f1 : f2;
    double a = t - 1e-6, b = t + 1e-6;
    if (ring_gap2_dt(T, a) < 0.0 && ring_gap2_dt(T, b) > 0.0) {
        for (int it = 0; it < 100 && b - a > 0.0; ++it) {
            double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (ring_gap2_dt(T, mid) < 0.0) a = mid;
            else b = mid;
        }
        t = 0.5 * (a + b);
        ft = ring_gap2(T, t);
    }
    *tmin = t;
    return ft;
}

/* d = x_b - x_a; ea, eb unit axes; Ra, Rb major and ra, rb minor radii.
 * out = [Phi, n(3), p_a - x_a (3), p_b - x_b (3)].  second (if not NULL):
 * the smallest centre-circle distance among the other refined minima more
 * than three sample steps away (+inf if none): a margin of uniqueness. */
void orc_snsd_torus(const double d[3], const double ea[3], double Ra, double ra, const double eb[3], double Rb,
                    double rb, double out[10], double *second) {
    torus_pair T;
    for (int i = 0; i < 3; ++i) { T.d[i] = d[i]; T.ea[i] = ea[i]; T.eb[i] = eb[i]; }
    T.Ra = Ra;
    T.Rb = Rb;
    plane_basis(ea, T.ua, T.va);
    double vb[3];
    plane_basis(eb, T.ub, vb);
    const double step = 2.0 * M_PI / ORC_TORUS_NS;
    double *f = malloc(sizeof(double) * ORC_TORUS_NS); /* per call: pairs run on several threads */
    for (int i = 0; i < ORC_TORUS_NS; ++i) f[i] = ring_gap2(&T, step * i);
    /* the ORC_TORUS_K smallest sampled local minima, in sample order on ties */
    int idx[ORC_TORUS_K];
    int nk = 0;
    for (int i = 0; i < ORC_TORUS_NS; ++i) {
        double fp = f[(i + ORC_TORUS_NS - 1) % ORC_TORUS_NS], fn = f[(i + 1) % ORC_TORUS_NS];
        if (!(f[i] <= fp && f[i] <= fn)) continue;
        int pos = nk;
        while (pos > 0 && f[idx[pos - 1]] > f[i]) --pos;
        if (pos >= ORC_TORUS_K) continue;
        int last = nk < ORC_TORUS_K ? nk : ORC_TORUS_K - 1;
        for (int j = last; j > pos; --j) idx[j] = idx[j - 1];
        idx[pos] = i;
        if (nk < ORC_TORUS_K) ++nk;
    }
    double tk[ORC_TORUS_K], fk[ORC_TORUS_K];
    int best = 0;
    for (int k = 0; k < nk; ++k) {
        double t0 = step * idx[k];
        fk[k] = golden_min(&T, t0 - step, t0 + step, &tk[k]);
        if (fk[k] < fk[best]) best = k;
    }
    free(f);
    if (second) {
        double sv = INFINITY;
        for (int k = 0; k < nk; ++k) {
            int di = abs(idx[k] - idx[best]);
            if (di > ORC_TORUS_NS / 2) di = ORC_TORUS_NS - di;
            if (di > 3 && fk[k] < sv) sv = fk[k];
        }
        *second = isinf(sv) ? sv : sqrt(sv);
    }
    double pa[3], pb[3], w[3], n[3];
    ring_point(&T, tk[best], pa);
    circle_closest(pa, d, eb, Rb, T.ub, pb);
    for (int i = 0; i < 3; ++i) w[i] = pb[i] - pa[i];
    double dist = norm3(w);
    if (dist >= 1e-12) {
        for (int i = 0; i < 3; ++i) n[i] = w[i] / dist;
    } else {
        double tpa[3], tpb[3], rel[3];
        cross3(ea, pa, tpa);
        for (int i = 0; i < 3; ++i) rel[i] = pb[i] - d[i];
        cross3(eb, rel, tpb);
        cross3(tpa, tpb, n);
        double l = norm3(n);
        if (l * l < 1e-12 * (dot3(tpa, tpa) * dot3(tpb, tpb) + 1e-300)) {
            for (int i = 0; i < 3; ++i) n[i] = ea[i];
            l = 1.0;
        }
        for (int i = 0; i < 3; ++i) n[i] /= l;
        if (dot3(n, d) < 0.0) for (int i = 0; i < 3; ++i) n[i] = -n[i];
    }
    out[0] = dist - ra - rb;
    for (int i = 0; i < 3; ++i) {
        out[1 + i] = n[i];
        out[4 + i] = pa[i] + ra * n[i];            /* p_a - x_a */
        out[7 + i] = (pb[i] - d[i]) - rb * n[i];   /* p_b - x_b */
    }
}

/* ------------------------------------------------------------------------ */
/* Body geometry and the pair list                                           */
/* ------------------------------------------------------------------------ */
/* kind 0 = ellipsoid with semiaxes p = (a, b, c) along body axes x, y, z;
 * kind 1 = spherocylinder p = (r, l, 0): radius r, cylinder length l (caps
 * excluded), axis = body x axis;
 * kind 2 = torus p = (R, r, 0): major radius R (centre circle), minor radius
 * r (tube), symmetry axis = body z axis. */
static double bounding_radius(int kind, const double p[3]) {
    if (kind == 0) return fmax(p[0], fmax(p[1], p[2]));
    if (kind == 2) return p[0] + p[1];
    return 0.5 * p[1] + p[0];
}

static void min_image(const double xa[3], const double xb[3], const double box[3], double d[3]) {
    for (int i = 0; i < 3; ++i) {
        d[i] = xb[i] - xa[i];
        if (box[i] > 0.0) d[i] -= box[i] * nearbyint(d[i] / box[i]);
    }
}

/* Candidate pairs ("near-contacting pairs", Sec. 3.1 iteration 0, Alg. 1):
 * every a < b whose bounding spheres are within `skin`, by brute force over
 * all pairs.  Returns the count (pairs written up to cap). */
int64_t orc_broadphase(int n, const double *x, const int *kind, const double *shape, const double box[3],
                       double skin, int64_t cap, int *pa, int *pb) {
    int64_t m = 0;
    for (int a = 0; a < n; ++a) {
        double Ra = bounding_radius(kind[a], shape + 3 * a);
        for (int b = a + 1; b < n; ++b) {
            double Rb = bounding_radius(kind[b], shape + 3 * b);
            double d[3];
            min_image(x + 3 * a, x + 3 * b, box, d);
            if (norm3(d) - Ra - Rb <= skin) {
                if (m < cap) { pa[m] = a; pb[m] = b; }
                ++m;
            }
        }
    }
    return m;
}

/* The same pairs, in the same order, found through a uniform grid of cells
 * (for large n; the step uses it above ORC_CELLS_FROM bodies).  A pair whose
 * bounding-sphere gap is <= skin has its centres (minimum image) within
 * h = 2 R_max + skin of each other, so with cells at least h wide its bodies
 * sit in the same or neighbouring cells along every direction.  Each
 * neighbouring cell is visited once even where a periodic direction has
 * fewer than three cells; the test applied to each candidate is the one of
 * orc_broadphase, and every body's partners are sorted, so the list is
 * identical to the all-pairs search. */
#define ORC_CELLS_FROM 4096

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

int64_t orc_broadphase_cells(int n, const double *x, const int *kind, const double *shape, const double box[3],
                             double skin, int64_t cap, int *pa, int *pb) {
    if (n <= 0) return 0;
    double Rmax = 0.0;
    for (int a = 0; a < n; ++a) Rmax = fmax(Rmax, bounding_radius(kind[a], shape + 3 * a));
    const double h = (2.0 * Rmax + skin) * (1.0 + 1e-9);
    double lo[3], w[3], ext[3];
    int nc[3];
    for (int k = 0; k < 3; ++k) {
        if (box[k] > 0.0) {
            lo[k] = 0.0;
            ext[k] = box[k];
            nc[k] = (int)floor(box[k] / h);
            if (nc[k] < 1) nc[k] = 1;
            w[k] = box[k] / nc[k];
        } else {
            double mn = INFINITY, mx = -INFINITY;
            for (int a = 0; a < n; ++a) { mn = fmin(mn, x[3 * a + k]); mx = fmax(mx, x[3 * a + k]); }
            lo[k] = mn;
            ext[k] = mx - mn;
            w[k] = h;
            nc[k] = (int)floor(ext[k] / w[k]) + 1;
        }
    }
    /* open directions: wider cells where the bodies are sparse */
    for (;;) {
        if ((double)nc[0] * nc[1] * nc[2] <= 8.0 * n + 64.0) break;
        int widened = 0;
        for (int k = 0; k < 3; ++k)
            if (!(box[k] > 0.0) && nc[k] > 1) {
                w[k] *= 2.0;
                nc[k] = (int)floor(ext[k] / w[k]) + 1;
                widened = 1;
            }
        if (!widened) break;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int *cell = malloc(sizeof(int) * (size_t)n);
    int *start = calloc((size_t)ncell + 1, sizeof(int));
    int *items = malloc(sizeof(int) * (size_t)n);
    int *cand = malloc(sizeof(int) * (size_t)n);
    int (*cc)[3] = malloc(sizeof(int[3]) * (size_t)n);
    for (int a = 0; a < n; ++a) {
        int64_t id = 0;
        for (int k = 0; k < 3; ++k) {
            double v = x[3 * a + k] - lo[k];
            if (box[k] > 0.0) v -= box[k] * floor(v / box[k]);
            int c = (int)floor(v / w[k]);
            if (c < 0) c = 0;
            if (c >= nc[k]) c = nc[k] - 1;
            cc[a][k] = c;
            id = id * nc[k] + c;
        }
        cell[a] = (int)id;
        start[id + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int *cur = malloc(sizeof(int) * (size_t)(ncell + 1));
        memcpy(cur, start, sizeof(int) * (size_t)(ncell + 1));
        for (int a = 0; a < n; ++a) items[cur[cell[a]]++] = a;
        free(cur);
    }
    int64_t m = 0;
    for (int a = 0; a < n; ++a) {
        const double Ra = bounding_radius(kind[a], shape + 3 * a);
        /* distinct neighbouring cell indices along each direction */
        int nb[3][3], cnt[3];
        for (int k = 0; k < 3; ++k) {
            cnt[k] = 0;
            for (int o = -1; o <= 1; ++o) {
                int c = cc[a][k] + o;
                if (box[k] > 0.0) c = (c % nc[k] + nc[k]) % nc[k];
                else if (c < 0 || c >= nc[k]) continue;
                int seen = 0;
                for (int t = 0; t < cnt[k]; ++t) seen |= nb[k][t] == c;
                if (!seen) nb[k][cnt[k]++] = c;
            }
        }
        int nck = 0;
        for (int i0 = 0; i0 < cnt[0]; ++i0)
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i2 = 0; i2 < cnt[2]; ++i2) {
                    int64_t id = ((int64_t)nb[0][i0] * nc[1] + nb[1][i1]) * nc[2] + nb[2][i2];
                    for (int t = start[id]; t < start[id + 1]; ++t) {
                        int b = items[t];
                        if (b <= a) continue;
                        double Rb = bounding_radius(kind[b], shape + 3 * b);
                        double d[3];
                        min_image(x + 3 * a, x + 3 * b, box, d);
                        if (norm3(d) - Ra - Rb <= skin) cand[nck++] = b;
                    }
                }
        qsort(cand, (size_t)nck, sizeof(int), cmp_int);
        for (int t = 0; t < nck; ++t) {
            if (m < cap) { pa[m] = a; pb[m] = cand[t]; }
            ++m;
        }
    }
    free(cell); free(start); free(items); free(cand); free(cc);
    return m;
}

/* SNSD of one pair at a configuration (x, q). */
static void pair_snsd(int a, int b, const double *x, const double *q, const int *kind, const double *shape,
                      const double box[3], int planar, double out[10]) {
    double d[3];
    min_image(x + 3 * a, x + 3 * b, box, d);
    if (kind[a] == 0) {
        orc_snsd_ellipsoid(d, q + 4 * a, shape + 3 * a, q + 4 * b, shape + 3 * b, 2000, out);
    } else if (kind[a] == 2) {
        double Ra[9], Rb[9];
        orc_quat_to_R(q + 4 * a, Ra);
        orc_quat_to_R(q + 4 * b, Rb);
        double ea[3] = {Ra[2], Ra[5], Ra[8]}, eb[3] = {Rb[2], Rb[5], Rb[8]};
        orc_snsd_torus(d, ea, shape[3 * a + 0], shape[3 * a + 1], eb, shape[3 * b + 0], shape[3 * b + 1], out,
                       NULL);
    } else {
        double Ra[9], Rb[9];
        orc_quat_to_R(q + 4 * a, Ra);
        orc_quat_to_R(q + 4 * b, Rb);
        double ta[3] = {Ra[0], Ra[3], Ra[6]}, tb[3] = {Rb[0], Rb[3], Rb[6]};
        orc_snsd_spherocyl(d, ta, shape[3 * a + 1], shape[3 * a + 0], tb, shape[3 * b + 1], shape[3 * b + 0],
                           planar, out);
    }
}

/* SNSD of a list of pairs (used by the tests and by the step).  Pairs are
 * independent, so they are shared among OpenMP threads; every pair's
 * arithmetic is the same whatever the thread count. */
void orc_snsd_pairs(int m, const int *pa, const int *pb, const double *x, const double *q, const int *kind,
                    const double *shape, const double box[3], int planar, double *out /* 10*m */) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int k = 0; k < m; ++k) pair_snsd(pa[k], pb[k], x, q, kind, shape, box, planar, out + 10 * k);
}

/* ------------------------------------------------------------------------ */
/* Laws of motion: the operator K and the free velocity                     */
/* ------------------------------------------------------------------------ */
/* Per body: translational diagonal kt[3] and rotational symmetric Kr[9] with
 *   U = U_free + K F  (both laws in the form used by the LCP):
 *  - overdamped, local drag (Sec. 2.1.2 Eq. law_overdamped; Eq.
 *    ellipsoid_mobility): K = M = (1/xi) diag(I/L, 12 I/L^3); L = 2 x major
 *    semiaxis for ellipsoids; reading for spherocylinders: L = l + 2r (tip to
 *    tip); for tori: L = 2 (R + r) (outer diameter); U_free = M F_ext.
 *  - inertial (Sec. 2.1.2 Eq. law_inertia, Eq. cqpp): K = dt M^{-1} with
 *    M^{-1} = diag(I/m, R diag(1/I_body) R^T) of a solid ellipsoid of density
 *    rho; U_free = U^k + dt M^{-1} F_ext.
 * Planar (monolayer) systems keep only in-plane translation and rotation
 * about z: K -> P K P with P = diag(1,1,0 | 0,0,1). */
static int body_K(int dynamics, int planar, double dt, int kind, const double p[3], const double q[4],
                  double rho_xi, double kt[3], double Kr[9]) {
    memset(Kr, 0, 9 * sizeof(double));
    if (dynamics == 0) {
        double L = (kind == 0) ? 2.0 * fmax(p[0], fmax(p[1], p[2]))
                 : (kind == 2 ? 2.0 * (p[0] + p[1]) : p[1] + 2.0 * p[0]);
        double xi = rho_xi;
        if (!(L > 0.0) || !(xi > 0.0)) return ORC_E_INVALID;
        double a = 1.0 / (xi * L), r = 12.0 / (xi * L * L * L);
        kt[0] = kt[1] = kt[2] = a;
        Kr[0] = Kr[4] = Kr[8] = r;
    } else {
        if (kind != 0) return ORC_E_INVALID;
        double A = p[0], B = p[1], C = p[2];
        double m = rho_xi * 4.0 / 3.0 * M_PI * A * B * C;
        double I[3] = {m * (B * B + C * C) / 5.0, m * (A * A + C * C) / 5.0, m * (A * A + B * B) / 5.0};
        kt[0] = kt[1] = kt[2] = dt / m;
        double R[9];
        orc_quat_to_R(q, R);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * i + k] * (1.0 / I[k]) * R[3 * j + k];
                Kr[3 * i + j] = dt * acc;
            }
    }
    if (planar) {
        kt[2] = 0.0;
        double kzz = Kr[8];
        memset(Kr, 0, 9 * sizeof(double));
        Kr[8] = kzz;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Constraint rows and the operators D gamma, D^T V                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int ia, ib, pair, rec;
    double n[3], ta[3], tb[3]; /* n, r_a x n, r_b x n */
    double phi;                /* true signed separation where the row was generated */
    double c;                  /* per-row constant of the closed form */
} orow;

/* Row alpha of D^T acting on the velocity (Sec. 2.1.5, linearized separation
 * rate; rigid wrench form in the proof of Thm. is_a_relcp):
 *   D_alpha^T U = -n.u_a - (r_a x n).w_a + n.u_b + (r_b x n).w_b            */
static double row_rate(const orow *r, const double *V) {
    const double *va = V + 6 * r->ia, *vb = V + 6 * r->ib;
    return -dot3(r->n, va) - dot3(r->ta, va + 3) + dot3(r->n, vb) + dot3(r->tb, vb + 3);
}

/* Wrench D gamma (Eq. collision_ft): body a receives (-n, -r_a x n) gamma and
 * body b receives (+n, +r_b x n) gamma. */
static void scatter(int n, int m, const orow *rows, const double *gam, double *W) {
    memset(W, 0, 6 * (size_t)n * sizeof(double));
    for (int k = 0; k < m; ++k) {
        const orow *r = rows + k;
        double g = gam[k];
        for (int i = 0; i < 3; ++i) {
            W[6 * r->ia + i] -= r->n[i] * g;
            W[6 * r->ia + 3 + i] -= r->ta[i] * g;
            W[6 * r->ib + i] += r->n[i] * g;
            W[6 * r->ib + 3 + i] += r->tb[i] * g;
        }
    }
}

/* U = U_free + K W */
static void apply_K(int n, const double *kt, const double *Kr, const double *Ufree, const double *W, double *U) {
    for (int b = 0; b < n; ++b) {
        const double *w = W + 6 * b;
        for (int i = 0; i < 3; ++i) U[6 * b + i] = Ufree[6 * b + i] + kt[3 * b + i] * w[i];
        double t[3];
        matvec3(Kr + 9 * b, w + 3, t);
        for (int i = 0; i < 3; ++i) U[6 * b + 3 + i] = Ufree[6 * b + 3 + i] + t[i];
    }
}

/* The LCP of one recursion, in the form 0 <= A gamma + qv  _|_  gamma >= 0
 * with A = dt D^T K D applied matrix-free (Eq. relcp; Eq. cqpp). */
typedef struct {
    int n, m;
    const orow *rows;
    const double *kt, *Kr;
    double dt;
    double *W, *U, *zero; /* work: 6n each */
} lcp_op;

/* Diagonal entry A_kk = dt D_k^T K D_k of one row. */
static double row_diag(const orow *r, const double *kt, const double *Kr, double dt) {
    double t1[3], t2[3], acc = 0.0;
    for (int i = 0; i < 3; ++i) acc += r->n[i] * kt[3 * r->ia + i] * r->n[i] + r->n[i] * kt[3 * r->ib + i] * r->n[i];
    matvec3(Kr + 9 * r->ia, r->ta, t1);
    matvec3(Kr + 9 * r->ib, r->tb, t2);
    acc += dot3(r->ta, t1) + dot3(r->tb, t2);
    return dt * acc;
}

static void op_apply(const lcp_op *op, const double *gam, double *out) {
    scatter(op->n, op->m, op->rows, gam, op->W);
    apply_K(op->n, op->kt, op->Kr, op->zero, op->W, op->U);
    for (int k = 0; k < op->m; ++k) out[k] = op->dt * row_rate(op->rows + k, op->U);
}

/* ------------------------------------------------------------------------ */
/* LCP solvers                                                               */
/* ------------------------------------------------------------------------ */
/* Symmetric eigen-decomposition by cyclic Jacobi rotations (textbook). */
static void jacobi_eig(int m, double *A, double *V, double *ev) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V[i * m + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) off += A[i * m + j] * A[i * m + j];
        if (off < 1e-300) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = A[p * m + q];
                if (fabs(apq) < 1e-300) continue;
                double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {
                    double akp = A[k * m + p], akq = A[k * m + q];
                    A[k * m + p] = c * akp - s * akq;
                    A[k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    double apk = A[p * m + k], aqk = A[q * m + k];
                    A[p * m + k] = c * apk - s * aqk;
                    A[q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    double vkp = V[k * m + p], vkq = V[k * m + q];
                    V[k * m + p] = c * vkp - s * vkq;
                    V[k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) ev[i] = A[i * m + i];
}

/* Exact LCP solve by enumerating complementary index sets (for m <= 12):
 * for every active set S (smallest first), gamma_S = -pinv(A_SS) qv_S,
 * gamma = 0 elsewhere; accept the first candidate with gamma >= 0, w = A gamma
 * + qv >= 0 and A_SS gamma_S = -qv_S (tolerance 1e-12 relative).  A is
 * dense m x m (row-major).  Returns 0 on success, -1 if none found. */
int orc_lcp_enumerate(int m, const double *A, const double *qv, double *gam) {
    if (m == 0) return 0;
    if (m > 16) return -1;
    double scaleA = 0.0, scaleq = 0.0;
    for (int i = 0; i < m * m; ++i) scaleA = fmax(scaleA, fabs(A[i]));
    for (int i = 0; i < m; ++i) scaleq = fmax(scaleq, fabs(qv[i]));
    double tolw = 1e-12 * (scaleq + 1e-300) + 1e-13 * scaleA;
    int idx[16];
    double As[256], V[256], ev[16], g[16], w[16], rhs[16], z[16];
    for (int size = 0; size <= m; ++size) {
        /* iterate subsets of the given size in lexicographic order */
        for (int mask = 0; mask < (1 << m); ++mask) {
            if (__builtin_popcount((unsigned)mask) != size) continue;
            int k = 0;
            for (int i = 0; i < m; ++i)
                if (mask & (1 << i)) idx[k++] = i;
            for (int i = 0; i < m; ++i) g[i] = 0.0;
            if (k > 0) {
                for (int i = 0; i < k; ++i)
                    for (int j = 0; j < k; ++j) As[i * k + j] = A[idx[i] * m + idx[j]];
                jacobi_eig(k, As, V, ev);
                double evmax = 0.0;
                for (int i = 0; i < k; ++i) evmax = fmax(evmax, fabs(ev[i]));
                for (int i = 0; i < k; ++i) rhs[i] = -qv[idx[i]];
                /* z = V^T rhs / ev (pseudo-inverse), gamma_S = V z */
                for (int i = 0; i < k; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < k; ++j) acc += V[j * k + i] * rhs[j];
                    z[i] = (fabs(ev[i]) > 1e-11 * evmax && evmax > 0.0) ? acc / ev[i] : 0.0;
                }
                for (int i = 0; i < k; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < k; ++j) acc += V[i * k + j] * z[j];
                    g[idx[i]] = acc;
                }
            }
            int ok = 1;
            for (int i = 0; i < m && ok; ++i) {
                if (g[i] < -1e-13 * (1.0 + fabs(g[i]))) ok = 0;
            }
            if (!ok) continue;
            double gmax = 0.0;
            for (int i = 0; i < m; ++i) gmax = fmax(gmax, fabs(g[i]));
            for (int i = 0; i < m; ++i) {
                double acc = qv[i];
                for (int j = 0; j < m; ++j) acc += A[i * m + j] * g[j];
                w[i] = acc;
            }
            double tw = tolw + 1e-12 * scaleA * gmax;
            for (int i = 0; i < m && ok; ++i) {
                if (mask & (1 << i)) { if (fabs(w[i]) > tw) ok = 0; }
                else if (w[i] < -tw) ok = 0;
            }
            if (!ok) continue;
            for (int i = 0; i < m; ++i) gam[i] = g[i] > 0.0 ? g[i] : 0.0;
            return 0;
        }
    }
    return -1;
}

/* Scaled natural residual max_a |min(A_aa gamma_a, w_a)| (length units). */
static double natural_residual(int m, const double *dA, const double *gam, const double *w) {
    double r = 0.0;
    for (int k = 0; k < m; ++k) {
        double a = dA[k] * gam[k], b = w[k];
        double v = fabs(a < b ? a : b);
        if (v > r) r = v;
    }
    return r;
}

/* Projected gradient with Barzilai-Borwein steps (one of the CQP solvers the
 * paper lists in Sec. 2.1.4 after Eq. cqpp; the paper does not say which it
 * used).  Jacobi-scaled, alternating BB1 / BB2 steps:
 *   gamma <- max(0, gamma - alpha w / A_diag),   s = dgamma, y = dw,
 *   even k: alpha = s^T D s / s^T y,   odd k: alpha = s^T y / y^T D^{-1} y
 * with D = diag(A), alpha_0 = 1, alpha kept when s^T y <= 0, clamped to
 * [1e-10, 1e10]; stop when the scaled natural residual <= tol.
 * Returns the number of iterations or -1 at max_iter. */
static int bb_pgd(const lcp_op *op, const double *qv, const double *dA, double *gam, double tol, int max_iter,
                  double *res_out) {
    int m = op->m;
    double *w = malloc(sizeof(double) * (m + 1));
    double *gn = malloc(sizeof(double) * (m + 1));
    double *wn = malloc(sizeof(double) * (m + 1));
    for (int k = 0; k < m; ++k) gam[k] = gam[k] > 0.0 ? gam[k] : 0.0;
    op_apply(op, gam, w);
    for (int k = 0; k < m; ++k) w[k] += qv[k];
    double res = natural_residual(m, dA, gam, w);
    double alpha = 1.0;
    int it = 0, status = 0;
    while (res > tol) {
        if (it >= max_iter) { status = -1; break; }
        for (int k = 0; k < m; ++k) {
            double v = gam[k] - alpha * w[k] / dA[k];
            gn[k] = v > 0.0 ? v : 0.0;
        }
        op_apply(op, gn, wn);
        for (int k = 0; k < m; ++k) wn[k] += qv[k];
        double ss = 0.0, sy = 0.0, yy = 0.0;
        for (int k = 0; k < m; ++k) {
            double s = gn[k] - gam[k], y = wn[k] - w[k];
            ss += dA[k] * s * s;
            sy += s * y;
            yy += y * y / dA[k];
        }
        for (int k = 0; k < m; ++k) { gam[k] = gn[k]; w[k] = wn[k]; }
        res = natural_residual(m, dA, gam, w);
        if (sy > 0.0) {
            double a = (it % 2 == 0) ? ss / sy : sy / yy;
            alpha = a < 1e-10 ? 1e-10 : (a > 1e10 ? 1e10 : a);
        }
        ++it;
    }
    free(w); free(gn); free(wn);
    if (res_out) *res_out = res;
    return status == 0 ? it : -1;
}

/* Standalone BB-PGD on explicit rows (for the pins and for GPU parity of the
 * solver in isolation).  rows given SoA: ia, ib, n(3m), ta(3m), tb(3m);
 * qv = constant vector. */
int orc_lcp_bbpgd_rows(int n, int m, const int *ia, const int *ib, const double *nrm, const double *ta,
                       const double *tb, const double *kt, const double *Kr, double dt, const double *qv,
                       double *gam, double tol, int max_iter, double *res_out) {
    orow *rows = calloc((size_t)m + 1, sizeof(orow));
    for (int k = 0; k < m; ++k) {
        rows[k].ia = ia[k]; rows[k].ib = ib[k];
        for (int i = 0; i < 3; ++i) {
            rows[k].n[i] = nrm[3 * k + i]; rows[k].ta[i] = ta[3 * k + i]; rows[k].tb[i] = tb[3 * k + i];
        }
    }
    double *work = calloc(18 * (size_t)n + 1, sizeof(double));
    lcp_op op = {n, m, rows, kt, Kr, dt, work, work + 6 * (size_t)n, work + 12 * (size_t)n};
    double *dA = malloc(sizeof(double) * (m + 1));
    double *e = calloc((size_t)m + 1, sizeof(double)), *col = malloc(sizeof(double) * (m + 1));
    for (int k = 0; k < m; ++k) {
        double v = row_diag(rows + k, kt, Kr, dt);
        dA[k] = v > 0.0 ? v : 1.0;
    }
    int it = bb_pgd(&op, qv, dA, gam, tol, max_iter, res_out);
    free(rows); free(work); free(dA); free(e); free(col);
    return it;
}

/* Dense A = dt D^T K D (for tests and the exact solver). */
static void dense_A(const lcp_op *op, double *A) {
    int m = op->m;
    double *e = calloc((size_t)m + 1, sizeof(double)), *col = malloc(sizeof(double) * (m + 1));
    for (int j = 0; j < m; ++j) {
        e[j] = 1.0;
        op_apply(op, e, col);
        for (int i = 0; i < m; ++i) A[i * m + j] = col[i];
        e[j] = 0.0;
    }
    free(e); free(col);
}

int orc_dense_A(int n, int m, const int *ia, const int *ib, const double *nrm, const double *ta, const double *tb,
                const double *kt, const double *Kr, double dt, double *A) {
    orow *rows = calloc((size_t)m + 1, sizeof(orow));
    for (int k = 0; k < m; ++k) {
        rows[k].ia = ia[k]; rows[k].ib = ib[k];
        for (int i = 0; i < 3; ++i) {
            rows[k].n[i] = nrm[3 * k + i]; rows[k].ta[i] = ta[3 * k + i]; rows[k].tb[i] = tb[3 * k + i];
        }
    }
    double *work = calloc(18 * (size_t)n + 1, sizeof(double));
    lcp_op op = {n, m, rows, kt, Kr, dt, work, work + 6 * (size_t)n, work + 12 * (size_t)n};
    dense_A(&op, A);
    free(rows); free(work);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One ReLCP time-step (Sec. 3.1, Alg. 1; inertial: Eq. relcp_inertial)      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dynamics;       /* 0 overdamped, 1 inertial */
    int planar;         /* 1: monolayer (z translation and x,y rotation frozen) */
    int max_recursions; /* cap on n; 0 reduces the step to the plain SNSD LCP */
    int lcp_mode;       /* 0: exact if N_C <= 12 else BB-PGD; 1: BB-PGD; 2: exact */
    int lcp_max_iters;
    int form;           /* 0: the paper's incremental form; 1: per-row constant form */
    double dt, eps, tol, skin;
} orc_params;

typedef struct {
    int status;
    int recursions;         /* n at acceptance */
    int n_pairs;            /* candidate pairs */
    int n_rows;             /* rows at acceptance */
    int n_contacts[ORC_MAXREC + 1];
    int n_new[ORC_MAXREC + 1];   /* violators found when checking trial n+1 */
    int lcp_iters[ORC_MAXREC + 1];
    double W[ORC_MAXREC + 1];    /* gamma_n^T A_n gamma_n */
    double margin[ORC_MAXREC + 1]; /* min over pairs of |Phi(C_{n+1}) + eps| */
    double residual;             /* scaled natural residual of the accepted LCP */
    double max_overlap;          /* max over pairs of -Phi at the accepted configuration */
    double max_disp;             /* max surface displacement bound of the accepted trial */
} orc_stats;

static int row_push(orow **rows, int *m, int *cap, const orow *r) {
    if (*m >= *cap) {
        int nc = *cap ? 2 * *cap : 64;
        orow *nr = realloc(*rows, (size_t)nc * sizeof(orow));
        if (!nr) return ORC_E_OOM;
        *rows = nr; *cap = nc;
    }
    (*rows)[(*m)++] = *r;
    return ORC_OK;
}

static void make_row(int a, int b, int pair, int rec, const double s[10], orow *r) {
    r->ia = a; r->ib = b; r->pair = pair; r->rec = rec;
    r->phi = s[0];
    for (int i = 0; i < 3; ++i) r->n[i] = s[1 + i];
    cross3(s + 4, s + 1, r->ta);
    cross3(s + 7, s + 1, r->tb);
    r->c = 0.0;
}

/* One overdamped (Alg. 1 / Eq. relcp) or inertial (Eq. relcp_inertial) step
 * for a single system.
 * Inputs: n bodies (x 3n, q 4n, u 6n or NULL = at rest), kind/shape/rho_xi,
 * periodic box (0 = open), external wrench fext (6n or NULL), warm start for
 * the iteration-0 rows from the previous step (n_prev pairs (prev_a, prev_b,
 * prev_lam), sorted by (a, b)).
 * Outputs: accepted configuration (x_out, q_out), accepted velocity U_out
 * (6n: V_n = U_free + K D_n gamma_n), rows (up to row_cap; arrays may be
 * NULL), stats.
 * Readings (the paper is silent): the near-contact set A_0 is every candidate
 * pair with Phi_0 <= skin; violators are pairs with Phi(C_{n+1}) < -eps
 * (strict; Eq. gap_stopping_rule), all of them each recursion (the default
 * implementation named in Cor. strictly-convex existence); a row keeps the
 * lever arms r_a, r_b of the configuration where it was generated; the step
 * fails with E_SKIN if a trial moves any surface point by more than skin/2
 * (the candidate list could then miss pairs), and with E_RECURSION_CAP after
 * max_recursions augmentations; on failure the inputs are untouched. */
int orc_relcp_step(int n, const double *x, const double *q, const double *u, const int *kind, const double *shape,
                   const double *rho_xi, const double box[3], const double *fext, int n_prev, const int *prev_a,
                   const int *prev_b, const double *prev_lam, const orc_params *P, double *x_out, double *q_out,
                   double *U_out, int row_cap, int *r_ia, int *r_ib, int *r_rec, int *r_pair, double *r_gamma,
                   double *r_phi, double *r_n, double *r_ta, double *r_tb, orc_stats *st) {
    memset(st, 0, sizeof(*st));
    const double dt = P->dt;
    int status = ORC_OK;
    double *kt = malloc(sizeof(double) * 3 * (size_t)n + 8);
    double *Kr = malloc(sizeof(double) * 9 * (size_t)n + 8);
    double *Ufree = calloc(6 * (size_t)n + 8, sizeof(double));
    double *work = calloc(18 * (size_t)n + 8, sizeof(double));
    double *Vn = calloc(6 * (size_t)n + 8, sizeof(double));
    double *xt = malloc(sizeof(double) * 3 * (size_t)n + 8);
    double *qt = malloc(sizeof(double) * 4 * (size_t)n + 8);
    double *Rb = malloc(sizeof(double) * (size_t)n + 8);
    orow *rows = NULL;
    int m = 0, rcap = 0;
    double *gam = NULL, *gprev = NULL, *phitil = NULL, *qv = NULL, *dA = NULL, *Ag = NULL;
    int *pa = NULL, *pb = NULL;
    double *snsd = NULL, *snsdt = NULL;

    /* K, U_free (Sec. 2.1.2) */
    for (int b = 0; b < n; ++b) {
        if (body_K(P->dynamics, P->planar, dt, kind[b], shape + 3 * b, q + 4 * b, rho_xi[b], kt + 3 * b,
                   Kr + 9 * b) != ORC_OK) { status = ORC_E_INVALID; goto done; }
        Rb[b] = bounding_radius(kind[b], shape + 3 * b);
    }
    {
        double *zero = work + 12 * (size_t)n;
        memset(zero, 0, 6 * (size_t)n * sizeof(double));
        double *U0 = calloc(6 * (size_t)n + 8, sizeof(double));
        if (P->dynamics == 1 && u) memcpy(U0, u, 6 * (size_t)n * sizeof(double));
        if (fext) apply_K(n, kt, Kr, U0, fext, Ufree);
        else memcpy(Ufree, U0, 6 * (size_t)n * sizeof(double));
        if (P->planar)
            for (int b = 0; b < n; ++b) { Ufree[6 * b + 2] = 0.0; Ufree[6 * b + 3] = 0.0; Ufree[6 * b + 4] = 0.0; }
        free(U0);
    }

    /* candidate pairs and SNSD at C^k (Alg. 1 initialisation) */
    int64_t (*search)(int, const double *, const int *, const double *, const double *, double, int64_t, int *,
                      int *) = n >= ORC_CELLS_FROM ? orc_broadphase_cells : orc_broadphase;
    int64_t np = search(n, x, kind, shape, box, P->skin, 0, NULL, NULL);
    pa = malloc(sizeof(int) * (size_t)(np + 1));
    pb = malloc(sizeof(int) * (size_t)(np + 1));
    search(n, x, kind, shape, box, P->skin, np, pa, pb);
    st->n_pairs = (int)np;
    snsd = malloc(sizeof(double) * 10 * (size_t)(np + 1));
    snsdt = malloc(sizeof(double) * 10 * (size_t)(np + 1));
    orc_snsd_pairs((int)np, pa, pb, x, q, kind, shape, box, P->planar, snsd);

    /* A_0: one row per near-contacting pair, Phi_0 <= skin */
    for (int64_t k = 0; k < np; ++k) {
        if (snsd[10 * k] <= P->skin) {
            orow r;
            make_row(pa[k], pb[k], (int)k, 0, snsd + 10 * k, &r);
            if (row_push(&rows, &m, &rcap, &r) != ORC_OK) { status = ORC_E_OOM; goto done; }
        }
    }

    lcp_op op = {n, 0, NULL, kt, Kr, dt, work, work + 6 * (size_t)n, work + 12 * (size_t)n};
    memset(work + 12 * (size_t)n, 0, 6 * (size_t)n * sizeof(double));

    /* Phi~_0 = Phi_0 + dt D^T U_free  (Alg. 1 initialisation; inertial form
     * after Eq. relcp_inertial uses U_free = U^k + dt M^{-1} F_ext) */
    int alloc = m + 16;
    gam = calloc((size_t)alloc, sizeof(double));
    gprev = calloc((size_t)alloc, sizeof(double));
    phitil = calloc((size_t)alloc, sizeof(double));
    qv = calloc((size_t)alloc, sizeof(double));
    dA = calloc((size_t)alloc, sizeof(double));
    Ag = calloc((size_t)alloc, sizeof(double));
    for (int k = 0; k < m; ++k) {
        phitil[k] = rows[k].phi + dt * row_rate(rows + k, Ufree);
        rows[k].c = rows[k].phi;
    }
    /* warm start of the iteration-0 rows: previous-step multiplier of the pair */
    for (int k = 0; k < m; ++k) {
        gam[k] = 0.0;
        int lo = 0, hi = n_prev - 1;
        while (lo <= hi) {
            int mid = (lo + hi) / 2;
            int ka = prev_a[mid], kb = prev_b[mid];
            if (ka == rows[k].ia && kb == rows[k].ib) { gam[k] = prev_lam[mid]; break; }
            if (ka < rows[k].ia || (ka == rows[k].ia && kb < rows[k].ib)) lo = mid + 1; else hi = mid - 1;
        }
    }
    int mprev = 0; /* size of gamma_{n-1} (0 at n = 0: iota of nothing) */

    for (int rec = 0;; ++rec) {
        op.m = m;
        op.rows = rows;
        /* LCP n: 0 <= Phi_{n+1} = Phi~_n + A_n (gamma_n - iota gamma_{n-1}) _|_ gamma_n >= 0
         * i.e. qv = Phi~_n - A_n iota(gamma_{n-1})                (Eq. relcp)
         * closed form: qv = c + dt D^T U_free                      (per-row constant) */
        for (int k = 0; k < m; ++k) gprev[k] = (k < mprev) ? gprev[k] : 0.0;
        if (P->form == 0) {
            op_apply(&op, gprev, Ag);
            for (int k = 0; k < m; ++k) qv[k] = phitil[k] - Ag[k];
        } else {
            for (int k = 0; k < m; ++k) qv[k] = rows[k].c + dt * row_rate(rows + k, Ufree);
        }
        for (int k = 0; k < m; ++k) {
            double v = row_diag(rows + k, kt, Kr, dt);
            dA[k] = v > 0.0 ? v : 1.0;
        }
        int iters = 0;
        double res = 0.0;
        int exact = (P->lcp_mode == 2) || (P->lcp_mode == 0 && m <= 12);
        if (m == 0) {
            iters = 0;
        } else if (exact) {
            double *A = malloc(sizeof(double) * (size_t)m * m);
            dense_A(&op, A);
            if (orc_lcp_enumerate(m, A, qv, gam) != 0) {
                /* fall back to the iterative solver at a tight tolerance */
                iters = bb_pgd(&op, qv, dA, gam, P->tol, P->lcp_max_iters, &res);
                if (iters < 0) { free(A); status = ORC_E_LCP_MAXITER; goto done; }
            }
            free(A);
        } else {
            iters = bb_pgd(&op, qv, dA, gam, P->tol, P->lcp_max_iters, &res);
            if (iters < 0) { status = ORC_E_LCP_MAXITER; goto done; }
        }
        /* residual and W_n = gamma^T A gamma */
        op_apply(&op, gam, Ag);
        double W = 0.0;
        for (int k = 0; k < m; ++k) { W += gam[k] * Ag[k]; Ag[k] += qv[k]; }
        st->residual = natural_residual(m, dA, gam, Ag);
        st->n_contacts[rec] = m;
        st->lcp_iters[rec] = iters;
        st->W[rec] = W;
        /* Phi_{n+1}: linearised separations of all current rows */
        if (P->form == 0)
            for (int k = 0; k < m; ++k) phitil[k] = Ag[k];

        /* V_n = U_free + K D_n gamma_n ; trial C_{n+1} = C^k (+) dt V_n */
        scatter(n, m, rows, gam, work);
        apply_K(n, kt, Kr, Ufree, work, Vn);
        double maxdisp = 0.0;
        for (int b = 0; b < n; ++b) {
            orc_integrate_body(x + 3 * b, q + 4 * b, Vn + 6 * b, dt, xt + 3 * b, qt + 4 * b);
            double dv = dt * norm3(Vn + 6 * b) + Rb[b] * dt * norm3(Vn + 6 * b + 3);
            if (dv > maxdisp) maxdisp = dv;
        }
        st->max_disp = maxdisp;
        if (maxdisp > 0.5 * P->skin) { status = ORC_E_SKIN; goto done; }

        /* check every candidate pair at C_{n+1} (Alg. 1 while-condition) */
        double minphi = INFINITY, margin = INFINITY;
        int nv = 0;
        int mold = m;
        orc_snsd_pairs((int)np, pa, pb, xt, qt, kind, shape, box, P->planar, snsdt);
        for (int64_t k = 0; k < np; ++k) {
            const double *s = snsdt + 10 * k;
            if (s[0] < minphi) minphi = s[0];
            double mg = fabs(s[0] + P->eps);
            if (mg < margin) margin = mg;
            if (s[0] < -P->eps) {
                ++nv;
                if (rec >= P->max_recursions) continue;
                /* new frozen-normal row generated at C_{n+1}, pulled back:
                 *   Phi~ entry = Phi(C_{n+1})                      (Eq. relcp)
                 *   c = Phi(C_{n+1}) - dt D_alpha^T V_n            (per-row form) */
                orow r;
                make_row(pa[k], pb[k], (int)k, rec + 1, s, &r);
                r.c = s[0] - dt * row_rate(&r, Vn);
                if (row_push(&rows, &m, &rcap, &r) != ORC_OK) { status = ORC_E_OOM; goto done; }
            }
        }
        st->margin[rec] = margin;
        st->n_new[rec] = nv;
        if (nv == 0) {
            st->recursions = rec;
            st->max_overlap = minphi < 0.0 ? -minphi : 0.0;
            break;
        }
        if (rec >= P->max_recursions) {
            if (P->max_recursions == 0) {
                /* plain SNSD LCP (no augmentation): accept the first trial */
                st->recursions = 0;
                st->max_overlap = minphi < 0.0 ? -minphi : 0.0;
                m = mold;
                break;
            }
            status = ORC_E_RECURSION_CAP; st->recursions = rec; goto done;
        }
        /* grow the vectors: Phi~_{n+1} = append(Phi_{n+1}, Phi(C_{n+1})|new);
         * gamma padded by iota */
        if (m > alloc) {
            alloc = 2 * m + 16;
            gam = realloc(gam, sizeof(double) * alloc);
            gprev = realloc(gprev, sizeof(double) * alloc);
            phitil = realloc(phitil, sizeof(double) * alloc);
            qv = realloc(qv, sizeof(double) * alloc);
            dA = realloc(dA, sizeof(double) * alloc);
            Ag = realloc(Ag, sizeof(double) * alloc);
        }
        for (int k = mold; k < m; ++k) { phitil[k] = rows[k].phi; gam[k] = 0.0; }
        for (int k = 0; k < mold; ++k) gprev[k] = gam[k];
        mprev = mold;
    }

    /* accept (Alg. 1 return) */
    memcpy(x_out, xt, sizeof(double) * 3 * (size_t)n);
    memcpy(q_out, qt, sizeof(double) * 4 * (size_t)n);
    if (U_out) memcpy(U_out, Vn, sizeof(double) * 6 * (size_t)n);
    st->n_rows = m;
    if (m > row_cap) { status = ORC_E_CAPACITY; goto done; }
    for (int k = 0; k < m; ++k) {
        if (r_ia) r_ia[k] = rows[k].ia;
        if (r_ib) r_ib[k] = rows[k].ib;
        if (r_rec) r_rec[k] = rows[k].rec;
        if (r_pair) r_pair[k] = rows[k].pair;
        if (r_gamma) r_gamma[k] = gam[k];
        if (r_phi) r_phi[k] = rows[k].phi;
        for (int i = 0; i < 3; ++i) {
            if (r_n) r_n[3 * k + i] = rows[k].n[i];
            if (r_ta) r_ta[3 * k + i] = rows[k].ta[i];
            if (r_tb) r_tb[3 * k + i] = rows[k].tb[i];
        }
    }

done:
    st->status = status;
    free(kt); free(Kr); free(Ufree); free(work); free(Vn); free(xt); free(qt); free(Rb);
    free(rows); free(gam); free(gprev); free(phitil); free(qv); free(dA); free(Ag);
    free(pa); free(pb); free(snsd); free(snsdt);
    return status;
}

/* OpenMP threads for the per-pair loops (n > 0 sets them); returns the
 * number in use. */
int orc_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* The body operator K for external callers (tests): kt 3n, Kr 9n. */
int orc_body_K(int n, int dynamics, int planar, double dt, const int *kind, const double *shape, const double *q,
               const double *rho_xi, double *kt, double *Kr) {
    for (int b = 0; b < n; ++b)
        if (body_K(dynamics, planar, dt, kind[b], shape + 3 * b, q + 4 * b, rho_xi[b], kt + 3 * b, Kr + 9 * b))
            return ORC_E_INVALID;
    return ORC_OK;
}

int orc_stats_size(void) { return (int)sizeof(orc_stats); }
int orc_params_size(void) { return (int)sizeof(orc_params); }
