// geometry.hip -- body set-up, trial integration, candidate pairs and the
// shared-normal signed distance (SNSD) narrowphase, all FP64.
//
// Paper: Palmer, Aktulga, Gao (arXiv 2506.14097).  SNSD: Sec. 2.1.4 and
// Fig. surface representation (a); stationarity p_b - p_a = Phi n: Lemma
// uniform interior tangent ball; ellipsoids Sec. 5.2, spherocylinders Sec.
// 5.3.  Laws of motion: Sec. 2.1.2 (Eq. law_inertia, Eq. law_overdamped, Eq.
// ellipsoid_mobility).
#include "geometry.h"
#include "scatter.h"

namespace relcp {

// ===========================================================================
// SNSD of two ellipsoids
// ===========================================================================
// The shared-normal pair is read as the maximiser of the support gap
//   f(n) = n.d - h_a(n) - h_b(n),  h(n) = sqrt(n^T Sigma n),  |n| = 1,
// d = x_b - x_a: the Euclidean distance when apart, minus the minimum
// translation depth when overlapping.  f is 1-homogeneous, so its gradient
// is p_b - p_a and a stationary point on the sphere is a shared normal.
// Maximised by a Riemannian Newton ascent with a gradient-ascent fallback
// where the projected Hessian is not negative definite.

__device__ inline double support_gap(d3 n, d3 d, const sym3 &A, const sym3 &B) {
    return dot(n, d) - sqrt(dot(n, mul(A, n))) - sqrt(dot(n, mul(B, n)));
}

// 1 / sqrt(q) for q in [1e-4, 1e4] (support radii squared, squared lengths
// of near-unit vectors): the hardware estimate (v_rsq_f64, relative error
// well under 1e-6) refined by two Newton steps y <- y + y (1 - q y^2) / 2,
// each of which squares the relative error, so the result is within a few
// ulp.  Cheaper than sqrt followed by a division.
__device__ inline double rsqrt_nr(double q) {
    double y = __builtin_amdgcn_rsq(q);
    double e = fma(-q * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-q * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

__device__ inline void tangent_frame(d3 n, d3 &e1, d3 &e2) {
    // cross with the coordinate axis least aligned with n (|e1|^2 >= 2/3)
    double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
    d3 a = (ax <= ay && ax <= az) ? mk(1, 0, 0) : ((ay <= az) ? mk(0, 1, 0) : mk(0, 0, 1));
    e1 = cross(n, a);
    e1 = rsqrt_nr(dot(e1, e1)) * e1;
    e2 = cross(n, e1);
}

// The support gap at a unit n with the pieces a Newton step reuses: A n,
// B n, the support radii h_a = sqrt(n.A n), h_b and their inverses.
struct GapEval {
    double F, ha, hb, ia, ib;
    d3 an, bn;
};
__device__ inline GapEval gap_eval(d3 n, d3 d, const sym3 &A, const sym3 &B) {
    GapEval g;
    g.an = mul(A, n);
    g.bn = mul(B, n);
    const double qa = dot(n, g.an), qb = dot(n, g.bn);
    g.ia = rsqrt_nr(qa);
    g.ib = rsqrt_nr(qb);
    g.ha = qa * g.ia;
    g.hb = qb * g.ib;
    g.F = dot(n, d) - g.ha - g.hb;
    return g;
}

__device__ double gap_newton(d3 &n, d3 d, const sym3 &A, const sym3 &B, int maxit) {
    GapEval G = gap_eval(n, d, A, B);
    const double dl = len(d);
    for (int it = 0; it < maxit; ++it) {
        const d3 an = G.an, bn = G.bn;
        const double ha = G.ha, hb = G.hb;
        const double ia = G.ia, ib = G.ib;
        d3 grad = d - ia * an - ib * bn;  // p_b - p_a
        double fn = dot(n, grad);
        d3 e1, e2;
        tangent_frame(n, e1, e2);
        double g1 = dot(e1, grad), g2 = dot(e2, grad);
        double scale = dl + ha + hb;
        double gn2 = g1 * g1 + g2 * g2;
        // Phi is stationary at the maximiser: a tangential gradient of 1e-11
        // of the scale leaves the normal good to ~1e-11 and Phi to ~1e-22
        if (gn2 <= 1e-22 * scale * scale) break;
        // projected Hessian of f on the sphere: P (Hess f) P - (n.grad f) P
        d3 Ae1 = mul(A, e1), Ae2 = mul(A, e2), Be1 = mul(B, e1), Be2 = mul(B, e2);
        double ia3 = ia * ia * ia, ib3 = ib * ib * ib;
        double a1 = dot(e1, an), a2 = dot(e2, an), b1 = dot(e1, bn), b2 = dot(e2, bn);
        double h11 = -(dot(e1, Ae1) * ia - a1 * a1 * ia3) - (dot(e1, Be1) * ib - b1 * b1 * ib3) - fn;
        double h12 = -(dot(e1, Ae2) * ia - a1 * a2 * ia3) - (dot(e1, Be2) * ib - b1 * b2 * ib3);
        double h22 = -(dot(e2, Ae2) * ia - a2 * a2 * ia3) - (dot(e2, Be2) * ib - b2 * b2 * ib3) - fn;
        double det = h11 * h22 - h12 * h12;
        double v1, v2;
        if (h11 < 0.0 && det > 0.0) {
            const double idet = 1.0 / det;
            v1 = (-h22 * g1 + h12 * g2) * idet;
            v2 = (h12 * g1 - h11 * g2) * idet;
        } else {
            const double gnorm = sqrt(gn2);
            double curv = fabs(h11) + fabs(h22) + 2.0 * fabs(h12) + 1e-300;
            double t = 1.0 / curv;
            if (t * gnorm > 0.5) t = 0.5 / gnorm;
            v1 = t * g1;
            v2 = t * g2;
        }
        double vl2 = v1 * v1 + v2 * v2;
        if (vl2 > 0.25) {
            const double f = 0.5 / sqrt(vl2);
            v1 *= f;
            v2 *= f;
            vl2 = 0.25;
        }
        double t = 1.0;
        bool ok = false;
        for (int ls = 0; ls < 40; ++ls) {
            d3 c = n + t * (v1 * e1 + v2 * e2);
            c = rsqrt_nr(dot(c, c)) * c;
            const GapEval Gc = gap_eval(c, d, A, B);
            if (Gc.F >= G.F - 1e-15 * scale) {
                n = c;
                G = Gc;
                ok = true;
                break;
            }
            t *= 0.5;
        }
        if (!ok) break;
        if (t * t * vl2 < 1e-30) break;
    }
    return G.F;
}

// Result: Phi, n (a -> b), r_a = p_a - x_a, r_b = p_b - x_b.
struct Snsd {
    double phi;
    d3 n, ra, rb;
};

__device__ Snsd snsd_ellipsoid(d3 d, const sym3 &A, const sym3 &B, d3 hint, bool has_hint) {
    double dl = len(d);
    d3 n0 = dl > 0.0 ? (1.0 / dl) * d : mk(1, 0, 0);
    // A hint (the normal of the same pair a moment earlier) is tried first;
    // if it converges to a separated or shallow configuration, where the
    // maximiser is unique, the centre-line start would reach the same point.
    d3 best_n = has_hint ? hint : n0;
    double best = gap_newton(best_n, d, A, B, 60);
    double ha = sqrt(dot(best_n, mul(A, best_n))), hb = sqrt(dot(best_n, mul(B, best_n)));
    if (has_hint && best < -0.05 * (ha + hb)) {
        d3 n1 = n0;
        double F1 = gap_newton(n1, d, A, B, 60);
        if (F1 > best) {
            best = F1;
            best_n = n1;
        }
        ha = sqrt(dot(best_n, mul(A, best_n)));
        hb = sqrt(dot(best_n, mul(B, best_n)));
    }
    // deep overlap: several local maxima are possible; seed from a coarse
    // Fibonacci sphere and keep the best converged value
    if (best < -0.05 * (ha + hb) || dl == 0.0) {
        const int ns = 64;
        double bs = -1e300;
        d3 bsn = n0;
        for (int i = 0; i < ns; ++i) {
            double z = 1.0 - (2.0 * i + 1.0) / ns;
            double r = sqrt(fmax(0.0, 1.0 - z * z));
            double ph = 2.399963229728653 * i;
            d3 c = mk(r * cos(ph), r * sin(ph), z);
            double Fc = support_gap(c, d, A, B);
            if (Fc > bs) {
                bs = Fc;
                bsn = c;
            }
        }
        double F2 = gap_newton(bsn, d, A, B, 60);
        if (F2 > best) {
            best = F2;
            best_n = bsn;
        }
    }
    d3 an = mul(A, best_n), bn = mul(B, best_n);
    Snsd o;
    o.phi = best;
    o.n = best_n;
    o.ra = rsqrt_nr(dot(best_n, an)) * an;
    o.rb = (-rsqrt_nr(dot(best_n, bn))) * bn;
    return o;
}

// ===========================================================================
// SNSD of two spherocylinders: closest points of the axis segments minus
// the cap radii (Sec. 5.3).  Readings for non-unique closest pairs:
// parallel axes (|t_a x t_b|^2 < 1e-12): midpoint of the overlap of B's
// projection onto A, else the nearer end of A; coincident axis points
// (|q - p| < 1e-12): normal t_a x t_b (in a monolayer: the in-plane normal
// of t_a), with parallel axes the part of d normal to t_a, signed n.d >= 0.
// ===========================================================================
__device__ inline double clampd(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

__device__ Snsd snsd_spherocyl(d3 d, d3 ta, double la, double ra, d3 tb, double lb, double rb, bool planar) {
    const double ha = 0.5 * la, hb = 0.5 * lb;
    const d3 c = cross(ta, tb);
    const double b = dot(ta, tb), ea = dot(ta, d), eb = dot(tb, d);
    double s, u;
    if (dot(c, c) < 1e-12) {
        double p0 = ea - hb * b, p1 = ea + hb * b;
        double lo = fmin(p0, p1), hi = fmax(p0, p1);
        double olo = fmax(lo, -ha), ohi = fmin(hi, ha);
        if (olo <= ohi)
            s = 0.5 * (olo + ohi);
        else
            s = (hi < -ha) ? -ha : ha;
        u = clampd(s * b - eb, -hb, hb);
    } else {
        // convex quadratic over a rectangle: interior stationary point, else
        // the best of the four clamped edge minimisers
        auto dist2 = [&](double ss, double uu) {
            d3 w = d + uu * tb - ss * ta;
            return dot(w, w);
        };
        double den = 1.0 - b * b;
        double s0 = (ea - b * eb) / den, u0 = (b * ea - eb) / den;
        double best = 1e300;
        s = 0.0;
        u = 0.0;
        if (s0 >= -ha && s0 <= ha && u0 >= -hb && u0 <= hb) {
            best = dist2(s0, u0);
            s = s0;
            u = u0;
        }
        for (int k = 0; k < 2; ++k) {
            double ss = k ? ha : -ha;
            double uu = clampd(ss * b - eb, -hb, hb);
            double v = dist2(ss, uu);
            if (v < best) {
                best = v;
                s = ss;
                u = uu;
            }
        }
        for (int k = 0; k < 2; ++k) {
            double uu = k ? hb : -hb;
            double ss = clampd(ea + uu * b, -ha, ha);
            double v = dist2(ss, uu);
            if (v < best) {
                best = v;
                s = ss;
                u = uu;
            }
        }
    }
    d3 p = s * ta;
    d3 qb = d + u * tb;
    d3 w = qb - p;
    double dist = len(w);
    d3 n;
    if (dist >= 1e-12) {
        n = (1.0 / dist) * w;
    } else {
        if (planar) {
            n = mk(-ta.y, ta.x, 0.0);
            n = (1.0 / len(n)) * n;
        } else if (dot(c, c) >= 1e-12) {
            n = (1.0 / len(c)) * c;
        } else {
            n = d - ea * ta;
            double l = len(n);
            if (l < 1e-12) {
                n = mk(-ta.y, ta.x, 0.0);
                l = len(n);
            }
            if (l < 1e-12) {
                n = mk(0.0, -ta.z, ta.y);
                l = len(n);
            }
            n = (1.0 / l) * n;
        }
        if (dot(n, d) < 0.0) n = -1.0 * n;
    }
    Snsd o;
    o.phi = dist - ra - rb;
    o.n = n;
    o.ra = p + ra * n;
    o.rb = (qb - d) - rb * n;
    return o;
}

// ===========================================================================
// SNSD of two tori (Sec. 6, rings): the distance between the two centre
// circles minus the two minor radii.  For a point y(t) of circle a (angle t)
// the squared distance to circle b is g(t) = |w|^2 - 2 R_b rho + R_b^2, with
// w = y - d and rho the distance of y from b's axis, so the 2-D minimisation
// over both angles is a 1-D one over t.  g is sampled at kTorusNs angles;
// each of the kTorusK smallest sampled local minima is refined by Newton's
// method on g' (analytic g', g'') inside its two neighbouring steps, with a
// bisection step whenever Newton leaves the bracket, and the smallest result
// wins (the earlier sample on ties).  Readings where the closest pair is
// degenerate: centre circles that meet get n = t_a x t_b (their tangents
// there), or the axis of a when the tangents are parallel, signed n.d >= 0;
// a point of a on b's axis takes b's first frame vector as the direction.
// ===========================================================================
constexpr int kTorusNs = 64;
constexpr int kTorusK = 4;

struct RingPoint {
    double g, g1, g2;
};

// g and (with kDeriv) its first two derivatives at (cos t, sin t) = (c, s).
template <bool kDeriv>
__device__ inline RingPoint ring_point(double c, double s, d3 e1, d3 e2, double Ra, d3 d, d3 eb, double Rb) {
    const d3 y = Ra * (c * e1 + s * e2);
    const d3 w = y - d;
    const double h = dot(w, eb);
    const d3 up = w - h * eb;
    const double rho = sqrt(dot(up, up));
    RingPoint r;
    r.g = dot(w, w) - 2.0 * Rb * rho + Rb * Rb;
    r.g1 = r.g2 = 0.0;
    if (kDeriv) {
        const d3 y1 = Ra * (c * e2 - s * e1);  // y' (and y'' = -y)
        const double irho = rho > 0.0 ? 1.0 / rho : 0.0;
        const double h1 = dot(y1, eb), uy1 = dot(up, y1), y1y1 = dot(y1, y1);
        const double rho1 = uy1 * irho;
        const double rho2 = (y1y1 - h1 * h1 - dot(up, y)) * irho - rho1 * rho1 * irho;
        r.g1 = 2.0 * dot(w, y1) - 2.0 * Rb * rho1;
        r.g2 = 2.0 * (y1y1 - dot(w, y)) - 2.0 * Rb * rho2;
    }
    return r;
}

__device__ Snsd snsd_torus(d3 d, d3 ea, double Ra, double ra, d3 eb, double Rb, double rb) {
    d3 e1, e2, f1, f2;
    tangent_frame(ea, e1, e2);
    tangent_frame(eb, f1, f2);
    const double step = 2.0 * M_PI / kTorusNs;
    double cs, sn;
    sincos(step, &sn, &cs);
    // the kTorusK smallest sampled local minima (value, sample, cos, sin),
    // ascending
    double kv[kTorusK], kc[kTorusK], ks[kTorusK];
    int ki[kTorusK];
#pragma unroll
    for (int k = 0; k < kTorusK; ++k) {
        kv[k] = 1e300;
        ki[k] = -1;
        kc[k] = 1.0;
        ks[k] = 0.0;
    }
    // samples by rotation of (cos, sin) by the step (drift of a few ulp over
    // the turn: the samples only pick the brackets)
    const double gl = ring_point<false>(cs, -sn, e1, e2, Ra, d, eb, Rb).g;  // t = -step
    const double g0 = ring_point<false>(1.0, 0.0, e1, e2, Ra, d, eb, Rb).g;
    double gp = gl, gc = g0, c = 1.0, s = 0.0;
    for (int i = 0; i < kTorusNs; ++i) {
        const double cn = c * cs - s * sn, snx = s * cs + c * sn;
        const double gn = i + 1 < kTorusNs ? ring_point<false>(cn, snx, e1, e2, Ra, d, eb, Rb).g : g0;
        if (gc <= gp && gc <= gn && gc < kv[kTorusK - 1]) {
            kv[kTorusK - 1] = gc;
            ki[kTorusK - 1] = i;
            kc[kTorusK - 1] = c;
            ks[kTorusK - 1] = s;
#pragma unroll
            for (int k = kTorusK - 1; k > 0; --k)
                if (kv[k] < kv[k - 1]) {
                    const double tv = kv[k], tc = kc[k], ts = ks[k];
                    kv[k] = kv[k - 1];
                    kc[k] = kc[k - 1];
                    ks[k] = ks[k - 1];
                    kv[k - 1] = tv;
                    kc[k - 1] = tc;
                    ks[k - 1] = ts;
                    const int ti = ki[k];
                    ki[k] = ki[k - 1];
                    ki[k - 1] = ti;
                }
        }
        gp = gc;
        gc = gn;
        c = cn;
        s = snx;
    }
    // Newton on g' from each candidate; (cos t, sin t) follow t by rotation
    // through the step taken (its cosine and sine by their Taylor series to
    // degree 8 and 9 below 0.05 rad, error under 1e-17; sincos above)
    double bg = 1e300, bc = 1.0, bs = 0.0;
#pragma unroll
    for (int k = 0; k < kTorusK; ++k) {
        if (ki[k] < 0) continue;
        double t = step * ki[k], lo = t - step, hi = t + step;
        double ct = kc[k], st = ks[k];
        for (int it = 0; it < 40; ++it) {
            const RingPoint r = ring_point<true>(ct, st, e1, e2, Ra, d, eb, Rb);
            if (r.g1 < 0.0)
                lo = t;
            else
                hi = t;
            double tn = r.g2 > 0.0 ? t - r.g1 / r.g2 : 0.5 * (lo + hi);
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            const double dl = tn - t;
            double cd, sd;
            if (fabs(dl) < 0.05) {
                const double z = dl * dl;
                cd = 1.0 - z * (1.0 / 2 - z * (1.0 / 24 - z * (1.0 / 720 - z * (1.0 / 40320))));
                sd = dl * (1.0 - z * (1.0 / 6 - z * (1.0 / 120 - z * (1.0 / 5040 - z * (1.0 / 362880)))));
            } else {
                sincos(dl, &sd, &cd);
            }
            const double cn = ct * cd - st * sd;
            st = st * cd + ct * sd;
            ct = cn;
            t = tn;
            if (fabs(dl) <= 1e-15 * (1.0 + fabs(t))) break;
        }
        const double g = ring_point<false>(ct, st, e1, e2, Ra, d, eb, Rb).g;
        if (g < bg) {
            bg = g;
            bc = ct;
            bs = st;
        }
    }
    const d3 pa = Ra * (bc * e1 + bs * e2);  // centre-circle point of a (relative to x_a)
    const d3 w = pa - d;
    const d3 up = w - dot(w, eb) * eb;
    const double rho = sqrt(dot(up, up));
    const d3 pb = d + (rho > 0.0 ? (Rb / rho) * up : Rb * f1);  // of b (relative to x_a)
    const d3 wc = pb - pa;
    const double dist = len(wc);
    d3 n;
    if (dist >= 1e-12) {
        n = (1.0 / dist) * wc;
    } else {
        const d3 ta = cross(ea, pa), tb = cross(eb, pb - d);
        n = cross(ta, tb);
        double l2 = dot(n, n);
        if (l2 < 1e-12 * (dot(ta, ta) * dot(tb, tb) + 1e-300)) {
            n = ea;
            l2 = 1.0;
        }
        n = (1.0 / sqrt(l2)) * n;
        if (dot(n, d) < 0.0) n = -1.0 * n;
    }
    Snsd o;
    o.phi = dist - ra - rb;
    o.n = n;
    o.ra = pa + ra * n;
    o.rb = (pb - d) - rb * n;
    return o;
}

// ===========================================================================
// per-body set-up at C^k: geometry (Sigma or axis), bounding radius,
// operator K, free velocity U_free
// ===========================================================================
// K per body (9 comps): translational diagonal (3) and rotational symmetric
// (6), already projected for a monolayer (z translation, x/y rotation off).
//  overdamped: K = M = (1/xi) diag(I/L, 12 I/L^3), L = 2 max semiaxis
//              (ellipsoid), l + 2 r (spherocylinder, tip to tip) or
//              2 (R + r) (torus, outer diameter)
//  inertial:   K = dt M^-1, M^-1 = diag(I/m, R diag(1/I_body) R^T), solid
//              ellipsoid of density rho
__global__ void k_body_setup(int nb, const double *__restrict__ q, int ldq, const int *__restrict__ kind,
                             const double *__restrict__ p, int ldp, const double *__restrict__ rho_xi,
                             const double *__restrict__ u, int ldu, const double *__restrict__ fext, int ldf,
                             int dynamics, int planar, double dt, double *__restrict__ geo, int ldg,
                             double *__restrict__ Rb, double *__restrict__ K, int ldk, float *__restrict__ K32,
                             double *__restrict__ vfree, int ldv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double qs = q[i], qx = q[ldq + i], qy = q[2 * ldq + i], qz = q[3 * ldq + i];
    d3 c0, c1, c2;
    quat_axes(qs, qx, qy, qz, c0, c1, c2);
    double a = p[i], b = p[ldp + i], c = p[2 * ldp + i];
    int kd = kind[i];
    if (kd == 0) {
        // Sigma = R diag(a^2, b^2, c^2) R^T
        double a2 = a * a, b2 = b * b, c2s = c * c;
        geo[0 * ldg + i] = a2 * c0.x * c0.x + b2 * c1.x * c1.x + c2s * c2.x * c2.x;
        geo[1 * ldg + i] = a2 * c0.y * c0.y + b2 * c1.y * c1.y + c2s * c2.y * c2.y;
        geo[2 * ldg + i] = a2 * c0.z * c0.z + b2 * c1.z * c1.z + c2s * c2.z * c2.z;
        geo[3 * ldg + i] = a2 * c0.x * c0.y + b2 * c1.x * c1.y + c2s * c2.x * c2.y;
        geo[4 * ldg + i] = a2 * c0.x * c0.z + b2 * c1.x * c1.z + c2s * c2.x * c2.z;
        geo[5 * ldg + i] = a2 * c0.y * c0.z + b2 * c1.y * c1.z + c2s * c2.y * c2.z;
        Rb[i] = fmax(a, fmax(b, c));
    } else {
        // the axis: body x (spherocylinder) or body z (torus)
        const d3 ax = kd == 2 ? c2 : c0;
        geo[0 * ldg + i] = ax.x;
        geo[1 * ldg + i] = ax.y;
        geo[2 * ldg + i] = ax.z;
        geo[3 * ldg + i] = 0.0;
        geo[4 * ldg + i] = 0.0;
        geo[5 * ldg + i] = 0.0;
        Rb[i] = kd == 2 ? a + b : 0.5 * b + a;
    }
    if (!K) return;
    double kt[3], kr[6];
    if (dynamics == 0) {
        double L = (kd == 0) ? 2.0 * fmax(a, fmax(b, c)) : (kd == 2 ? 2.0 * (a + b) : b + 2.0 * a);
        double xi = rho_xi[i];
        double t = 1.0 / (xi * L), r = 12.0 / (xi * L * L * L);
        kt[0] = kt[1] = kt[2] = t;
        kr[0] = kr[1] = kr[2] = r;
        kr[3] = kr[4] = kr[5] = 0.0;
    } else {
        double m = rho_xi[i] * (4.0 / 3.0) * M_PI * a * b * c;
        double I0 = m * (b * b + c * c) / 5.0, I1 = m * (a * a + c * c) / 5.0, I2 = m * (a * a + b * b) / 5.0;
        double w0 = dt / I0, w1 = dt / I1, w2 = dt / I2;
        kt[0] = kt[1] = kt[2] = dt / m;
        kr[0] = w0 * c0.x * c0.x + w1 * c1.x * c1.x + w2 * c2.x * c2.x;
        kr[1] = w0 * c0.y * c0.y + w1 * c1.y * c1.y + w2 * c2.y * c2.y;
        kr[2] = w0 * c0.z * c0.z + w1 * c1.z * c1.z + w2 * c2.z * c2.z;
        kr[3] = w0 * c0.x * c0.y + w1 * c1.x * c1.y + w2 * c2.x * c2.y;
        kr[4] = w0 * c0.x * c0.z + w1 * c1.x * c1.z + w2 * c2.x * c2.z;
        kr[5] = w0 * c0.y * c0.z + w1 * c1.y * c1.z + w2 * c2.y * c2.z;
    }
    if (planar) {
        kt[2] = 0.0;
        kr[0] = kr[1] = kr[3] = kr[4] = kr[5] = 0.0;
    }
    for (int k = 0; k < 3; ++k) {
        K[k * ldk + i] = kt[k];
        K32[k * ldk + i] = (float)kt[k];
    }
    for (int k = 0; k < 6; ++k) {
        K[(3 + k) * ldk + i] = kr[k];
        K32[(3 + k) * ldk + i] = (float)kr[k];
    }
    // U_free = U^k (inertial) + K F_ext
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (dynamics == 1 && u)
        for (int k = 0; k < 6; ++k) v[k] = u[k * ldu + i];
    if (fext) {
        double f[6];
        for (int k = 0; k < 6; ++k) f[k] = fext[k * ldf + i];
        v[0] += kt[0] * f[0];
        v[1] += kt[1] * f[1];
        v[2] += kt[2] * f[2];
        v[3] += kr[0] * f[3] + kr[3] * f[4] + kr[4] * f[5];
        v[4] += kr[3] * f[3] + kr[1] * f[4] + kr[5] * f[5];
        v[5] += kr[4] * f[3] + kr[5] * f[4] + kr[2] * f[5];
    }
    if (planar) {
        v[2] = 0.0;
        v[3] = 0.0;
        v[4] = 0.0;
    }
    for (int k = 0; k < 6; ++k) vfree[k * ldv + i] = v[k];
}

// ===========================================================================
// trial configuration C_{n+1} = C^k (+) dt V_n   (Alg. 1; Eq. relcp)
// ===========================================================================
// Reading of the configuration map: positions x + dt v exactly; orientation
// exp(dt w) (x) q with world-frame w, renormalised (agrees with the linear
// G^k to first order in dt).
__device__ inline unsigned long long dbl_bits(double v) { return (unsigned long long)__double_as_longlong(v); }

__global__ void k_trial(int nb, const double *__restrict__ x, int ldx, const double *__restrict__ q, int ldq,
                        const double *__restrict__ vfree, const double *__restrict__ vc, int ldv, double dt,
                        const int *__restrict__ kind, const double *__restrict__ p, int ldp,
                        const double *__restrict__ Rb, double *__restrict__ xt, double *__restrict__ qt,
                        double *__restrict__ geo, int ldg, double *__restrict__ vout,
                        unsigned long long *__restrict__ maxdisp, RowsT<double> R, BodiesT<double> Bd,
                        int vc_rows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double disp = 0.0;
    if (i < nb) {
        double v[6];
        if (vc_rows) {
            // the body's contact velocity K D max(0, gamma) over its incident
            // rows (the LCP's own scatter arithmetic), also stored if Bd.vc
            // is set
            double w[6];
            scatter_body<double, 0>(R, Bd, i, 0.0, VRegs<double>{w});
            for (int k = 0; k < 6; ++k) {
                if (Bd.vc) Bd.vc[k * Bd.ld + i] = w[k];
                v[k] = (vfree ? vfree[k * ldv + i] : 0.0) + w[k];
            }
        } else {
            for (int k = 0; k < 6; ++k) v[k] = (vfree ? vfree[k * ldv + i] : 0.0) + vc[k * ldv + i];
        }
        if (vout)
            for (int k = 0; k < 6; ++k) vout[k * ldv + i] = v[k];
        for (int k = 0; k < 3; ++k) xt[k * ldx + i] = x[k * ldx + i] + dt * v[k];
        d3 th = mk(dt * v[3], dt * v[4], dt * v[5]);
        double ang = len(th);
        double es, ek;
        if (ang < 1e-8) {
            es = 1.0 - ang * ang / 8.0;
            ek = 0.5 - ang * ang / 48.0;
        } else {
            es = cos(0.5 * ang);
            ek = sin(0.5 * ang) / ang;
        }
        d3 ew = ek * th;
        double s0 = q[i];
        d3 w0 = mk(q[ldq + i], q[2 * ldq + i], q[3 * ldq + i]);
        double rs = es * s0 - dot(ew, w0);
        d3 rw = es * w0 + s0 * ew + cross(ew, w0);
        double nr = sqrt(rs * rs + dot(rw, rw));
        rs /= nr;
        rw = (1.0 / nr) * rw;
        qt[i] = rs;
        qt[ldq + i] = rw.x;
        qt[2 * ldq + i] = rw.y;
        qt[3 * ldq + i] = rw.z;
        // geometry at the trial orientation
        d3 c0, c1, c2;
        quat_axes(rs, rw.x, rw.y, rw.z, c0, c1, c2);
        if (kind[i] == 0) {
            double a2 = p[i] * p[i], b2 = p[ldp + i] * p[ldp + i], cc = p[2 * ldp + i] * p[2 * ldp + i];
            geo[0 * ldg + i] = a2 * c0.x * c0.x + b2 * c1.x * c1.x + cc * c2.x * c2.x;
            geo[1 * ldg + i] = a2 * c0.y * c0.y + b2 * c1.y * c1.y + cc * c2.y * c2.y;
            geo[2 * ldg + i] = a2 * c0.z * c0.z + b2 * c1.z * c1.z + cc * c2.z * c2.z;
            geo[3 * ldg + i] = a2 * c0.x * c0.y + b2 * c1.x * c1.y + cc * c2.x * c2.y;
            geo[4 * ldg + i] = a2 * c0.x * c0.z + b2 * c1.x * c1.z + cc * c2.x * c2.z;
            geo[5 * ldg + i] = a2 * c0.y * c0.z + b2 * c1.y * c1.z + cc * c2.y * c2.z;
        } else {
            const d3 ax = kind[i] == 2 ? c2 : c0;
            geo[0 * ldg + i] = ax.x;
            geo[1 * ldg + i] = ax.y;
            geo[2 * ldg + i] = ax.z;
            geo[3 * ldg + i] = 0.0;
            geo[4 * ldg + i] = 0.0;
            geo[5 * ldg + i] = 0.0;
        }
        // bound on the displacement of any surface point
        disp = dt * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + Rb[i] * ang;
    }
    // block max into this block's slot (reduced in a fixed order later)
    __shared__ double wmax[4];
    for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) disp = fmax(disp, __shfl_xor(disp, o, RELCP_WAVE));
    if ((threadIdx.x & (RELCP_WAVE - 1)) == 0) wmax[threadIdx.x / RELCP_WAVE] = disp;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int k = 0; k < (int)(blockDim.x / RELCP_WAVE); ++k) mx = fmax(mx, wmax[k]);
        maxdisp[blockIdx.x] = dbl_bits(mx);  // non-negative doubles order like their bit patterns
    }
}

// ===========================================================================
// SNSD over a pair list
// ===========================================================================
// Sortable key of a double (monotone map to unsigned 64-bit).
__device__ inline unsigned long long order_key(double v) {
    unsigned long long b = dbl_bits(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// KIND = -1: every shape kind; KIND = 2: tori only (the ellipsoid Newton
// code, whose register demand spills the kernel for every kind, is absent).
template <int KIND>
__global__ void __launch_bounds__(256, 4) k_snsd_pairs(SnsdArgs A) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    double phi = 1e300, marg = 1e300;
    int fl = 0;
    if (k < A.m) {
        const int a = A.pa[k], b = A.pb[k];
        const int ir = A.init_row ? A.init_row[k] : -1;
        // Every datum the pair may need is loaded up front, so the loads
        // form two dependent groups (pair, then bodies) and the packing's
        // box a third: the hint with the pair indices, then positions,
        // bounding radii, kind and geometry of both bodies together.
        d3 hint = mk(1, 0, 0);
        if (A.hint) hint = mk(A.hint[k], A.hint[A.ldo + k], A.hint[2 * A.ldo + k]);
        const int pk = A.body_batch ? A.body_batch[a] : 0;
        const d3 xa = mk(A.x[a], A.x[A.ldx + a], A.x[2 * A.ldx + a]);
        const d3 xb = mk(A.x[b], A.x[A.ldx + b], A.x[2 * A.ldx + b]);
        const double rba = A.Rb ? A.Rb[a] : 0.0, rbb = A.Rb ? A.Rb[b] : 0.0;
        const int kd = KIND >= 0 ? KIND : A.kind[a];
        double ga[6], gb[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            ga[t] = A.geo[t * A.ldg + a];
            gb[t] = A.geo[t * A.ldg + b];
        }
        const double lam0 = ir >= 0 ? A.init_gam[ir] : 0.0;
        const double *bx = A.boxes + 3 * pk;
        const double L0 = bx[0], L1 = bx[1], L2 = bx[2];
        d3 d = xb - xa;
        if (L0 > 0.0) d.x -= L0 * rint(d.x / L0);
        if (L1 > 0.0) d.y -= L1 * rint(d.y / L1);
        if (L2 > 0.0) d.z -= L2 * rint(d.z / L2);
        Snsd s;
        const double dl = len(d);
        const double sgap = A.Rb ? dl - rba - rbb : -1e300;
        if (sgap > (A.mode == 0 ? A.thresh : 0.0) && dl > 0.0) {
            s.phi = sgap;
            s.n = (1.0 / dl) * d;
            s.ra = rba * s.n;
            s.rb = (-rbb) * s.n;
        } else if (KIND < 0 && kd == 0) {
            const sym3 Sa{ga[0], ga[1], ga[2], ga[3], ga[4], ga[5]};
            const sym3 Sb{gb[0], gb[1], gb[2], gb[3], gb[4], gb[5]};
            bool has = false;
            if (A.hint) {
                const double hl = len(hint);
                has = hl > 0.5;
                if (has) hint = (1.0 / hl) * hint;
            }
            s = snsd_ellipsoid(d, Sa, Sb, has ? hint : mk(1, 0, 0), has);
        } else if (kd == 2) {
            s = snsd_torus(d, mk(ga[0], ga[1], ga[2]), A.p[a], A.p[A.ldp + a], mk(gb[0], gb[1], gb[2]), A.p[b],
                           A.p[A.ldp + b]);
        } else if (KIND < 0) {
            const d3 ta = mk(ga[0], ga[1], ga[2]);
            const d3 tb = mk(gb[0], gb[1], gb[2]);
            s = snsd_spherocyl(d, ta, A.p[A.ldp + a], A.p[a], tb, A.p[A.ldp + b], A.p[b], A.planar != 0);
        }
        A.out[k] = s.phi;
        A.out[1 * A.ldo + k] = s.n.x;
        A.out[2 * A.ldo + k] = s.n.y;
        A.out[3 * A.ldo + k] = s.n.z;
        A.out[4 * A.ldo + k] = s.ra.x;
        A.out[5 * A.ldo + k] = s.ra.y;
        A.out[6 * A.ldo + k] = s.ra.z;
        A.out[7 * A.ldo + k] = s.rb.x;
        A.out[8 * A.ldo + k] = s.rb.y;
        A.out[9 * A.ldo + k] = s.rb.z;
        phi = s.phi;
        marg = fabs(s.phi + A.eps);
        fl = (A.mode == 0) ? (s.phi <= A.thresh ? 1 : 0) : (s.phi < -A.eps ? 1 : 0);
        if (A.flag) A.flag[k] = fl;
        if (A.clear) A.clear[k] = lam0;
    }
    if (A.bcount) {
        // this block's count of set flags (the compaction's tile offsets)
        __shared__ int wcnt[4];
        const int c = __popcll(__ballot(fl != 0));
        if ((threadIdx.x & (RELCP_WAVE - 1)) == 0) wcnt[threadIdx.x / RELCP_WAVE] = c;
        __syncthreads();
        if (threadIdx.x == 0) A.bcount[blockIdx.x] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    }
    if (A.minphi) {
        // block minima into this block's slots (reduced in a fixed order later)
        __shared__ double wphi[4], wmarg[4];
        for (int o = RELCP_WAVE / 2; o > 0; o >>= 1) {
            phi = fmin(phi, __shfl_xor(phi, o, RELCP_WAVE));
            marg = fmin(marg, __shfl_xor(marg, o, RELCP_WAVE));
        }
        if ((threadIdx.x & (RELCP_WAVE - 1)) == 0) {
            wphi[threadIdx.x / RELCP_WAVE] = phi;
            wmarg[threadIdx.x / RELCP_WAVE] = marg;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double mp = 1e300, mm = 1e300;
            for (int k = 0; k < (int)(blockDim.x / RELCP_WAVE); ++k) {
                mp = fmin(mp, wphi[k]);
                mm = fmin(mm, wmarg[k]);
            }
            A.minphi[blockIdx.x] = mp < 1e300 ? order_key(mp) : ~0ull;
            A.minmarg[blockIdx.x] = mm < 1e300 ? order_key(mm) : ~0ull;
        }
    }
}

// ===========================================================================
// candidate pairs by a per-packing cell list
// ===========================================================================
__device__ inline int cell_coord(double v, int k, const PackGrid &g) {
    if (g.periodic[k]) {
        double t = v / g.box[k];
        t -= floor(t);
        int c = (int)(t * g.nc[k]);
        return c >= g.nc[k] ? g.nc[k] - 1 : (c < 0 ? 0 : c);
    }
    int c = (int)floor((v - g.org[k]) / g.cs[k]);
    return c < 0 ? 0 : (c >= g.nc[k] ? g.nc[k] - 1 : c);
}

__global__ void k_cell_assign(int nb, const double *__restrict__ x, int ldx, const int *__restrict__ body_batch,
                              const PackGrid *__restrict__ grids, int *__restrict__ body_cell,
                              int *__restrict__ cell_count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    int pk = body_batch ? body_batch[i] : 0;
    PackGrid g = grids[pk];
    int cx = cell_coord(x[i], 0, g), cy = cell_coord(x[ldx + i], 1, g), cz = cell_coord(x[2 * ldx + i], 2, g);
    long long c = g.cell_off + ((long long)cz * g.nc[1] + cy) * g.nc[0] + cx;
    body_cell[i] = (int)c;
    atomicAdd(cell_count + c, 1);
}

__global__ void k_cell_fill(int nb, const int *__restrict__ body_cell, const int *__restrict__ cell_start,
                            int *__restrict__ cursor, int *__restrict__ items) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    int c = body_cell[i];
    int pos = cell_start[c] + atomicAdd(cursor + c, 1);
    items[pos] = i;
}

// neighbour offsets of one direction: unique cells among c-1, c, c+1
__device__ inline int nbr_cells(int c, int k, const PackGrid &g, int out[3]) {
    int n = g.nc[k];
    if (g.periodic[k]) {
        if (n == 1) {
            out[0] = 0;
            return 1;
        }
        if (n == 2) {
            out[0] = 0;
            out[1] = 1;
            return 2;
        }
        out[0] = (c + n - 1) % n;
        out[1] = c;
        out[2] = (c + 1) % n;
        return 3;
    }
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int cc = c + o;
        if (cc >= 0 && cc < n) out[m++] = cc;
    }
    return m;
}

// Shape of a body for its support radius h(n) = max over the body of
// n.(y - x), n a unit vector: sqrt(n^T Sigma n) for an ellipsoid, r + (l/2)
// |t.n| for a spherocylinder (axis t, radius r = p0, length l = p1), and
// R sqrt(1 - (e.n)^2) + r for a torus (axis e, radii R = p0, r = p1).
struct SupportShape {
    int kind;
    sym3 S;     // Sigma, or the axis in its first three entries
    double r, l;  // shape parameters p0, p1 (0 for an ellipsoid)
};
__device__ inline SupportShape support_shape(const PairShapes &P, int i) {
    const double *g = P.geo;
    const int L = P.ldg;
    SupportShape s;
    s.kind = P.kind[i];
    s.S = sym3{g[i], g[L + i], g[2 * L + i], g[3 * L + i], g[4 * L + i], g[5 * L + i]};
    s.r = s.kind == 0 ? 0.0 : P.p[i];
    s.l = s.kind == 0 ? 0.0 : P.p[P.ldp + i];
    return s;
}
__device__ inline double support_radius(const SupportShape &s, d3 n) {
    if (s.kind == 0) return sqrt(dot(n, mul(s.S, n)));
    const double c = s.S.xx * n.x + s.S.yy * n.y + s.S.zz * n.z;  // axis . n
    if (s.kind == 2) return s.r * sqrt(fmax(0.0, 1.0 - c * c)) + s.l;
    return s.r + 0.5 * s.l * fabs(c);
}

template <bool kFill>
__global__ void __launch_bounds__(256) k_pairs(int nb, const double *__restrict__ x, int ldx,
                                               const double *__restrict__ Rb, const int *__restrict__ body_batch,
                                               const PackGrid *__restrict__ grids, const int *__restrict__ body_cell,
                                               const int *__restrict__ cell_start, const int *__restrict__ cell_count,
                                               const int *__restrict__ items, double skin,
                                               int *__restrict__ pair_count, const int *__restrict__ pair_off,
                                               int *__restrict__ pa, int *__restrict__ pb, int cap, PairShapes sh) {
    // threads walk the bodies in cell order, so neighbouring lanes scan the
    // same neighbour cells
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    int a = items[t];
    int pk = body_batch ? body_batch[a] : 0;
    PackGrid g = grids[pk];
    double xa = x[a], ya = x[ldx + a], za = x[2 * ldx + a], ra = Rb[a];
    long long local = body_cell[a] - g.cell_off;
    int cx = (int)(local % g.nc[0]);
    int cy = (int)((local / g.nc[0]) % g.nc[1]);
    int cz = (int)(local / ((long long)g.nc[0] * g.nc[1]));
    int ox[3], oy[3], oz[3];
    int nx = nbr_cells(cx, 0, g, ox), ny = nbr_cells(cy, 1, g, oy), nz = nbr_cells(cz, 2, g, oz);
    SupportShape sa{};
    if (sh.geo) sa = support_shape(sh, a);  // body a's shape, once
    int cnt = 0;
    int base = kFill ? pair_off[a] : 0;
    // per row of neighbour cells (fixed z and y offsets): the ranges of its
    // (up to) three cells first, then the candidates in batches of kU whose
    // indices, then positions, are loaded together; the order is that of the
    // cells and of their items
    constexpr int kU = 8;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy) {
            const long long rowc = g.cell_off + ((long long)oz[iz] * g.nc[1] + oy[iy]) * g.nc[0];
            int s0[3] = {0, 0, 0}, n0[3] = {0, 0, 0};
#pragma unroll
            for (int ix = 0; ix < 3; ++ix)
                if (ix < nx) {
                    const long long c = rowc + ox[ix];
                    s0[ix] = cell_start[c];
                    n0[ix] = cell_count[c];
                }
            const int tot = n0[0] + n0[1] + n0[2];
            for (int j0 = 0; j0 < tot; j0 += kU) {
                int bb[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int j = j0 + u;
                    const int tt = j < n0[0] ? s0[0] + j : (j < n0[0] + n0[1] ? s0[1] + j - n0[0] : s0[2] + j - n0[0] - n0[1]);
                    bb[u] = j < tot ? items[tt] : -1;
                }
                double bx[kU], by[kU], bz[kU], br[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int b = bb[u] > a ? bb[u] : a;  // a itself for a skipped slot: in bounds
                    bx[u] = x[b];
                    by[u] = x[ldx + b];
                    bz[u] = x[2 * ldx + b];
                    br[u] = Rb[b];
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int b = bb[u];
                    if (b <= a) continue;  // also past the last candidate (b = -1)
                    double dx = bx[u] - xa, dy = by[u] - ya, dz = bz[u] - za;
                    if (g.periodic[0]) dx -= g.box[0] * rint(dx / g.box[0]);
                    if (g.periodic[1]) dy -= g.box[1] * rint(dy / g.box[1]);
                    if (g.periodic[2]) dz -= g.box[2] * rint(dz / g.box[2]);
                    const double dl = sqrt(dx * dx + dy * dy + dz * dz);
                    bool near = dl - ra - br[u] <= skin;
                    if (near && sh.geo && dl > 0.0) {
                        // the support gap along the centre line is a lower
                        // bound of Phi (Phi is its maximum over normals)
                        const d3 u3 = mk(dx / dl, dy / dl, dz / dl);
                        near = dl - support_radius(sa, u3) - support_radius(support_shape(sh, b), u3) <= skin;
                    }
                    if (near) {
                        if (kFill) {
                            int pos = base + cnt;
                            if (pos < cap) {
                                pa[pos] = a;
                                pb[pos] = b;
                            }
                        }
                        ++cnt;
                    }
                }
            }
        }
    if (!kFill) {
        pair_count[a] = cnt;
    } else {
        // order the partners of a by index (insertion sort of a short list)
        int lo = base, hi = min(base + cnt, cap);
        for (int i = lo + 1; i < hi; ++i) {
            int v = pb[i];
            int j = i - 1;
            while (j >= lo && pb[j] > v) {
                pb[j + 1] = pb[j];
                --j;
            }
            pb[j + 1] = v;
        }
    }
}

// ===========================================================================
// host launchers
// ===========================================================================
static inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

void launch_body_setup(const BodySetupArgs &a, hipStream_t s) {
    if (a.nb <= 0) return;
    hipLaunchKernelGGL(k_body_setup, dim3(nblk(a.nb, 256)), dim3(256), 0, s, a.nb, a.q, a.ldq, a.kind, a.p, a.ldp,
                       a.rho_xi, a.u, a.ldu, a.fext, a.ldf, a.dynamics, a.planar, a.dt, a.geo, a.ldg, a.Rb, a.K, a.ldk,
                       a.K32, a.vfree, a.ldv);
}

void launch_trial(int nb, const double *x, int ldx, const double *q, int ldq, const double *vfree, const double *vc,
                  int ldv, double dt, const int *kind, const double *p, int ldp, const double *Rb, double *xt,
                  double *qt, double *geo, int ldg, double *vout, unsigned long long *maxdisp, hipStream_t s,
                  const RowsT<double> *R, const BodiesT<double> *Bd) {
    if (nb <= 0) return;
    const bool rows = R && Bd;
    launch_k(k_trial, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, x, ldx, q, ldq, vfree, vc, ldv, dt, kind, p,
             ldp, Rb, xt, qt, geo, ldg, vout, maxdisp, rows ? *R : RowsT<double>{}, rows ? *Bd : BodiesT<double>{},
             rows ? 1 : 0);
}

int snsd_blocks(int m) { return nblk(m > 0 ? m : 1, 256); }
int trial_blocks(int nb) { return nblk(nb > 0 ? nb : 1, 256); }

void launch_snsd_pairs(const SnsdArgs &a, hipStream_t s) {
    if (a.m <= 0) return;
    if (a.only_kind == 2)
        launch_k(k_snsd_pairs<2>, dim3(nblk(a.m, 256)), dim3(256), 0, s, a);
    else
        launch_k(k_snsd_pairs<-1>, dim3(nblk(a.m, 256)), dim3(256), 0, s, a);
}

void launch_cell_assign(int nb, const double *x, int ldx, const int *body_batch, const PackGrid *grids,
                        int *body_cell, int *cell_count, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_cell_assign, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, x, ldx, body_batch, grids, body_cell,
                       cell_count);
}

void launch_cell_fill(int nb, const int *body_cell, const int *cell_start, int *cursor, int *items, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_cell_fill, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, body_cell, cell_start, cursor, items);
}

void launch_pairs(bool fill, int nb, const double *x, int ldx, const double *Rb, const int *body_batch,
                  const PackGrid *grids, const int *body_cell, const int *cell_start, const int *cell_count,
                  const int *items, double skin, int *pair_count, const int *pair_off, int *pa, int *pb, int cap,
                  hipStream_t s, const PairShapes *shapes) {
    if (nb <= 0) return;
    const PairShapes sh = shapes ? *shapes : PairShapes{};
    if (fill)
        launch_k(k_pairs<true>, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, x, ldx, Rb, body_batch, grids,
                 body_cell, cell_start, cell_count, items, skin, pair_count, pair_off, pa, pb, cap, sh);
    else
        launch_k(k_pairs<false>, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, x, ldx, Rb, body_batch, grids,
                 body_cell, cell_start, cell_count, items, skin, pair_count, pair_off, pa, pb, cap, sh);
}

}  // namespace relcp
