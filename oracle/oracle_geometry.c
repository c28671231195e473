/*
 * oracle_geometry.c -- closest points used by the narrow phase (App. C,
 * Algorithm 3: closestPointOnFace and closestPointOnEdge), in FP64.
 *
 * TEST INFRASTRUCTURE ONLY (see ccfr_oracle.h).
 *
 * Point-triangle: the classical Voronoi-region walk (vertex regions, then edge
 * regions, then the face interior), as in Ericson, "Real-Time Collision
 * Detection", Sec. 5.1.5.  Segment-segment: the clamped minimisation of the
 * squared distance over [0,1]^2 (Ericson Sec. 5.1.9), plus the parallel-segment
 * rule the paper leaves open: when |d1 x d2|^2 <= 1e-10 |d1|^2 |d2|^2,
 * s is the midpoint of the overlap of the second segment projected onto the first
 * (clamped to [0,1]) and t is the clamped projection of the resulting point.
 */
#include "ccfr_oracle.h"

#include <math.h>

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double a[3], const double b[3], double o[3]) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

int orc_closest_point_triangle(const double p[3], const double a[3], const double b[3],
                               const double c[3], double q[3], double bary[3]) {
    double ab[3], ac[3], ap[3], bp[3], cp[3], nrm[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    cross3(ab, ac, nrm);
    /* a triangle of (numerically) zero area has no face region */
    if (dot3(nrm, nrm) <= 1e-12 * dot3(ab, ab) * dot3(ac, ac)) return -1;

    sub3(p, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { bary[0] = 1; bary[1] = 0; bary[2] = 0; goto done; }

    sub3(p, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { bary[0] = 0; bary[1] = 1; bary[2] = 0; goto done; }

    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        bary[0] = 1.0 - v; bary[1] = v; bary[2] = 0; goto done;
    }

    sub3(p, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { bary[0] = 0; bary[1] = 0; bary[2] = 1; goto done; }

    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        bary[0] = 1.0 - w; bary[1] = 0; bary[2] = w; goto done;
    }

    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        bary[0] = 0; bary[1] = 1.0 - w; bary[2] = w; goto done;
    }
    {
        double den = 1.0 / (va + vb + vc);
        double v = vb * den, w = vc * den;
        bary[0] = 1.0 - v - w; bary[1] = v; bary[2] = w;
    }
done:
    for (int k = 0; k < 3; ++k) q[k] = bary[0] * a[k] + bary[1] * b[k] + bary[2] * c[k];
    return 0;
}

int orc_closest_points_segments(const double a[3], const double b[3], const double c[3],
                                const double d[3], double* s_out, double* t_out) {
    double d1[3], d2[3], r[3], cr[3];
    sub3(b, a, d1);
    sub3(d, c, d2);
    sub3(a, c, r);
    double A = dot3(d1, d1), E = dot3(d2, d2), F = dot3(d2, r);
    if (A <= 0.0 || E <= 0.0) return -1;            /* zero-length edge */
    double C = dot3(d1, r), B = dot3(d1, d2);
    cross3(d1, d2, cr);
    double s, t;
    if (dot3(cr, cr) <= 1e-10 * A * E) {             /* parallel */
        double ca[3], da[3];
        sub3(c, a, ca);
        sub3(d, a, da);
        double tc = dot3(ca, d1) / A, td = dot3(da, d1) / A;
        double lo = fmin(tc, td), hi = fmax(tc, td);
        double olo = fmax(lo, 0.0), ohi = fmin(hi, 1.0);
        if (olo <= ohi) s = 0.5 * (olo + ohi);
        else s = (hi < 0.0) ? 0.0 : 1.0;
        double pc[3];
        for (int k = 0; k < 3; ++k) pc[k] = a[k] + s * d1[k] - c[k];
        t = clamp01(dot3(pc, d2) / E);
        *s_out = s;
        *t_out = t;
        return 1;
    }
    double den = A * E - B * B;
    s = clamp01((B * F - C * E) / den);
    t = (B * s + F) / E;
    if (t < 0.0) {
        t = 0.0;
        s = clamp01(-C / A);
    } else if (t > 1.0) {
        t = 1.0;
        s = clamp01((B - C) / A);
    }
    *s_out = s;
    *t_out = t;
    return 0;
}

/* Closest point q = (1 - t) a + t b on segment ab to p (Ericson Sec. 5.1.2:
 * the projection parameter clamped to [0, 1]).  Returns -1 for a segment of
 * zero length. */
int orc_closest_point_segment(const double p[3], const double a[3], const double b[3], double* t) {
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    const double L = dot3(ab, ab);
    if (L <= 0.0) return -1;
    *t = clamp01(dot3(ap, ab) / L);
    return 0;
}
