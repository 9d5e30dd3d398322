/*
 * TEST INFRASTRUCTURE -- FP64 CPU oracle of the exact swept-disc surface
 * ("ORACLE-X"), the limit that the depth-d method of Binder & Keller
 * (arXiv 1811.03374) converges to.
 *
 * Only the test suite and the benchmark's self-check load this library; the
 * HIP path shares nothing with it.
 *
 * Definition. The fiber is the solid swept by a circular disc of radius r(u)
 * centred on the cubic Bezier curve C(u) in the plane normal to C'(u),
 * u in [0, 1] (abstract, Sections 1 and 3.3: circular cross section, radius
 * interpolated by the same Bezier basis), with flat end caps at u = 0 and
 * u = 1 (the caps of the end cylinders, Section 3.3). The result is the
 * smallest t in [0, tmax) at which the ray O + t*D/|D| lies in that solid.
 *
 * Computation, in the FP64 frame of the ray (origin at 0, direction +z):
 *   side  roots u in [0,1] of F(u) = Dz^2 (Cx^2 + Cy^2) + (Cx Dx + Cy Dy)^2
 *         - r^2 Dz^2 with D = C'/3, where the ray meets the boundary circle of
 *         the disc at u; that point is at t = <C, D> / Dz;
 *   caps  u = 0 and u = 1 when the ray meets the end disc (F <= 0); where
 *         the end tangent vanishes the disc is normal to its limit direction
 *         (the next control-polygon edge from that end);
 *   inside the origin lies in a disc: a root of <C, D> with |C| <= r (t = 0);
 *   planar when Dz vanishes identically (every disc plane contains the ray
 *         direction), the ray lies in the disc at the roots of
 *         <(Cx, Cy), (Dx, Dy)> and enters it at Cz - sqrt(r^2 - Cx^2 - Cy^2);
 *   edge-on when every disc plane lies within 1e-6 rad of the ray (a curve
 *         in a plane nearly normal to the ray), the side roots come from the
 *         two factors of F (see edge_on_sides), whose roots F's expanded
 *         coefficients cannot separate.
 * Every candidate lies in the solid, and the first point of the solid along
 * the ray is one of them as long as no disc passes through a focal point of
 * the sweep (radius below the radius of curvature: the "thin fiber"
 * condition of Section 3.4). Roots are isolated in Bernstein form by de
 * Casteljau subdivision with Descartes' rule of signs (variation
 * diminishing), then bisected to the last bit with the function evaluated
 * in extended precision (long double).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXDEG 10

/* Bernstein coefficients on [0,1], in extended precision: near a ray that is
 * almost parallel to the disc planes, F only dips below zero by ~1e-17 of
 * coefficients of order 1e-2, which double rounding would hide. */
typedef long double real;
typedef struct { real c[MAXDEG + 1]; int n; } bpoly;

static real binom(int n, int k)
{
    real r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static bpoly bmul(const bpoly *a, const bpoly *b)
{
    bpoly r;
    r.n = a->n + b->n;
    for (int k = 0; k <= r.n; ++k) r.c[k] = 0.0;
    for (int i = 0; i <= a->n; ++i)
        for (int j = 0; j <= b->n; ++j)
            r.c[i + j] += binom(a->n, i) * binom(b->n, j) / binom(r.n, i + j) * a->c[i] * b->c[j];
    return r;
}

static bpoly belevate(const bpoly *a, int n)
{
    /* degree elevation of a to degree n */
    bpoly r = *a;
    while (r.n < n) {
        bpoly e;
        e.n = r.n + 1;
        for (int k = 0; k <= e.n; ++k) {
            const real w = (real)k / e.n;
            e.c[k] = (k > 0 ? w * r.c[k - 1] : 0.0L) + (k < e.n ? (1.0L - w) * r.c[k] : 0.0L);
        }
        r = e;
    }
    return r;
}

static bpoly badd(const bpoly *a, const bpoly *b, real sb)
{
    const int n = a->n > b->n ? a->n : b->n;
    bpoly x = belevate(a, n), y = belevate(b, n), r;
    r.n = n;
    for (int k = 0; k <= n; ++k) r.c[k] = x.c[k] + sb * y.c[k];
    return r;
}

/* split a Bernstein polynomial on [0,1] at 1/2 (de Casteljau) */
static void bsplit(const bpoly *a, bpoly *L, bpoly *R)
{
    real w[MAXDEG + 1];
    const int n = a->n;
    memcpy(w, a->c, sizeof(real) * (n + 1));
    L->n = R->n = n;
    for (int k = 0; k <= n; ++k) {
        L->c[k] = w[0];
        R->c[n - k] = w[n - k];
        for (int i = 0; i < n - k; ++i) w[i] = 0.5L * (w[i] + w[i + 1]);
    }
}

static int sign_changes(const bpoly *a)
{
    int changes = 0, last = 0;
    for (int k = 0; k <= a->n; ++k) {
        const int s = a->c[k] > 0.0L ? 1 : (a->c[k] < 0.0L ? -1 : 0);
        if (s == 0) continue;
        if (last != 0 && s != last) changes++;
        last = s;
    }
    return changes;
}

/* ------------------------------------------------------------------------ */
/* Curve in the ray frame                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double q[4][4];     /* control points: x, y, z, r */
} curve_t;

static void eval(const curve_t *c, double u, double C[4], double D[3])
{
    const double v = 1.0 - u;
    const double b[4] = {v * v * v, 3 * u * v * v, 3 * u * u * v, u * u * u};
    const double e[3] = {v * v, 2 * u * v, u * u};
    for (int k = 0; k < 4; ++k) {
        C[k] = 0.0;
        for (int j = 0; j < 4; ++j) C[k] += b[j] * c->q[j][k];
    }
    for (int k = 0; k < 3; ++k) {
        D[k] = 0.0;
        for (int j = 0; j < 3; ++j) D[k] += e[j] * (c->q[j + 1][k] - c->q[j][k]);
    }
}

/* F(u) evaluated from the curve directly, in long double */
static long double F_ld(const curve_t *c, long double u)
{
    const long double v = 1.0L - u;
    const long double b[4] = {v * v * v, 3 * u * v * v, 3 * u * u * v, u * u * u};
    const long double e[3] = {v * v, 2 * u * v, u * u};
    long double C[4] = {0, 0, 0, 0}, D[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j) C[k] += b[j] * (long double)c->q[j][k];
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) D[k] += e[j] * ((long double)c->q[j + 1][k] - (long double)c->q[j][k]);
    const long double xy = C[0] * D[0] + C[1] * D[1];
    return D[2] * D[2] * (C[0] * C[0] + C[1] * C[1]) + xy * xy - C[3] * C[3] * D[2] * D[2];
}

static long double G_ld(const curve_t *c, long double u)
{
    const long double v = 1.0L - u;
    const long double b[4] = {v * v * v, 3 * u * v * v, 3 * u * u * v, u * u * u};
    const long double e[3] = {v * v, 2 * u * v, u * u};
    long double C[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 4; ++j) C[k] += b[j] * (long double)c->q[j][k];
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) D[k] += e[j] * ((long double)c->q[j + 1][k] - (long double)c->q[j][k]);
    return C[0] * D[0] + C[1] * D[1] + C[2] * D[2];
}

/* <(Cx, Cy), (Dx, Dy)>: zero where the ray line lies in a disc plane that
 * contains the ray direction */
static long double XY_ld(const curve_t *c, long double u)
{
    const long double v = 1.0L - u;
    const long double b[4] = {v * v * v, 3 * u * v * v, 3 * u * u * v, u * u * u};
    const long double e[3] = {v * v, 2 * u * v, u * u};
    long double C[2] = {0, 0}, D[2] = {0, 0};
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 4; ++j) C[k] += b[j] * (long double)c->q[j][k];
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 3; ++j) D[k] += e[j] * ((long double)c->q[j + 1][k] - (long double)c->q[j][k]);
    return C[0] * D[0] + C[1] * D[1];
}

/* The factors of F for an edge-on ray: g_s(u) = xy - s Dz sqrt(r^2 - rho^2)
 * (s = +1 or -1), where F = -g_{+1} g_{-1}. A root of g_s with rho <= r is a
 * point of the ray on the boundary circle of the disc at u, at
 * t = Cz + s sqrt(r^2 - rho^2). *ok is 0 outside rho <= r. */
static long double gs_ld(const curve_t *c, long double u, int s, int *ok, long double *t)
{
    const long double v = 1.0L - u;
    const long double b[4] = {v * v * v, 3 * u * v * v, 3 * u * u * v, u * u * u};
    const long double e[3] = {v * v, 2 * u * v, u * u};
    long double C[4] = {0, 0, 0, 0}, D[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 4; ++j) C[k] += b[j] * (long double)c->q[j][k];
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) D[k] += e[j] * ((long double)c->q[j + 1][k] - (long double)c->q[j][k]);
    const long double rest = C[3] * C[3] - C[0] * C[0] - C[1] * C[1];
    *ok = rest >= 0.0L;
    const long double sr = *ok ? sqrtl(rest) : 0.0L;
    if (t) *t = C[2] + s * sr;
    return C[0] * D[0] + C[1] * D[1] - s * D[2] * sr;
}

/* Is the ray edge-on to the curve: every disc plane within 1e-6 rad of the
 * ray direction (|C'z| <= 1e-6 |C'| wherever C' does not vanish)? Checked at
 * 257 parameters. */
static int edge_on(const curve_t *c)
{
    for (int k = 0; k <= 256; ++k) {
        const double u = k / 256.0, v = 1.0 - u;
        const double e[3] = {v * v, 2 * u * v, u * u};
        double D[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[i] += e[j] * (c->q[j + 1][i] - c->q[j][i]);
        const double dn = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        if (fabs(D[2]) > 1e-6 * dn) return 0;
    }
    return 1;
}

/* Side points of an edge-on ray: crossings of g_{+1} and g_{-1} where
 * rho <= r, found on 2^14 + 1 parameters and bisected in long double. Near
 * each zero of xy each factor crosses once, so the entry and the exit of
 * the disc there (1e-9 apart in u) are found separately. The earliest
 * t in [0, tmax) is kept in (best, bu). */
static void edge_on_sides(const curve_t *c, double tmax, double *best, double *bu)
{
    double scale = 0.0;
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k) scale = fmax(scale, fabs(c->q[j][k]));
    enum { N = 1 << 14 };
    for (int s = -1; s <= 1; s += 2) {
        int pok;
        long double pg = gs_ld(c, 0.0L, s, &pok, NULL);
        for (int k = 1; k <= N; ++k) {
            const long double u = (long double)k / N;
            int cok;
            const long double cg = gs_ld(c, u, s, &cok, NULL);
            if (pok && cok && (pg < 0.0L) != (cg < 0.0L)) {
                long double lo = (long double)(k - 1) / N, hi = u, glo = pg;
                for (int it = 0; it < 200; ++it) {
                    const long double mid = 0.5L * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    int mok;
                    const long double gm = gs_ld(c, mid, s, &mok, NULL);
                    if (!mok) break;
                    if ((gm < 0.0L) == (glo < 0.0L)) { lo = mid; glo = gm; }
                    else hi = mid;
                }
                long double t;
                int tok;
                gs_ld(c, 0.5L * (lo + hi), s, &tok, &t);
                /* where C' vanishes (a stalled end) g_s vanishes with it:
                 * no disc plane, no boundary point */
                double Cu[4], Du[3];
                eval(c, (double)(0.5L * (lo + hi)), Cu, Du);
                const int has_disc = sqrt(Du[0] * Du[0] + Du[1] * Du[1] + Du[2] * Du[2]) > 1e-12 * scale;
                if (tok && has_disc && t >= 0.0L && t < tmax && t < *best) {
                    *best = (double)t;
                    *bu = (double)(0.5L * (lo + hi));
                }
            }
            pg = cg;
            pok = cok;
        }
    }
}

typedef long double (*fn_t)(const curve_t *, long double);

/* Root of f in [a, b] where f(a) and f(b) differ in sign: bisection to the
 * last bit of long double. */
static double bisect(const curve_t *c, fn_t f, double a, double b)
{
    long double lo = a, hi = b;
    long double flo = f(c, lo);
    for (int it = 0; it < 200 && hi - lo > 0; ++it) {
        const long double mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const long double fm = f(c, mid);
        if (fm == 0.0L) return (double)mid;
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; }
        else hi = mid;
    }
    return (double)(0.5L * (lo + hi));
}

/* Collect roots of the Bernstein polynomial p (of function f) on [a, b]. */
static void isolate(const curve_t *c, fn_t f, const bpoly *p, double a, double b,
                    double *roots, int *nr, int maxr, int depth)
{
    if (*nr >= maxr) return;
    const int sc = sign_changes(p);
    if (sc == 0) {
        /* an exact zero coefficient at an end is a root at that end */
        if (p->c[0] == 0.0L && a == 0.0) roots[(*nr)++] = 0.0;
        if (*nr < maxr && p->c[p->n] == 0.0L && b == 1.0) roots[(*nr)++] = 1.0;
        return;
    }
    if (sc == 1 && p->c[0] != 0.0L && p->c[p->n] != 0.0L) {
        roots[(*nr)++] = bisect(c, f, a, b);
        return;
    }
    if (depth > 60 || b - a < 1e-15) {           /* cluster of roots: report its centre */
        roots[(*nr)++] = 0.5 * (a + b);
        return;
    }
    bpoly L, R;
    bsplit(p, &L, &R);
    const double m = 0.5 * (a + b);
    isolate(c, f, &L, a, m, roots, nr, maxr, depth + 1);
    isolate(c, f, &R, m, b, roots, nr, maxr, depth + 1);
}

/* candidate t of the disc at u: the ray point in the disc plane. From the
 * plane, t = <C, D> / Dz; on the boundary circle the same point is also
 * Cz +- sqrt(r^2 - Cx^2 - Cy^2), which stays well conditioned when the disc
 * plane is nearly parallel to the ray (Dz -> 0). For a point known to lie on
 * the circle (a root of F) the form with the smaller rounding estimate is
 * used; an end-cap point may lie anywhere in the disc, so it uses the plane.
 * F (if requested) is evaluated in long double. */
static int disc_t(const curve_t *c, double u, int on_circle, double *t, double *Fout)
{
    double C[4], D[3];
    eval(c, u, C, D);
    const double dn = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (!(dn > 0.0)) return 0;
    const double xy = C[0] * D[0] + C[1] * D[1];
    const double cn = sqrt(C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
    const double rest = C[3] * C[3] - C[0] * C[0] - C[1] * C[1];
    const double err_div = D[2] != 0.0 ? cn * dn / fabs(D[2]) : INFINITY;
    double err_sq = INFINITY, tsq = 0.0;
    /* a point of the ray on the disc's circle needs rho <= r: a root of F
     * reported where rho clearly exceeds r is a cluster of rounding (F's
     * positive dip below its coefficients' resolution), not a boundary point */
    if (on_circle && rest < -1e-9 * C[3] * C[3] - 1e-15 * (C[0] * C[0] + C[1] * C[1])) return 0;
    if (on_circle && rest >= 0.0) {
        const double sr = sqrt(rest);
        const double tm = C[2] - sr, tp = C[2] + sr;
        /* the sign that satisfies the plane equation (t - Cz) Dz = xy */
        tsq = fabs((tm - C[2]) * D[2] - xy) <= fabs((tp - C[2]) * D[2] - xy) ? tm : tp;
        err_sq = C[3] * C[3] / fmax(sr, 1e-300);
    }
    if (err_div == INFINITY && err_sq == INFINITY) return 0;
    *t = err_sq < err_div ? tsq : (xy + C[2] * D[2]) / D[2];
    if (Fout) *Fout = (double)F_ld(c, u);
    return 1;
}

/* Normal of the end disc at u = e (0 or 1): the end tangent, or where it is
 * negligible (squared length at most 2^-40 of the squared chord) the next
 * control-polygon edge from that end, then the chord -- the limit of the
 * tangent direction at the end. */
static void end_normal(const curve_t *c, int e, double n[3])
{
    const double (*q)[4] = c->q;
    double a[3], cand[3][3];
    for (int k = 0; k < 3; ++k) {
        a[k] = q[3][k] - q[0][k];
        cand[0][k] = e == 0 ? q[1][k] - q[0][k] : q[3][k] - q[2][k];
        cand[1][k] = e == 0 ? q[2][k] - q[0][k] : q[3][k] - q[1][k];
        cand[2][k] = a[k];
    }
    const double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    int j = 0;
    while (j < 2 && cand[j][0] * cand[j][0] + cand[j][1] * cand[j][1] + cand[j][2] * cand[j][2] <= 0x1p-40 * aa)
        ++j;
    for (int k = 0; k < 3; ++k) n[k] = cand[j][k];
}

/* Does the ray meet the end disc at u = e, and where: the ray point in the
 * disc's plane, inside the disc when its distance to C(e) is at most r(e)
 * (evaluated in long double: F of the side polynomial with the disc normal
 * in place of C', which is homogeneous in it). */
static int end_disc(const curve_t *c, int e, double *t)
{
    double n[3];
    end_normal(c, e, n);
    if (n[2] == 0.0) return 0;
    const long double Cx = c->q[3 * e][0], Cy = c->q[3 * e][1], Cz = c->q[3 * e][2], r = c->q[3 * e][3];
    const long double xy = Cx * n[0] + Cy * n[1];
    const long double nz = n[2];
    const long double F = nz * nz * (Cx * Cx + Cy * Cy) + xy * xy - r * r * nz * nz;
    if (F > 0.0L) return 0;
    *t = (double)((xy + Cz * nz) / nz);
    return 1;
}

/* Side points about the discs that nearly contain the ray. At a zero u0 of
 * xy (where a disc plane contains the ray line's direction, or nearly so)
 * with rho < r, F = -g_{+1} g_{-1} has two roots about u0: the ray enters
 * and leaves the disc of u0's neighbourhood there, on its circle at
 * t = Cz -+ sqrt(r^2 - rho^2). The roots lie about |Dz| sqrt(r^2 - rho^2) /
 * |xy'| from u0; when the disc plane turns towards the ray (Dz -> 0) they
 * merge below the rounding of F's coefficients, and F's sign pattern can
 * lose one or both. Each factor g_s changes sign once near u0: its sign
 * change is bracketed by widening steps from u0 and bisected in long
 * double. Points where C' vanishes are not boundary points (no disc). */
static void near_edge_on_sides(const curve_t *c, const bpoly *xy, double scale, double tmax,
                               double *best, double *bu)
{
    double z[64];
    int nz = 0;
    isolate(c, XY_ld, xy, 0.0, 1.0, z, &nz, 64, 0);
    for (int i = 0; i < nz; ++i) {
        double Cu[4], Du[3];
        eval(c, z[i], Cu, Du);
        if (!(sqrt(Du[0] * Du[0] + Du[1] * Du[1] + Du[2] * Du[2]) > 1e-12 * scale)) continue;
        for (int s = -1; s <= 1; s += 2) {
            int ok0;
            const long double g0 = gs_ld(c, z[i], s, &ok0, NULL);
            if (!ok0) continue;
            long double lo = z[i], hi = z[i], glo = g0;
            int found = g0 == 0.0L;
            for (double w = 0x1p-44; !found && w <= 0x1p-6; w *= 4.0) {
                for (int side = -1; side <= 1 && !found; side += 2) {
                    const double ub = z[i] + side * w;
                    if (ub < 0.0 || ub > 1.0) continue;
                    int okb;
                    const long double gb = gs_ld(c, ub, s, &okb, NULL);
                    if (okb && (gb < 0.0L) != (g0 < 0.0L)) {
                        lo = z[i];
                        hi = ub;
                        found = 1;
                    }
                }
            }
            if (!found) continue;
            /* bisected to adjacent long doubles, rho <= r all the way */
            int conv = glo == 0.0L;
            for (int it = 0; it < 200 && !conv; ++it) {
                const long double mid = 0.5L * (lo + hi);
                if (mid == lo || mid == hi) { conv = 1; break; }
                int okm;
                const long double gm = gs_ld(c, mid, s, &okm, NULL);
                if (!okm) break;
                if (gm == 0.0L) { lo = hi = mid; conv = 1; break; }
                if ((gm < 0.0L) == (glo < 0.0L)) { lo = mid; glo = gm; }
                else hi = mid;
            }
            if (!conv) continue;
            const double ur = (double)(0.5L * (lo + hi));
            double Cr[4], Dr[3];
            eval(c, ur, Cr, Dr);
            if (!(sqrt(Dr[0] * Dr[0] + Dr[1] * Dr[1] + Dr[2] * Dr[2]) > 1e-12 * scale)) continue;
            int okt;
            long double t;
            gs_ld(c, ur, s, &okt, &t);
            if (okt && t >= 0.0L && t < tmax && t < *best) { *best = (double)t; *bu = ur; }
        }
    }
}

/* Exact first entry; kind: 0 miss, 1 side, 2 start cap, 3 end cap, 4 inside */
static int exact_hit(const curve_t *c, double tmax, double *t_out, double *u_out)
{
    /* Bernstein forms of Cx, Cy, Cz, r (degree 3) and Dx, Dy, Dz (degree 2) */
    bpoly C[4], D[3];
    for (int k = 0; k < 4; ++k) {
        C[k].n = 3;
        for (int j = 0; j < 4; ++j) C[k].c[j] = c->q[j][k];
    }
    for (int k = 0; k < 3; ++k) {
        D[k].n = 2;
        for (int j = 0; j < 3; ++j) D[k].c[j] = c->q[j + 1][k] - c->q[j][k];
    }
    const bpoly Dz2 = bmul(&D[2], &D[2]);
    const bpoly Cx2 = bmul(&C[0], &C[0]), Cy2 = bmul(&C[1], &C[1]);
    const bpoly rho = badd(&Cx2, &Cy2, 1.0);
    const bpoly a1 = bmul(&Dz2, &rho);
    const bpoly cxdx = bmul(&C[0], &D[0]), cydy = bmul(&C[1], &D[1]);
    const bpoly xy = badd(&cxdx, &cydy, 1.0);
    const bpoly a2 = bmul(&xy, &xy);
    const bpoly r2 = bmul(&C[3], &C[3]);
    const bpoly a3 = bmul(&r2, &Dz2);
    bpoly F = badd(&a1, &a2, 1.0);
    F = badd(&F, &a3, -1.0);

    double best = INFINITY, bu = NAN;
    int kind = 0;

    /* origin inside the solid */
    const bpoly czdz = bmul(&C[2], &D[2]);
    bpoly G = badd(&xy, &czdz, 1.0);
    double groots[64];
    int ng = 0;
    isolate(c, G_ld, &G, 0.0, 1.0, groots, &ng, 64, 0);
    for (int i = 0; i < ng; ++i) {
        double Cu[4], Du[3];
        eval(c, groots[i], Cu, Du);
        if (Cu[0] * Cu[0] + Cu[1] * Cu[1] + Cu[2] * Cu[2] <= Cu[3] * Cu[3]) {
            *t_out = 0.0;
            *u_out = groots[i];
            return tmax > 0.0 ? 4 : 0;
        }
    }

    /* every disc plane contains the ray direction (C'z == 0 identically, e.g.
     * a straight fiber or a curve in a plane normal to the ray): the ray lies
     * in the disc at u exactly where <(Cx, Cy), (Dx, Dy)> = 0, and enters it
     * at t = Cz - sqrt(r^2 - Cx^2 - Cy^2) */
    if (D[2].c[0] == 0.0 && D[2].c[1] == 0.0 && D[2].c[2] == 0.0) {
        double proots[64];
        int np = 0;
        isolate(c, XY_ld, &xy, 0.0, 1.0, proots, &np, 64, 0);
        for (int i = 0; i < np; ++i) {
            double Cu[4], Du[3];
            eval(c, proots[i], Cu, Du);
            const double rest = Cu[3] * Cu[3] - Cu[0] * Cu[0] - Cu[1] * Cu[1];
            if (rest < 0.0) continue;
            const double t = Cu[2] - sqrt(rest);
            if (t >= 0.0 && t < tmax && t < best) { best = t; bu = proots[i]; kind = 1; }
        }
        *t_out = best;
        *u_out = bu;
        return kind;
    }

    /* side surface */
    double roots[128];
    int nr = 0;
    const int eo = edge_on(c);
    if (eo) {
        /* F's two roots about each zero of xy are then closer than the
         * rounding of its coefficients resolves: use its factors */
        double bs = INFINITY, bus = NAN;
        edge_on_sides(c, tmax, &bs, &bus);
        if (bs < best) { best = bs; bu = bus; kind = 1; }
    } else {
        isolate(c, F_ld, &F, 0.0, 1.0, roots, &nr, 128, 0);
    }
    double scale = 0.0;
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k) scale = fmax(scale, fabs(c->q[j][k]));
    if (!eo) {
        double bs = INFINITY, bus = NAN;
        near_edge_on_sides(c, &xy, scale, tmax, &bs, &bus);
        if (bs < best) { best = bs; bu = bus; kind = 1; }
    }
    for (int i = 0; i < nr; ++i) {
        double t;
        double Cu[4], Du[3];
        eval(c, roots[i], Cu, Du);
        const double dn = sqrt(Du[0] * Du[0] + Du[1] * Du[1] + Du[2] * Du[2]);
        if (dn <= 1e-12 * (scale + 1e-300)) continue;      /* cusp: F vanishes with C' */
        if (!disc_t(c, roots[i], 1, &t, NULL)) continue;
        if (t >= 0.0 && t < tmax && t < best) { best = t; bu = roots[i]; kind = 1; }
    }
    /* end caps: the disc at u = 0 (1) lies in the plane normal to the end
     * tangent. Where that tangent vanishes (p1 = p0 or p2 = p3) the disc
     * planes of the nearby u still converge: to the plane normal to the
     * first non-negligible of p2 - p0, p3 - p0 (p3 - p1, p3 - p0), the
     * direction C'(u) takes as u approaches the end. */
    for (int e = 0; e < 2; ++e) {
        double t;
        if (!end_disc(c, e, &t)) continue;
        if (t >= 0.0 && t < tmax && t < best) { best = t; bu = (double)e; kind = 2 + e; }
    }
    *t_out = best;
    *u_out = bu;
    return kind;
}

/* Outward unit normal of the solid at the entry (ray frame).
 * Side (kind 1): the side surface is X(u, phi) = C(u) + r(u) e(u, phi) with e
 * a unit vector normal to C'(u). Its normal is normal to the circle's
 * tangent, so it lies in the plane of e and T = C'/|C'|; being normal to
 * dX/du = C' + r' e + r de/du as well, with <T, de/du> = -<e, C''>/|C'|,
 * it is e - r' / (|C'| - r <e, C''>/|C'|) T (a cone's tilt against its
 * widening; zero for a constant radius). e is the unit direction from C(u)
 * to the entry point (0, 0, t).
 * Caps (kinds 2, 3): minus the start disc's normal, the end disc's normal.
 * Origin inside (kind 4): no surface crossing, NaN. */
static void exact_normal(const curve_t *c, int kind, double t, double u, double n[3])
{
    n[0] = n[1] = n[2] = NAN;
    if (kind == 2 || kind == 3) {
        end_normal(c, kind - 2, n);
        const double s = (kind == 2 ? -1.0 : 1.0) / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) n[k] *= s;
        return;
    }
    if (kind != 1) return;
    const double (*q)[4] = c->q;
    const double v = 1.0 - u;
    double C[4], D1[4], D2[3];
    for (int k = 0; k < 4; ++k) {
        C[k] = v * v * v * q[0][k] + 3.0 * u * v * v * q[1][k] + 3.0 * u * u * v * q[2][k] + u * u * u * q[3][k];
        D1[k] = 3.0 * (v * v * (q[1][k] - q[0][k]) + 2.0 * u * v * (q[2][k] - q[1][k]) + u * u * (q[3][k] - q[2][k]));
        if (k < 3)
            D2[k] = 6.0 * (v * (q[2][k] - 2.0 * q[1][k] + q[0][k]) + u * (q[3][k] - 2.0 * q[2][k] + q[1][k]));
    }
    double e[3] = {-C[0], -C[1], t - C[2]};
    const double el = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double dl = sqrt(D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2]);
    for (int k = 0; k < 3; ++k) e[k] /= el;
    const double ec2 = e[0] * D2[0] + e[1] * D2[1] + e[2] * D2[2];
    const double beta = -D1[3] / (dl - C[3] * ec2 / dl);
    double len = 0.0;
    for (int k = 0; k < 3; ++k) {
        n[k] = e[k] + beta * D1[k] / dl;
        len += n[k] * n[k];
    }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) n[k] /= len;
}

/* Duff et al. 2017 basis (same published construction as the depth oracle;
 * repeated here so that this file stands alone). */
static void onb_x(const double w[3], double u[3], double v[3])
{
    const double s = copysign(1.0, w[2]);
    const double a = -1.0 / (s + w[2]);
    const double b = w[0] * w[1] * a;
    u[0] = 1.0 + s * w[0] * w[0] * a;  u[1] = s * b;  u[2] = -s * w[0];
    v[0] = b;  v[1] = s + w[1] * w[1] * a;  v[2] = -w[1];
}

/* n_out (may be NULL): the unit normal at the entry in world space (NaN on a
 * miss or with the origin inside). */
int fx_intersect(const double ray[7], const double fiber[16], double *t_out, double *u_out,
                 double n_out[3])
{
    *t_out = INFINITY;
    *u_out = NAN;
    if (n_out) n_out[0] = n_out[1] = n_out[2] = NAN;
    const double *O = ray, *Dr = ray + 3;
    const double len = sqrt(Dr[0] * Dr[0] + Dr[1] * Dr[1] + Dr[2] * Dr[2]);
    if (!(len > 0.0) || !isfinite(len) || !(ray[6] == ray[6])) return 0;
    const double w[3] = {Dr[0] / len, Dr[1] / len, Dr[2] / len};
    double u[3], v[3];
    onb_x(w, u, v);
    curve_t c;
    for (int k = 0; k < 4; ++k) {
        const double d0 = fiber[4 * k] - O[0], d1 = fiber[4 * k + 1] - O[1], d2 = fiber[4 * k + 2] - O[2];
        c.q[k][0] = d0 * u[0] + d1 * u[1] + d2 * u[2];
        c.q[k][1] = d0 * v[0] + d1 * v[1] + d2 * v[2];
        c.q[k][2] = d0 * w[0] + d1 * w[1] + d2 * w[2];
        c.q[k][3] = fiber[4 * k + 3];
    }
    double t, uu;
    const int kind = exact_hit(&c, ray[6], &t, &uu);
    if (kind == 0) return 0;
    *t_out = t;
    *u_out = uu;
    if (n_out) {
        double n[3];
        exact_normal(&c, kind, t, uu, n);
        for (int k = 0; k < 3; ++k) n_out[k] = n[0] * u[k] + n[1] * v[k] + n[2] * w[k];
    }
    return kind;
}

void fx_batch(const float *rays, int64_t ray_stride, int64_t n_rays,
              const float *fibers, int64_t fiber_stride, int64_t n_fibers,
              const int32_t *pair_ray, const int32_t *pair_fiber, int64_t n,
              double radius_scale, double *t_out, double *u_out, int32_t *kind_out,
              int nthreads, double *normal_out)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ri = pair_ray ? pair_ray[i] : i;
        const int64_t fi = pair_fiber ? pair_fiber[i] : i;
        double ray[7], fib[16], t = INFINITY, u = NAN, nn[3] = {NAN, NAN, NAN};
        int kind = 0;
        if (ri >= 0 && ri < n_rays && fi >= 0 && fi < n_fibers) {
            for (int r = 0; r < 7; ++r) ray[r] = rays[r * ray_stride + ri];
            for (int r = 0; r < 16; ++r) fib[r] = fibers[r * fiber_stride + fi];
            for (int k = 0; k < 4; ++k) fib[4 * k + 3] *= radius_scale;
            kind = fx_intersect(ray, fib, &t, &u, nn);
        }
        if (normal_out)
            for (int k = 0; k < 3; ++k) normal_out[3 * i + k] = nn[k];
        t_out[i] = t;
        u_out[i] = u;
        kind_out[i] = kind;
    }
}

/* Quadratic fibers (12 rows: p0, p1, p2, each x, y, z, r): the swept solid
 * of a quadratic is that of its exact cubic elevation. */
void fx_batch_quad(const float *rays, int64_t ray_stride, int64_t n_rays,
                   const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                   const int32_t *pair_ray, const int32_t *pair_fiber, int64_t n,
                   double radius_scale, double *t_out, double *u_out, int32_t *kind_out,
                   int nthreads, double *normal_out)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ri = pair_ray ? pair_ray[i] : i;
        const int64_t fi = pair_fiber ? pair_fiber[i] : i;
        double ray[7], p[12], fib[16], t = INFINITY, u = NAN, nn[3] = {NAN, NAN, NAN};
        int kind = 0;
        if (ri >= 0 && ri < n_rays && fi >= 0 && fi < n_fibers) {
            for (int r = 0; r < 7; ++r) ray[r] = rays[r * ray_stride + ri];
            for (int r = 0; r < 12; ++r) p[r] = fibers[r * fiber_stride + fi];
            for (int k = 0; k < 3; ++k) p[4 * k + 3] *= radius_scale;
            for (int c = 0; c < 4; ++c) {
                fib[c] = p[c];
                fib[4 + c] = (p[c] + 2.0 * p[4 + c]) / 3.0;
                fib[8 + c] = (2.0 * p[4 + c] + p[8 + c]) / 3.0;
                fib[12 + c] = p[8 + c];
            }
            kind = fx_intersect(ray, fib, &t, &u, nn);
        }
        t_out[i] = t;
        u_out[i] = u;
        kind_out[i] = kind;
        if (normal_out)
            for (int k = 0; k < 3; ++k) normal_out[3 * i + k] = nn[k];
    }
}

/* Nearest entry over a candidate list per ray (the exact counterpart of
 * fo_nearest_d): candidates in list order, each against the ray shortened to
 * the latest entry found; the first of equal entries is kept. */
void fx_nearest(const float *rays, int64_t ray_stride, int64_t n_rays,
                const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                const int64_t *off, const int32_t *cand, int max_cand, double radius_scale,
                double *t_out, double *u_out, int32_t *kind_out, int32_t *fiber_out, int nthreads,
                double *normal_out)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t r = 0; r < n_rays; ++r) {
        double ray[7];
        for (int k = 0; k < 7; ++k) ray[k] = rays[k * ray_stride + r];
        double best_t = INFINITY, best_u = NAN, best_n[3] = {NAN, NAN, NAN};
        int best_kind = 0;
        int32_t best_f = -1;
        int64_t end = off[r + 1];
        if (end - off[r] > max_cand) end = off[r] + max_cand;
        for (int64_t j = off[r]; j < end; ++j) {
            const int64_t fi = cand[j];
            if (fi < 0 || fi >= n_fibers) continue;
            double fib[16], t, u, nn[3];
            for (int k = 0; k < 16; ++k) fib[k] = fibers[k * fiber_stride + fi];
            for (int k = 0; k < 4; ++k) fib[4 * k + 3] *= radius_scale;
            const int kind = fx_intersect(ray, fib, &t, &u, nn);
            if (kind) {
                best_t = t;
                best_u = u;
                best_kind = kind;
                best_f = (int32_t)fi;
                for (int k = 0; k < 3; ++k) best_n[k] = nn[k];
                ray[6] = t;
            }
        }
        t_out[r] = best_t;
        u_out[r] = best_u;
        kind_out[r] = best_kind;
        fiber_out[r] = best_f;
        if (normal_out)
            for (int k = 0; k < 3; ++k) normal_out[3 * r + k] = best_n[k];
    }
}

/* Bernstein coefficients of F for a curve given in the ray frame (pins). */
int fx_side_polynomial(const double q16[16], double coef[MAXDEG + 1])
{
    curve_t c;
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k) c.q[j][k] = q16[4 * j + k];
    bpoly C[4], D[3];
    for (int k = 0; k < 4; ++k) { C[k].n = 3; for (int j = 0; j < 4; ++j) C[k].c[j] = c.q[j][k]; }
    for (int k = 0; k < 3; ++k) { D[k].n = 2; for (int j = 0; j < 3; ++j) D[k].c[j] = c.q[j + 1][k] - c.q[j][k]; }
    const bpoly Dz2 = bmul(&D[2], &D[2]);
    const bpoly Cx2 = bmul(&C[0], &C[0]), Cy2 = bmul(&C[1], &C[1]);
    const bpoly rho = badd(&Cx2, &Cy2, 1.0);
    const bpoly a1 = bmul(&Dz2, &rho);
    const bpoly cxdx = bmul(&C[0], &D[0]), cydy = bmul(&C[1], &D[1]);
    const bpoly xy = badd(&cxdx, &cydy, 1.0);
    const bpoly a2 = bmul(&xy, &xy);
    const bpoly r2 = bmul(&C[3], &C[3]);
    const bpoly a3 = bmul(&r2, &Dz2);
    bpoly F = badd(&a1, &a2, 1.0);
    F = badd(&F, &a3, -1.0);
    for (int k = 0; k <= MAXDEG; ++k) coef[k] = F.c[k];
    return F.n;
}
