/*
 * TEST INFRASTRUCTURE -- FP64 CPU oracle for the ray/fiber intersection of
 * Binder & Keller, "Fast, High Precision Ray/Fiber Intersection using Tight,
 * Disjoint Bounding Volumes" (arXiv 1811.03374).
 *
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg load this library. The product (HIP) path never calls it and shares no
 * code, header, table or helper with it.
 *
 * What it computes ("ORACLE-D(d)"): the paper's depth-d method executed in
 * IEEE double precision, written as the recursion that the paper's bit string
 * encodes (Section 3.3, "Recursive subdivision is performed by an iterative
 * process ..."). Each node of the recursion is a cubic sub-curve held as its
 * four 4-D control points (position + radius, Section 3.3); children come from
 * de Casteljau subdivision at the domain centre (Appendix B.2). Per node:
 *
 *   1. conservative radius: largest distance of the two inner control points
 *      to the chord axis plus the largest radius control value (Section 3.3,
 *      convex hull property);
 *   2. unit ray against the infinite cylinder about the chord (Appendix A);
 *   3. visibility against the current t interval (Section 3.3, cropping by the
 *      end-cap planes; Section 3.2, cropping by split planes);
 *   4. at depth d: hit at the entry into the capped leaf cylinder, u from the
 *      projection of the hit point onto the chord (Section 3.3, last
 *      paragraph);
 *   5. otherwise split at u = 1/2 by the plane through the split point normal
 *      to the split tangent, visit first the half the ray meets first, and
 *      the other half only if the ray crosses the plane inside the cylinder
 *      (Section 3.2 and Fig. "bounding_cylinder"); a hit ends the search
 *      (instant termination, Section 3).
 *
 * Interval bookkeeping follows the paper's iteration exactly: descending into
 * the first child narrows the interval by the split plane; a second child is
 * reached by backtracking, and there the interval is recomputed from that
 * node's own end caps (Section 3.3: "one of the interval bounds is updated;
 * both are recalculated after backtracking").
 *
 * Readings where the paper is silent or its listings are inconsistent (each
 * also listed in the design notes):
 *   R1  leaf t = max(cylinder entry, interval start): the entry into the
 *       capped leaf cylinder, never before the cap plane nor behind the origin.
 *   R2  visible <=> max(t_entry, t_lo) <= min(t_exit, t_hi).
 *   R3  a plane whose normal is perpendicular to the ray (n.z == 0): the whole
 *       ray lies on the side given by the sign of <(0,0,t) - s, n>; a split
 *       sends the ray to that side without narrowing; a ray exactly in the
 *       plane visits both halves; a cap that excludes the ray empties the
 *       interval.
 *   R4  axis parallel to the ray (g == 0): inside -> (-inf, +inf), outside ->
 *       explicit miss.
 *   R5  misses are explicit flags, never (FLT_MAX, FLT_MAX) sentinels.
 *   R6  interval recomputation after backtracking uses the ray's tmax.
 *   R7  the radius channel passes through the ray-frame rotation unchanged.
 *   R8  the ray direction is normalised; t and tmax are distances along it.
 *   R11 hit <=> t < tmax (t >= 0 by construction).
 *   R12 depth d means leaves of parametric size 2^-d, 0 <= d <= 23.
 *   R13 a negligible tangent -- squared length at most 2^-40 of the squared
 *       chord q3 - q0, below which its direction is rounding noise (a zero
 *       end tangent, a cusp) -- is replaced for cap normals by the first
 *       non-negligible of (q1-q0, q2-q0, q3-q0) at the start and
 *       (q3-q2, q3-q1, q3-q0) at the end; a split tangent (1/8 of
 *       -q0 - q1 + q2 + q3, the children's tangent at the split point) by
 *       the chord as the split plane's normal, and the children take that
 *       tangent as exactly zero (a cusp: snap_cusp). A zero-length chord
 *       gives distances to the point q0.
 *   R14 the method's result is not continuous in its inputs: where a pruning
 *       or ordering comparison is a near tie, a rounding-sized perturbation
 *       selects another (equally valid) leaf. A comparison is a tie when its
 *       two sides differ by at most the error bound of an FP32 evaluation
 *       (see node_err and the *_err terms below); fo_tie_outcomes enumerates
 *       the results reachable by flipping such ties, and a lower-precision
 *       implementation must reproduce the unflipped result or one of these.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z, w; } v4;

static v4 mk4(double x, double y, double z, double w) { v4 r = {x, y, z, w}; return r; }
static v4 add4(v4 a, v4 b) { return mk4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
static v4 sub4(v4 a, v4 b) { return mk4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }
static v4 scale4(v4 a, double s) { return mk4(a.x * s, a.y * s, a.z * s, a.w * s); }
static double dot3(v4 a, v4 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static int zero3(v4 a) { return a.x == 0.0 && a.y == 0.0 && a.z == 0.0; }

/* ------------------------------------------------------------------------ */
/* Ray frame (Section 3.3): the ray starts at the origin and runs along +z.  */
/* ------------------------------------------------------------------------ */

/* Orthonormal basis (u, v) completing the unit vector w: Duff et al. 2017,
 * "Building an Orthonormal Basis, Revisited" (the revision of Frisvad's
 * method cited in Section 3.3). */
static void onb(const double w[3], double u[3], double v[3])
{
    const double s = copysign(1.0, w[2]);
    const double a = -1.0 / (s + w[2]);
    const double b = w[0] * w[1] * a;
    u[0] = 1.0 + s * w[0] * w[0] * a;  u[1] = s * b;  u[2] = -s * w[0];
    v[0] = b;  v[1] = s + w[1] * w[1] * a;  v[2] = -w[1];
}

/* Control points of one fiber in the frame of one ray. Returns 0 when the
 * ray direction is zero or not finite (then the pair is a miss). */
static int ray_frame(const double O[3], const double D[3], const double P[16],
                     v4 q[4], double *len_out, double frame[9])
{
    const double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (!(len > 0.0) || !isfinite(len)) return 0;
    const double w[3] = {D[0] / len, D[1] / len, D[2] / len};
    double u[3], v[3];
    onb(w, u, v);
    if (frame) {
        for (int k = 0; k < 3; ++k) { frame[k] = u[k]; frame[3 + k] = v[k]; frame[6 + k] = w[k]; }
    }
    for (int k = 0; k < 4; ++k) {
        const double d0 = P[4 * k + 0] - O[0];
        const double d1 = P[4 * k + 1] - O[1];
        const double d2 = P[4 * k + 2] - O[2];
        q[k] = mk4(d0 * u[0] + d1 * u[1] + d2 * u[2],
                   d0 * v[0] + d1 * v[1] + d2 * v[2],
                   d0 * w[0] + d1 * w[1] + d2 * w[2],
                   P[4 * k + 3]);
        if (!isfinite(q[k].x) || !isfinite(q[k].y) || !isfinite(q[k].z) || !isfinite(q[k].w))
            return 0;
    }
    if (len_out) *len_out = len;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Geometry of one node                                                      */
/* ------------------------------------------------------------------------ */

/* R13: a tangent whose squared length is at most 2^-40 of the squared chord
 * has no reliable direction. With a zero chord only the zero vector is
 * negligible. */
static int negligible(v4 v, v4 chord)
{
    return dot3(v, v) <= 0x1p-40 * dot3(chord, chord);
}

static v4 start_cap_normal(const v4 q[4])
{
    const v4 a = sub4(q[3], q[0]);
    v4 n = sub4(q[1], q[0]);
    if (negligible(n, a)) n = sub4(q[2], q[0]);
    if (negligible(n, a)) n = a;
    return n;
}

static v4 end_cap_normal(const v4 q[4])
{
    const v4 a = sub4(q[3], q[0]);
    v4 n = sub4(q[3], q[2]);
    if (negligible(n, a)) n = sub4(q[3], q[1]);
    if (negligible(n, a)) n = a;
    return n;
}

/* Error bound of the crossing t = <s, n> / n_z of a plane through s with
 * normal n, for node coordinates known to +-delta in an FP32 evaluation: the
 * point error seen along the ray through the plane's obliquity (the normal's
 * own error, relative to it, is of the same order and covered by the factor
 * 2), plus the rounding of the quotient. */
static double plane_err(double delta, v4 n, double t)
{
    return 2.0 * delta * sqrt(dot3(n, n)) / fabs(n.z) + 4.0 * 0x1p-24 * fabs(t);
}

/* t interval of the ray between the node's two end-cap planes, intersected
 * with [0, tmax] (Section 3.3, cropping of the infinite cylinders). The start
 * cap passes through q0 with the start tangent as normal (the curve lies on
 * its positive side); the end cap passes through q3 with the end tangent (the
 * curve lies on its negative side). The node is given as its first control
 * point o and the control points relative to it (see node_t). elo/ehi (may be
 * NULL) receive the error bounds of the two ends for node coordinates known
 * to +-delta (0 for the ends 0 and tmax). */
static void cap_interval_e(v4 o, const v4 q[4], double tmax, double delta, double *lo, double *hi,
                           double *elo, double *ehi)
{
    double l = 0.0, h = tmax, el = 0.0, eh = 0.0;
    const v4 n0 = start_cap_normal(q);
    const double c0 = dot3(o, n0) + dot3(q[0], n0);       /* inside <=> t*n0.z >= c0 */
    if (n0.z != 0.0) {
        const double t = c0 / n0.z;
        if (n0.z > 0.0 && t > l) { l = t; el = plane_err(delta, n0, t); }
        if (n0.z < 0.0 && t < h) { h = t; eh = plane_err(delta, n0, t); }
    } else if (c0 > 0.0) {
        l = INFINITY; h = -INFINITY;
    }
    const v4 n1 = end_cap_normal(q);
    const double c1 = dot3(o, n1) + dot3(q[3], n1);       /* inside <=> t*n1.z <= c1 */
    if (n1.z != 0.0) {
        const double t = c1 / n1.z;
        if (n1.z > 0.0 && t < h) { h = t; eh = plane_err(delta, n1, t); }
        if (n1.z < 0.0 && t > l) { l = t; el = plane_err(delta, n1, t); }
    } else if (c1 < 0.0) {
        l = INFINITY; h = -INFINITY;
    }
    *lo = l;
    *hi = h;
    if (elo) *elo = el;
    if (ehi) *ehi = eh;
}

/* Squared distance of point e (relative to the axis origin) to the line
 * through the origin along a; a zero axis gives the distance to the point. */
static double dist2_to_axis(v4 e, v4 a)
{
    const double c = dot3(a, a);
    if (c > 0.0) {
        const double b = dot3(e, a) / c;
        e = mk4(e.x - b * a.x, e.y - b * a.y, e.z - b * a.z, 0.0);
    }
    return dot3(e, e);
}

/* Conservative radius of the cylinder about the chord q0 -> q3 (Section 3.3):
 * the end points lie on the axis, so the two inner control points give the
 * largest distance of the control polygon; the radius Bezier is bounded by its
 * largest coefficient. */
static double conservative_radius(const v4 q[4])
{
    const v4 a = sub4(q[3], q[0]);
    const double d1 = dist2_to_axis(sub4(q[1], q[0]), a);
    const double d2 = dist2_to_axis(sub4(q[2], q[0]), a);
    const double rmax = fmax(fmax(q[0].w, q[1].w), fmax(q[2].w, q[3].w));
    return sqrt(fmax(d1, d2)) + rmax;
}

/* Quadratic fibers (Appendix B.1) are held as their exact cubic elevation
 * (q1 = (p0 + 2 p1) / 3, q2 = (2 p1 + p2) / 3, radius included): the same
 * curve and radius function, and de Casteljau halving commutes with
 * elevation, so the recursion, the split planes (normal to the tangent at
 * the centre, which for a quadratic is the chord p2 - p0) and the cap planes
 * are the quadratic's own. Only the bound is the quadratic's: the distance
 * of the middle control point p1 = (3 q1 - q0) / 2 = (3 q2 - q3) / 2 to the
 * chord (3/2 of the elevated inner points' distance) plus the largest of
 * the three radius control values. */
static double quadratic_radius(const v4 q[4])
{
    const v4 a = sub4(q[3], q[0]);
    const double d1 = dist2_to_axis(sub4(q[1], q[0]), a);
    const double d2 = dist2_to_axis(sub4(q[2], q[0]), a);
    const double r1a = 0.5 * (3.0 * q[1].w - q[0].w), r1b = 0.5 * (3.0 * q[2].w - q[3].w);
    const double rmax = fmax(fmax(q[0].w, q[3].w), fmax(r1a, r1b));
    return 1.5 * sqrt(fmax(d1, d2)) + rmax;
}

/* Exact cubic elevation of a quadratic (p0, p1, p2; x, y, z, r each). */
static void elevate_quadratic(const double p[12], double q[16])
{
    for (int c = 0; c < 4; ++c) {
        q[c] = p[c];
        q[4 + c] = (p[c] + 2.0 * p[4 + c]) / 3.0;
        q[8 + c] = (2.0 * p[4 + c] + p[8 + c]) / 3.0;
        q[12 + c] = p[8 + c];
    }
}

/* Unit ray (origin, +z) against the infinite cylinder of radius r whose axis
 * passes through o along a (Appendix A). With g = a.x^2 + a.y^2 the ray
 * meets it where e = r^2 - dist^2 >= 0 (dist: distance between the ray and
 * the axis line), over [t_cpa - s, t_cpa + s]. */
typedef struct {
    int parallel;          /* g == 0: axis parallel to the ray (R4) */
    double g, e, dist, t_cpa, s;
} cyl_t;

static cyl_t cylinder_terms(v4 o, v4 a, double r)
{
    cyl_t c;
    memset(&c, 0, sizeof c);
    c.g = a.x * a.x + a.y * a.y;
    if (c.g == 0.0) {
        c.parallel = 1;
        c.e = r * r - (o.x * o.x + o.y * o.y);
        return c;
    }
    const double dd = a.x * o.y - a.y * o.x;      /* sqrt(g) * ray-axis distance */
    c.dist = fabs(dd) / sqrt(c.g);
    c.e = r * r - dd * dd / c.g;
    c.t_cpa = o.z - a.z * (a.x * o.x + a.y * o.y) / c.g;
    c.s = c.e > 0.0 ? sqrt(c.e * (a.z * a.z + c.g) / c.g) : 0.0;
    return c;
}

/* Returns 0 on a miss. */
static int unit_ray_cylinder(v4 o, v4 a, double r, double *t0, double *t1)
{
    const cyl_t c = cylinder_terms(o, a, r);
    if (c.parallel) {
        if (c.e > 0.0) { *t0 = -INFINITY; *t1 = INFINITY; return 1; }
        return 0;
    }
    if (c.e < 0.0) return 0;
    *t0 = c.t_cpa - c.s;
    *t1 = c.t_cpa + c.s;
    return 1;
}

/* de Casteljau subdivision at u = 1/2 (Appendix B.2). */
static void split_half(const v4 q[4], v4 L[4], v4 R[4])
{
    const v4 m01 = scale4(add4(q[0], q[1]), 0.5);
    const v4 m12 = scale4(add4(q[1], q[2]), 0.5);
    const v4 m23 = scale4(add4(q[2], q[3]), 0.5);
    const v4 m012 = scale4(add4(m01, m12), 0.5);
    const v4 m123 = scale4(add4(m12, m23), 0.5);
    const v4 s = scale4(add4(m012, m123), 0.5);
    L[0] = q[0]; L[1] = m01; L[2] = m012; L[3] = s;
    R[0] = s; R[1] = m123; R[2] = m23; R[3] = q[3];
}

/* Normal of the partitioning plane: the curve tangent at the split point,
 * proportional to -q0 - q1 + q2 + q3 (Appendix B.2), which is 8 times the
 * children's tangent there; the chord when that tangent is negligible (R13). */
static v4 split_normal(const v4 q[4])
{
    v4 t = sub4(add4(q[2], q[3]), add4(q[0], q[1]));
    const v4 a = sub4(q[3], q[0]);
    if (negligible(scale4(t, 0.125), a)) t = a;
    return t;
}

/* A node of the recursion: its first control point o (xyz in the ray frame)
 * and its four control points relative to o (q[0] = 0; .w holds the radius
 * control values themselves). Subdividing relative points keeps a deep
 * node's shape at full relative precision: averaging absolute points would
 * round it at the magnitude of the node's position, which matters where the
 * parametrisation stalls (a zero end tangent makes the end nodes' chords
 * shrink like 4^-depth). In exact arithmetic this is de Casteljau's
 * subdivision of the absolute points. */
typedef struct {
    v4 o;
    v4 q[4];
} node_t;

static node_t anchored(const v4 qa[4])
{
    node_t n;
    n.o = mk4(qa[0].x, qa[0].y, qa[0].z, 0.0);
    for (int k = 0; k < 4; ++k) n.q[k] = mk4(qa[k].x - n.o.x, qa[k].y - n.o.y, qa[k].z - n.o.z, qa[k].w);
    return n;
}

/* the two halves at u = 1/2; the right half is re-anchored at the split point */
/* R13 at a split: where the split tangent (l3 - l2 = r1 - r0, 1/8 of
 * -q0 - q1 + q2 + q3) is negligible against the parent chord, its direction
 * is rounding noise of the exact value zero -- the split point is a cusp. The
 * children then take the exact value: their control points next to the split
 * point coincide with it (xyz; the radius channel is untouched). This is
 * what splitting the curve at the cusp beforehand gives (Sec. 3.4 requires
 * splitting curves with cusps): two curves whose end tangents vanish there. */
static void snap_cusp(const v4 q[4], v4 l[4], v4 r[4])
{
    if (!negligible(sub4(l[3], l[2]), sub4(q[3], q[0]))) return;
    l[2] = mk4(l[3].x, l[3].y, l[3].z, l[2].w);
    r[1] = mk4(r[0].x, r[0].y, r[0].z, r[1].w);
}

static void split_node(const node_t *a, node_t *L, node_t *R)
{
    v4 l[4], r[4];
    split_half(a->q, l, r);
    snap_cusp(a->q, l, r);
    const v4 s = l[3];
    L->o = a->o;
    R->o = mk4(a->o.x + s.x, a->o.y + s.y, a->o.z + s.z, 0.0);
    for (int k = 0; k < 4; ++k) {
        L->q[k] = l[k];
        R->q[k] = mk4(r[k].x - s.x, r[k].y - s.y, r[k].z - s.z, r[k].w);
    }
}

/* ------------------------------------------------------------------------ */
/* The recursion                                                             */
/* ------------------------------------------------------------------------ */

/* Near ties (R14). An FP32 implementation starts from the root correctly
 * rounded in its {p, d, t0, t1} form and forms each child with a few
 * roundings at the magnitude of the root's coordinates, so the coordinates
 * of a node at `level` are known to
 *     delta = (2 + 2 level) u X,   u = 2^-24,
 * X the largest |x|, |y|, |z| of the root control points in the ray frame
 * (measured growth: at most (1 + level) u X). Every t the search compares is
 * a function of those coordinates; its error bound is delta times the
 * function's sensitivity (plane_err for plane crossings, cyl_err for the
 * cylinder), plus a few roundings of its own. A comparison whose sides differ
 * by at most the sum of their bounds (times `scale`) is a tie. With scale > 0
 * the search numbers the ties it meets and flips tie j when bit j of
 * flip_mask is set; enumerating masks yields the results reachable by
 * flipping ties. */
typedef struct {
    double scale;
    double X;
    uint64_t flip_mask;
    int n_ties;
    int force_vis;      /* +1: every visibility tie decided visible */
} ties_t;

typedef struct {
    int depth;
    double tmax;
    int64_t tests, splits, backtracks;
    double t, u;
    double t_err;       /* error bound of t in an FP32 evaluation (as for ties) */
    int level;
    ties_t ties;
    v4 cap0, cap1;      /* the curve's start and end cap normals (ray frame, R13) */
    v4 end0, end1;      /* the curve's end points p0, p3 (ray frame) */
    double n[3];        /* normal at the hit, ray frame (R9) */
    double n_alt[3];    /* the other normal where cap and side entry tie (else n) */
    double n_err;       /* angle bound (radians) of n in an FP32 evaluation */
    int entry;          /* 0 side, 1 start cap, 2 end cap, 3 another plane (split plane, origin) */
    int quad;           /* the fiber is an elevated quadratic: its own bound */
    double stall_abs;   /* R19: (2^-20 X)^2, the FP32 resolution of node positions, squared */
    double stall_rel;   /* R19: 2^-16 times the root's extent (scaled by 4^-level per node) */
} search_t;

static double node_err(const search_t *S, int level)
{
    return (2.0 + 2.0 * level) * 0x1p-24 * S->ties.X;
}

/* Error bound of the cylinder's entry and exit: moving the axis by delta
 * moves t_cpa by up to delta (1 + |a.z| / sqrt(g)) and, through dist and r,
 * the half-length s by delta |a| / sqrt(g) * (dist + r) / sqrt(e) (large
 * near a tangent ray). */
static double cyl_err(double delta, const cyl_t *c, v4 a, double r)
{
    const double amp = sqrt(a.z * a.z + c->g) / sqrt(c->g);
    const double root = sqrt(fmax(c->e, 0.0));
    return amp * delta * (2.0 + (c->dist + r) / fmax(root, 1e-300)) +
           4.0 * 0x1p-24 * (fabs(c->t_cpa) + c->s);
}

/* `value` is the outcome of a comparison whose sides differ by `diff`, each
 * known to within the bounds that sum to `margin`; flip it if this is a
 * selected tie. */
static int decide(search_t *S, int value, double diff, double margin)
{
    if (S->ties.scale > 0.0 && isfinite(diff) && fabs(diff) <= S->ties.scale * margin) {
        const int j = S->ties.n_ties++;
        if (j < 64 && ((S->ties.flip_mask >> j) & 1u)) value = !value;
    }
    return value;
}

/* A visibility test (does the ray meet the node's cylinder inside its
 * interval?). A grazing ray meets the nodes on its path to a leaf near their
 * tangent point, so their visibility tests tie together, with correlated
 * rounding: force_vis > 0 decides all of them visible (as a radius larger
 * by the error bound would), which no choice of two single flips can reach.
 * The opposite choice is not offered: below the FP32 resolution every leaf's
 * visibility is a tie, and deciding all of them invisible would drop a ray
 * that passes through the union of neighbouring leaves. */
static int decide_vis(search_t *S, int value, double diff, double margin)
{
    if (S->ties.force_vis != 0 && S->ties.scale > 0.0 && isfinite(diff) &&
        fabs(diff) <= S->ties.scale * margin) {
        S->ties.n_ties++;
        return S->ties.force_vis > 0;
    }
    return decide(S, value, diff, margin);
}

/* Normal at a leaf hit (R9; the paper's final computation of an
 * intersection, with its undefined names read as the leaf chord and the ray
 * direction). A hit through the leaf cylinder's side gets the direction from
 * the chord point at the hit's projection to the hit point. A hit through a
 * plane (the interval's start: a cap or split plane, or the origin) that
 * lies on the curve's start or end cap plane -- within (8 + 2 level) 2^-24 X
 * (the node error bound of the leaf's level plus the rounding of the test
 * itself in FP32), measured along the plane's unit normal -- gets
 * that cap's outward normal (minus the start tangent, the end tangent; their
 * R13 limits where they vanish); other plane entries keep the radial
 * direction. The tolerance makes the rule independent of which of the
 * first leaves an FP32 evaluation enters: at depth 22 a leaf is shorter than
 * that error, and an empty-looking first leaf hands the hit to the next one
 * through their common split plane. */
static void unit3(v4 n, double out[3])
{
    const double len = sqrt(dot3(n, n));
    out[0] = n.x / len;
    out[1] = n.y / len;
    out[2] = n.z / len;
}

/* distance of the ray point at t to the plane through e with normal n */
static double plane_dist(double t, v4 e, v4 n)
{
    return fabs(t * n.z - dot3(e, n)) / sqrt(dot3(n, n));
}

/* te, lo: the cylinder entry and the interval's start, with error bounds ec
 * and elo (R14); delta the leaf's coordinate error. The side or plane entry
 * may go either way where te and lo are within those bounds of each other,
 * and the cap test where the distance is within a factor 2 of its tolerance: the
 * other normal is recorded for those ties. The angle bound of the side
 * normal is the hit point's and the chord point's error over the normal's
 * length; a cap normal comes from the root's tangent, exact up to rounding. */
static void leaf_normal(search_t *S, const node_t *N, v4 a, double t, double ul, double te,
                        double lo, double ec, double elo, double delta)
{
    const v4 ap = add4(mk4(N->o.x, N->o.y, N->o.z, 0.0), add4(N->q[0], scale4(a, ul)));
    const v4 side = mk4(-ap.x, -ap.y, t - ap.z, 0.0);
    const double tol = delta + 6.0 * 0x1p-24 * S->ties.X;
    const double d0 = plane_dist(t, S->end0, S->cap0) / tol;
    const double d1 = plane_dist(t, S->end1, S->cap1) / tol;
    const int near1 = d1 < d0;
    const double dc = near1 ? d1 : d0;
    const v4 cap = near1 ? S->cap1 : scale4(S->cap0, -1.0);
    const int plane = te < lo;
    const int on_cap = plane && dc <= 1.0;
    S->entry = !plane ? 0 : (on_cap ? 1 + near1 : 3);
    unit3(on_cap ? cap : side, S->n);
    const int tie = (fabs(te - lo) <= ec + elo && dc <= 2.0) || (plane && dc > 0.5 && dc < 2.0);
    unit3(tie ? (on_cap ? side : cap) : (on_cap ? cap : side), S->n_alt);
    const double ns = sqrt(dot3(side, side));
    const double e_side = 2.0 * (S->t_err + 3.0 * delta) / ns + 0x1p-20;
    S->n_err = !on_cap ? e_side : (tie ? fmax(e_side, 0x1p-20) : 0x1p-20);
}

/* largest squared length of a node's chord and end tangents */
static double node_extent(const v4 q[4])
{
    const v4 a = sub4(q[3], q[0]), b = sub4(q[1], q[0]), c = sub4(q[3], q[2]);
    return fmax(dot3(a, a), fmax(dot3(b, b), dot3(c, c)));
}

static int visit(search_t *S, const node_t *N, double lo, double hi, double elo, double ehi,
                 int level, double u0, double u1)
{
    S->tests++;
    const v4 *q = N->q;
    const v4 a = sub4(q[3], q[0]);
    const double R = S->quad ? quadratic_radius(q) : conservative_radius(q);
    const double delta = node_err(S, level);
    double te, tx, ec = 0.0;
    const cyl_t cy = cylinder_terms(N->o, a, R);
    if (cy.parallel) {                                   /* R4 */
        if (!(cy.e > 0.0)) return 0;
        te = -INFINITY;
        tx = INFINITY;
    } else {
        /* e = R^2 - dist^2 moves by up to 2 (R + dist) delta per unit of R and dist */
        if (!decide_vis(S, cy.e >= 0.0, cy.e, 4.0 * (R + cy.dist) * delta)) return 0;
        te = cy.t_cpa - cy.s;                            /* a flipped tangency: s = 0 */
        tx = cy.t_cpa + cy.s;
        ec = cyl_err(delta, &cy, a, R);
    }
    const double enter = fmax(te, lo), leave = fmin(tx, hi);
    const double e_enter = te >= lo ? ec : elo, e_leave = tx <= hi ? ec : ehi;
    if (!decide_vis(S, enter <= leave, leave - enter, e_enter + e_leave)) return 0;

    /* R19: a stalled end node is a leaf. It holds an end of the curve
     * (u = 0 or u = 1), and its extent (the largest squared length of its
     * chord and end tangents) is below the FP32 resolution of node positions,
     * (2^-20 X)^2, and below 2^-16 of the root's extent scaled to the level
     * (4^-level): the curve's speed vanishes at that end, all the node's
     * control points coincide to working precision, and halving it further
     * resolves only rounding noise. Near a vanishing end tangent the curve
     * leaves its end along a fixed direction, so the node's chord and end
     * planes stay perpendicular and its cylinder stays closed; an interior
     * stall (a cusp, where the direction reverses) is not cut short. */
    const double ext = node_extent(q);
    const int stalled = (u0 == 0.0 || u1 == 1.0) && ext <= S->stall_abs &&
                        ext <= ldexp(S->stall_rel, -2 * level);
    if (level >= S->depth || stalled) {
        const double t = enter;
        const double c = dot3(a, a);
        double ul = 0.0;
        if (c > 0.0) {
            const v4 h = mk4(-N->o.x, -N->o.y, t - N->o.z, 0.0);
            ul = fmin(1.0, fmax(0.0, dot3(h, a) / c));
        }
        S->t = t;
        S->t_err = e_enter;
        S->u = u0 + ul * (u1 - u0);
        S->level = level;
        leaf_normal(S, N, a, t, ul, te, lo, ec, elo, delta);
        return 1;
    }

    S->splits++;
    node_t Lc, Rc;
    split_node(N, &Lc, &Rc);
    const v4 n = split_normal(q);
    const double c = dot3(N->o, n) + dot3(Lc.q[3], n);    /* <split point, n> */
    int go_right, both;
    double flo = lo, fhi = hi, eflo = elo, efhi = ehi;
    if (n.z != 0.0) {
        const double tp = c / n.z;
        const double ep = plane_err(delta, n, tp);
        const int beyond_entry = decide(S, tp > te, tp - te, ep + ec);
        const int before_exit = decide(S, tp < tx, tx - tp, ep + ec);
        /* a flipped side of the entry stands for an FP32 crossing on the
         * other side of it: the half it narrows takes the crossing at the
         * far end of its error bound (for a plane nearly parallel to the
         * ray, ep is large and the crossing's sign itself is undetermined) */
        double tpn = tp;
        if (beyond_entry != (tp > te)) tpn = beyond_entry ? tp + ep : tp - ep;
        go_right = beyond_entry != (n.z > 0.0);
        both = beyond_entry && before_exit;
        if (beyond_entry) { if (tpn < fhi) { fhi = tpn; efhi = ep; } }
        else              { if (tpn > flo) { flo = tpn; eflo = ep; } }
    } else {
        const double side = -c;            /* <(0,0,t) - s, n> for every t */
        go_right = side > 0.0;
        both = side == 0.0;
    }
    const double um = 0.5 * (u0 + u1);
    const node_t *first = go_right ? &Rc : &Lc;
    const node_t *second = go_right ? &Lc : &Rc;
    const double f0 = go_right ? um : u0, f1 = go_right ? u1 : um;
    const double s0 = go_right ? u0 : um, s1 = go_right ? um : u1;

    if (visit(S, first, flo, fhi, eflo, efhi, level + 1, f0, f1)) return 1;
    if (!both) return 0;
    S->backtracks++;
    double blo, bhi, eblo, ebhi;
    cap_interval_e(second->o, second->q, S->tmax, node_err(S, level + 1), &blo, &bhi, &eblo, &ebhi);
    return visit(S, second, blo, bhi, eblo, ebhi, level + 1, s0, s1);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (ctypes)                                            */
/* ------------------------------------------------------------------------ */

int fo_version(void) { return 1; }

/* One pair. ray = (ox, oy, oz, dx, dy, dz, tmax); fiber = 16 values p0..p3
 * (x, y, z, r). stats (may be NULL) receives node tests, splits, backtracks
 * and the level of the leaf that was hit (-1 on a miss). Returns 1 on a hit. */
static int intersect_with_ties(const double ray[7], const double fiber[16], int depth,
                               double scale, uint64_t flip_mask, int force_vis, int *n_ties,
                               double *t_out, double *u_out, int64_t stats[4], double *t_err,
                               double normal_out[8], int quad)
{
    double frame[9];
    search_t S;
    memset(&S, 0, sizeof S);
    S.quad = quad;
    S.ties.scale = scale;
    S.ties.flip_mask = flip_mask;
    S.ties.force_vis = force_vis;
    S.depth = depth;
    S.tmax = ray[6];
    S.level = -1;
    int hit = 0;
    v4 q[4];
    if (depth >= 0 && depth <= 23 && ray[6] == ray[6] &&
        ray_frame(ray, ray + 3, fiber, q, NULL, frame)) {
        double lo, hi, elo, ehi;
        for (int k = 0; k < 4; ++k)
            S.ties.X = fmax(S.ties.X, fmax(fabs(q[k].x), fmax(fabs(q[k].y), fabs(q[k].z))));
        S.stall_abs = 0x1p-40 * S.ties.X * S.ties.X;
        S.stall_rel = 0x1p-16 * node_extent(q);
        const node_t root = anchored(q);
        S.cap0 = start_cap_normal(root.q);
        S.cap1 = end_cap_normal(root.q);
        S.end0 = q[0];
        S.end1 = q[3];
        cap_interval_e(root.o, root.q, S.tmax, node_err(&S, 0), &lo, &hi, &elo, &ehi);
        if (visit(&S, &root, lo, hi, elo, ehi, 0, 0.0, 1.0) && S.t < S.tmax) hit = 1;
    }
    if (!hit) { S.t = INFINITY; S.u = NAN; S.level = -1; }
    *t_out = S.t;
    *u_out = S.u;
    if (stats) {
        stats[0] = S.tests; stats[1] = S.splits; stats[2] = S.backtracks; stats[3] = S.level;
    }
    if (n_ties) *n_ties = S.ties.n_ties;
    if (t_err) {
        /* the node error model needs X, which the tie search sets up */
        *t_err = hit ? S.t_err : 0.0;
    }
    if (normal_out) {
        /* back to world space: n = n.x u + n.y v + n.z w */
        for (int k = 0; k < 3; ++k) {
            normal_out[k] = hit ? S.n[0] * frame[k] + S.n[1] * frame[3 + k] + S.n[2] * frame[6 + k] : NAN;
            normal_out[3 + k] = hit ? S.n_alt[0] * frame[k] + S.n_alt[1] * frame[3 + k] +
                                      S.n_alt[2] * frame[6 + k] : NAN;
        }
        normal_out[6] = hit ? S.n_err : NAN;
        normal_out[7] = hit ? (double)S.entry : NAN;
    }
    return hit;
}

int fo_intersect_d(const double ray[7], const double fiber[16], int depth,
                   double *t_out, double *u_out, int64_t stats[4])
{
    return intersect_with_ties(ray, fiber, depth, 0.0, 0, 0, NULL, t_out, u_out, stats, NULL, NULL, 0);
}

/* Every result reachable from one pair by flipping at most max_flips (1 or 2)
 * near-tie decisions (sides within `scale` times their FP32 error bounds,
 * R14), and the result with every visibility tie decided visible
 * (decide_vis). Writes up to max_out results (t, u, hit), the unflipped one
 * first; returns how many were written. */
static int tie_outcomes(const double ray[7], const double fiber[16], int depth, double scale,
                        int max_flips, int max_out, double *t_out, double *u_out, int *hit_out, int quad)
{
    int n = 0, k0 = 0;
    double t, u;
    int h = intersect_with_ties(ray, fiber, depth, scale, 0, 0, &k0, &t, &u, NULL, NULL, NULL, quad);
    if (max_out < 1) return 0;
    t_out[n] = t; u_out[n] = u; hit_out[n] = h; n++;
    if (scale > 0.0 && n < max_out) {
        h = intersect_with_ties(ray, fiber, depth, scale, 0, 1, NULL, &t, &u, NULL, NULL, NULL, quad);
        t_out[n] = t; u_out[n] = u; hit_out[n] = h; n++;
    }
    for (int j = 0; j < k0 && j < 64 && n < max_out; ++j) {
        int kj = 0;
        h = intersect_with_ties(ray, fiber, depth, scale, 1ull << j, 0, &kj, &t, &u, NULL, NULL, NULL, quad);
        t_out[n] = t; u_out[n] = u; hit_out[n] = h; n++;
        if (max_flips < 2) continue;
        for (int k = j + 1; k < kj && k < 64 && n < max_out; ++k) {
            h = intersect_with_ties(ray, fiber, depth, scale, (1ull << j) | (1ull << k), 0, NULL,
                                    &t, &u, NULL, NULL, NULL, quad);
            t_out[n] = t; u_out[n] = u; hit_out[n] = h; n++;
        }
    }
    return n;
}

int fo_tie_outcomes(const double ray[7], const double fiber[16], int depth, double scale,
                    int max_flips, int max_out, double *t_out, double *u_out, int *hit_out)
{
    return tie_outcomes(ray, fiber, depth, scale, max_flips, max_out, t_out, u_out, hit_out, 0);
}

/* The same for a quadratic fiber (12 values: p0, p1, p2, each x, y, z, r). */
int fo_tie_outcomes_quad(const double ray[7], const double fiber12[12], int depth, double scale,
                         int max_flips, int max_out, double *t_out, double *u_out, int *hit_out)
{
    double q[16];
    elevate_quadratic(fiber12, q);
    return tie_outcomes(ray, q, depth, scale, max_flips, max_out, t_out, u_out, hit_out, 1);
}

/* The constraint of Appendix B.1 for a quadratic: <p1 - p0, p1 - p2> <= 0
 * (returns 1 when it holds). */
int fo_quadratic_constraint(const double p[12])
{
    const v4 a = mk4(p[4] - p[0], p[5] - p[1], p[6] - p[2], 0.0);
    const v4 b = mk4(p[4] - p[8], p[5] - p[9], p[6] - p[10], 0.0);
    return dot3(a, b) <= 0.0;
}

/* Many pairs from the structure-of-arrays layout of the library (rays: 7 rows
 * of ray_stride floats; fibers: 16 rows of fiber_stride floats). Pair i uses
 * ray pair_ray[i] (or i when NULL) and fiber pair_fiber[i] (or i), at depth
 * pair_depth[i] (or depth). Radius control values are multiplied by
 * radius_scale (silhouette-band probes). stats_out (may be NULL) holds 4
 * int32 per pair; terr_out (may be NULL) the error bound of each hit's t in
 * an FP32 evaluation (the entry's bound from the tie model, R14; 0 on a
 * miss); normal_out (may be NULL) 8 per pair: the unit normal at the hit in
 * world space (R9), the normal of the other entry where the cap and side
 * entries tie (else the same), the angle bound in radians of the normal in
 * an FP32 evaluation, and how the leaf was entered (0 through its cylinder's
 * side, 1 through a plane on the curve's start cap plane, 2 on its end cap
 * plane, 3 through another plane or at the origin); NaN on a miss. Pairs
 * whose indices fall outside [0, n_rays) or [0, n_fibers) are misses. With
 * quad set, fibers are quadratics (12 rows: p0, p1, p2, each x, y, z, r),
 * held as their exact cubic elevation with the quadratic's own bound. */
void fo_batch_d(const float *rays, int64_t ray_stride, int64_t n_rays,
                const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                const int32_t *pair_ray, const int32_t *pair_fiber,
                const uint8_t *pair_depth, int depth, int64_t n,
                double radius_scale, double *t_out, double *u_out,
                uint8_t *hit_out, int32_t *stats_out, int nthreads, double *terr_out, double *normal_out,
                int quad)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ri = pair_ray ? pair_ray[i] : i;
        const int64_t fi = pair_fiber ? pair_fiber[i] : i;
        const int d = pair_depth ? (int)pair_depth[i] : depth;
        double ray[7], fib[16], t = INFINITY, u = NAN, te = 0.0;
        int64_t st[4] = {0, 0, 0, -1};
        int hit = 0;
        if (ri >= 0 && ri < n_rays && fi >= 0 && fi < n_fibers) {
            for (int r = 0; r < 7; ++r) ray[r] = rays[r * ray_stride + ri];
            if (quad) {
                double p[12];
                for (int r = 0; r < 12; ++r) p[r] = fibers[r * fiber_stride + fi];
                for (int k = 0; k < 3; ++k) p[4 * k + 3] *= radius_scale;
                elevate_quadratic(p, fib);
            } else {
                for (int r = 0; r < 16; ++r) fib[r] = fibers[r * fiber_stride + fi];
                for (int k = 0; k < 4; ++k) fib[4 * k + 3] *= radius_scale;
            }
            hit = intersect_with_ties(ray, fib, d, 0.0, 0, 0, NULL, &t, &u, st, &te,
                                      normal_out ? normal_out + 8 * i : NULL, quad);
        } else if (normal_out) {
            for (int k = 0; k < 8; ++k) normal_out[8 * i + k] = NAN;
        }
        if (terr_out) terr_out[i] = te;
        t_out[i] = t;
        u_out[i] = u;
        hit_out[i] = (uint8_t)hit;
        if (stats_out) {
            for (int k = 0; k < 4; ++k) stats_out[4 * i + k] = (int32_t)st[k];
        }
    }
}

/* Nearest hit over a candidate list per ray: the interface a renderer's
 * top-level hierarchy uses (Sec. 1 and Sec. 4: the fibers referenced by the
 * hierarchy leaves a ray reaches are tested one after another, and a hit
 * shortens the ray for the fibers after it). Ray r's candidates are
 * cand[off[r]] .. cand[off[r + 1] - 1], tested in that order at depth d (or
 * cand_depth[k]) with tmax = the ray's tmax until the first hit and the
 * latest hit's t after it; a hit counts when its t is below that tmax, so of
 * equal hits the first in the list is kept. At most max_cand candidates of a
 * ray are tested (the first ones). Per ray: t, u, hit, the fiber of the kept
 * hit (-1 on a miss), and when given t_err and the 8 normal values as
 * fo_batch_d. */
void fo_nearest_d(const float *rays, int64_t ray_stride, int64_t n_rays,
                  const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                  const int64_t *off, const int32_t *cand, const uint8_t *cand_depth, int depth,
                  int max_cand, double radius_scale, double *t_out, double *u_out, uint8_t *hit_out,
                  int32_t *fiber_out, int nthreads, double *terr_out, double *normal_out)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t r = 0; r < n_rays; ++r) {
        double ray[7];
        for (int k = 0; k < 7; ++k) ray[k] = rays[k * ray_stride + r];
        double best_t = INFINITY, best_u = NAN, best_e = 0.0, best_n[8];
        int32_t best_f = -1;
        for (int k = 0; k < 8; ++k) best_n[k] = NAN;
        int64_t end = off[r + 1];
        if (end - off[r] > max_cand) end = off[r] + max_cand;
        for (int64_t j = off[r]; j < end; ++j) {
            const int64_t fi = cand[j];
            if (fi < 0 || fi >= n_fibers) continue;
            const int d = cand_depth ? (int)cand_depth[j] : depth;
            double fib[16], t, u, te = 0.0, nn[8];
            for (int k = 0; k < 16; ++k) fib[k] = fibers[k * fiber_stride + fi];
            for (int k = 0; k < 4; ++k) fib[4 * k + 3] *= radius_scale;
            if (intersect_with_ties(ray, fib, d, 0.0, 0, 0, NULL, &t, &u, NULL, &te, nn, 0)) {
                best_t = t;
                best_u = u;
                best_e = te;
                best_f = (int32_t)fi;
                for (int k = 0; k < 8; ++k) best_n[k] = nn[k];
                ray[6] = t;                     /* later candidates must come nearer */
            }
        }
        t_out[r] = best_t;
        u_out[r] = best_u;
        hit_out[r] = best_f >= 0;
        fiber_out[r] = best_f;
        if (terr_out) terr_out[r] = best_e;
        if (normal_out)
            for (int k = 0; k < 8; ++k) normal_out[8 * r + k] = best_n[k];
    }
}

/* Building blocks exported for the pins in the test suite. */

void fo_split_half(const double q[16], double L[16], double R[16])
{
    v4 a[4], l[4], r[4];
    for (int k = 0; k < 4; ++k) a[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
    split_half(a, l, r);
    for (int k = 0; k < 4; ++k) {
        L[4 * k] = l[k].x; L[4 * k + 1] = l[k].y; L[4 * k + 2] = l[k].z; L[4 * k + 3] = l[k].w;
        R[4 * k] = r[k].x; R[4 * k + 1] = r[k].y; R[4 * k + 2] = r[k].z; R[4 * k + 3] = r[k].w;
    }
}

/* The children the recursion uses: de Casteljau halves with the cusp rule
 * (snap_cusp). */
void fo_split_children(const double q[16], double L[16], double R[16])
{
    v4 a[4], l[4], r[4];
    for (int k = 0; k < 4; ++k) a[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
    split_half(a, l, r);
    snap_cusp(a, l, r);
    for (int k = 0; k < 4; ++k) {
        L[4 * k] = l[k].x; L[4 * k + 1] = l[k].y; L[4 * k + 2] = l[k].z; L[4 * k + 3] = l[k].w;
        R[4 * k] = r[k].x; R[4 * k + 1] = r[k].y; R[4 * k + 2] = r[k].z; R[4 * k + 3] = r[k].w;
    }
}

void fo_split_plane(const double q[16], double s[3], double n[3])
{
    v4 a[4], l[4], r[4];
    for (int k = 0; k < 4; ++k) a[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
    split_half(a, l, r);
    const v4 t = split_normal(a);
    s[0] = l[3].x; s[1] = l[3].y; s[2] = l[3].z;
    n[0] = t.x; n[1] = t.y; n[2] = t.z;
}

int fo_unit_ray_cylinder(const double o[3], const double a[3], double r,
                         double *t0, double *t1)
{
    return unit_ray_cylinder(mk4(o[0], o[1], o[2], 0), mk4(a[0], a[1], a[2], 0), r, t0, t1);
}

double fo_conservative_radius(const double q[16])
{
    v4 a[4];
    for (int k = 0; k < 4; ++k) a[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
    return conservative_radius(a);
}

void fo_cap_interval(const double q[16], double tmax, double out[2])
{
    v4 a[4];
    for (int k = 0; k < 4; ++k) a[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]);
    const node_t n = anchored(a);
    cap_interval_e(n.o, n.q, tmax, 0.0, &out[0], &out[1], NULL, NULL);
}

int fo_ray_frame(const double ray[7], const double fiber[16], double out[16])
{
    v4 q[4];
    if (!ray_frame(ray, ray + 3, fiber, q, NULL, NULL)) return 0;
    for (int k = 0; k < 4; ++k) {
        out[4 * k] = q[k].x; out[4 * k + 1] = q[k].y; out[4 * k + 2] = q[k].z; out[4 * k + 3] = q[k].w;
    }
    return 1;
}

/* The five cubic constraints of Section 3.4 (proved in Appendix B.2): returns
 * a bit mask, bit k set when inequality k holds; 31 means the curve can be
 * split recursively into sub-curves with disjoint bounding volumes. */
int fo_cubic_constraints(const double q[16])
{
    v4 p[4];
    for (int k = 0; k < 4; ++k) p[k] = mk4(q[4 * k], q[4 * k + 1], q[4 * k + 2], 0.0);
    const double c[5] = {
        dot3(sub4(p[2], p[0]), sub4(p[1], p[0])),
        dot3(sub4(p[3], p[1]), sub4(p[1], p[0])),
        dot3(sub4(p[3], p[1]), sub4(p[3], p[2])),
        dot3(sub4(p[2], p[0]), sub4(p[3], p[2])),
        dot3(sub4(p[2], p[0]), sub4(p[3], p[1])),
    };
    int m = 0;
    for (int k = 0; k < 5; ++k) if (c[k] >= 0.0) m |= 1 << k;
    return m;
}
