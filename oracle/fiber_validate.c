/*
 * TEST INFRASTRUCTURE -- FP64 CPU oracle for the validation and
 * pre-subdivision of fibers (Section 3.4 of Binder & Keller, "Fast, High
 * Precision Ray/Fiber Intersection using Tight, Disjoint Bounding Volumes").
 * Only the test suite loads it; the HIP path shares nothing with it.
 *
 * A fiber is valid for the method when
 *   1. the five cubic constraints of Section 3.4 hold (every split then
 *      separates the halves by the split plane, Appendix B.2), and
 *   2. no disc of the swept solid reaches across the curve's start or end
 *      cap plane (Section 3.4, Fig. "EvilConfiguration": a thick fiber, or
 *      a strongly bent one, would have part of its surface cropped by the
 *      plane). Reading R17: the disc at u (centre C(u), radius r(u), normal
 *      C'(u)) reaches furthest along a plane normal n at the point
 *      C(u) + r(u) m(u), m(u) the unit component of n normal to C'(u)
 *      (Gram-Schmidt), so its excess over the plane through the end point is
 *        start:  h0(u) = r(u) sin(angle(C'(u), n0)) - <C(u) - p0, n0>
 *        end:    h1(u) = r(u) sin(angle(C'(u), n1)) - <p3 - C(u), n1>
 *      with n0, n1 the unit cap normals (R13's limit chain where an end
 *      tangent vanishes). The paper writes the touching condition with
 *      p3 - p_u + r n_u, whose sign makes it vanish only at tangency on the
 *      wrong side; the excess above is the reading used here. A fiber is
 *      thick at an end when the largest excess over u in [0, 1] exceeds
 *      1e-9 of its extent (|p3 - p0| plus the largest radius value): at the
 *      end point itself the excess is exactly zero. Points where C'(u)
 *      vanishes have no disc plane and are skipped.
 *
 * Here the largest excess is found by brute force: 8,193 evenly spaced
 * samples, 32 samples packed geometrically towards each end (u = 2^-j and
 * 1 - 2^-j, j = 14 .. 45, where the excess is of the order of the distance
 * to the end), and a golden-section search in the neighbourhood of every
 * local maximum of the samples.
 *
 * Pre-subdivision (Section 3.4: curves that break the constraints "must be
 * subdivided beforehand"): a fiber is halved by de Casteljau's construction
 * at u = 1/2 (Appendix B.2), depth first, left half first, until a piece is
 * valid or max_level halvings deep; every piece is emitted with its
 * parameter interval and its validity mask.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z; } vec;

static vec vsub(vec a, vec b) { vec r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static double vdot(vec a, vec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec vcross(vec a, vec b)
{
    vec r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}

static vec pt(const double q[16], int k) { vec r = {q[4 * k], q[4 * k + 1], q[4 * k + 2]}; return r; }

/* C(u) with the radius, and C'(u) (xyz) from the power form */
static void curve_at(const double q[16], double u, vec *C, double *r, vec *D)
{
    const double v = 1.0 - u;
    const double b[4] = {v * v * v, 3.0 * u * v * v, 3.0 * u * u * v, u * u * u};
    const double e[3] = {3.0 * v * v, 6.0 * u * v, 3.0 * u * u};
    C->x = C->y = C->z = 0.0;
    *r = 0.0;
    D->x = D->y = D->z = 0.0;
    for (int k = 0; k < 4; ++k) {
        C->x += b[k] * q[4 * k];
        C->y += b[k] * q[4 * k + 1];
        C->z += b[k] * q[4 * k + 2];
        *r += b[k] * q[4 * k + 3];
    }
    for (int k = 0; k < 3; ++k) {
        D->x += e[k] * (q[4 * k + 4] - q[4 * k]);
        D->y += e[k] * (q[4 * k + 5] - q[4 * k + 1]);
        D->z += e[k] * (q[4 * k + 6] - q[4 * k + 2]);
    }
}

/* unit cap normal at an end: the end tangent, or R13's limit chain */
static vec cap_dir(const double q[16], int end)
{
    const vec a = vsub(pt(q, 3), pt(q, 0));
    const double lim = 0x1p-40 * vdot(a, a);
    vec c[3];
    c[0] = end ? vsub(pt(q, 3), pt(q, 2)) : vsub(pt(q, 1), pt(q, 0));
    c[1] = end ? vsub(pt(q, 3), pt(q, 1)) : vsub(pt(q, 2), pt(q, 0));
    c[2] = a;
    int j = 0;
    while (j < 2 && vdot(c[j], c[j]) <= lim) ++j;
    const double l = sqrt(vdot(c[j], c[j]));
    vec n = {c[j].x / l, c[j].y / l, c[j].z / l};
    return n;
}

/* excess of the disc at u over the cap plane of `end` (-inf without a disc) */
static double excess(const double q[16], int end, vec n, double u)
{
    vec C, D;
    double r;
    curve_at(q, u, &C, &r, &D);
    const double dl = sqrt(vdot(D, D));
    if (!(dl > 0.0)) return -INFINITY;
    const vec x = vcross(D, n);
    const double s = sqrt(vdot(x, x)) / dl;
    const double along = end ? vdot(vsub(pt(q, 3), C), n) : vdot(vsub(C, pt(q, 0)), n);
    return r * s - along;
}

/* largest excess over [0, 1] (brute force, see the header) */
static double max_excess(const double q[16], int end)
{
    const vec n = cap_dir(q, end);
    enum { NS = 8192, NG = 32 };
    double us[NS + 1 + 2 * NG], hs[NS + 1 + 2 * NG];
    int m = 0;
    for (int j = 45; j >= 14; --j) us[m++] = ldexp(1.0, -j);
    for (int k = 0; k <= NS; ++k) us[m++] = (double)k / NS;
    for (int j = 14; j <= 45; ++j) us[m++] = 1.0 - ldexp(1.0, -j);
    /* sort the few out-of-order entries (the geometric ones lie inside the
     * first and last even intervals) */
    for (int i = 1; i < m; ++i) {
        const double v = us[i];
        int k = i - 1;
        while (k >= 0 && us[k] > v) { us[k + 1] = us[k]; --k; }
        us[k + 1] = v;
    }
    double best = -INFINITY;
    for (int i = 0; i < m; ++i) {
        hs[i] = excess(q, end, n, us[i]);
        if (hs[i] > best) best = hs[i];
    }
    for (int i = 1; i + 1 < m; ++i) {
        if (!(hs[i] >= hs[i - 1] && hs[i] >= hs[i + 1]) || hs[i] == -INFINITY) continue;
        const double g = 0.38196601125010515;
        double a = us[i - 1], b = us[i + 1];
        double x1 = a + g * (b - a), x2 = b - g * (b - a);
        double f1 = excess(q, end, n, x1), f2 = excess(q, end, n, x2);
        for (int it = 0; it < 80; ++it) {
            if (f1 > f2) { b = x2; x2 = x1; f2 = f1; x1 = a + g * (b - a); f1 = excess(q, end, n, x1); }
            else         { a = x1; x1 = x2; f1 = f2; x2 = b - g * (b - a); f2 = excess(q, end, n, x2); }
        }
        if (f1 > best) best = f1;
        if (f2 > best) best = f2;
    }
    return best;
}

static double extent(const double q[16])
{
    const vec a = vsub(pt(q, 3), pt(q, 0));
    double rmax = 0.0;
    for (int k = 0; k < 4; ++k) rmax = fmax(rmax, fabs(q[4 * k + 3]));
    return sqrt(vdot(a, a)) + rmax;
}

/* Validity mask of one fiber (0: valid): bit k (0..4) inequality k of
 * Section 3.4 fails, bit 5 thick at the start, bit 6 thick at the end, bit 7
 * a non-finite control point. ex0/ex1 (may be NULL) receive the largest
 * excesses relative to the fiber's extent. */
int fv_validate(const double q[16], double *ex0, double *ex1)
{
    for (int k = 0; k < 16; ++k)
        if (!isfinite(q[k])) return 1 << 7;
    const vec p0 = pt(q, 0), p1 = pt(q, 1), p2 = pt(q, 2), p3 = pt(q, 3);
    const double c[5] = {
        vdot(vsub(p2, p0), vsub(p1, p0)),
        vdot(vsub(p3, p1), vsub(p1, p0)),
        vdot(vsub(p3, p1), vsub(p3, p2)),
        vdot(vsub(p2, p0), vsub(p3, p2)),
        vdot(vsub(p2, p0), vsub(p3, p1)),
    };
    int mask = 0;
    for (int k = 0; k < 5; ++k) if (!(c[k] >= 0.0)) mask |= 1 << k;
    const double X = extent(q);
    const double e0 = max_excess(q, 0) / X, e1 = max_excess(q, 1) / X;
    if (e0 > 1e-9) mask |= 1 << 5;
    if (e1 > 1e-9) mask |= 1 << 6;
    if (ex0) *ex0 = e0;
    if (ex1) *ex1 = e1;
    return mask;
}

/* de Casteljau halves at u = 1/2 (4-D) */
static void halves(const double q[16], double L[16], double R[16])
{
    for (int c = 0; c < 4; ++c) {
        const double a = q[c], b = q[4 + c], d = q[8 + c], e = q[12 + c];
        const double m01 = (a + b) * 0.5, m12 = (b + d) * 0.5, m23 = (d + e) * 0.5;
        const double m012 = (m01 + m12) * 0.5, m123 = (m12 + m23) * 0.5;
        const double s = (m012 + m123) * 0.5;
        L[c] = a; L[4 + c] = m01; L[8 + c] = m012; L[12 + c] = s;
        R[c] = s; R[4 + c] = m123; R[8 + c] = m23; R[12 + c] = e;
    }
}

static int split_rec(const double q[16], int level, int max_level, double u0, double u1, double *pieces,
                     double *pu0, double *pu1, int32_t *pmask, int count, int max_pieces)
{
    const int mask = fv_validate(q, NULL, NULL);
    if (mask == 0 || level >= max_level || (mask & (1 << 7))) {
        if (count < max_pieces) {
            memcpy(pieces + 16 * count, q, 16 * sizeof(double));
            pu0[count] = u0;
            pu1[count] = u1;
            pmask[count] = mask;
        }
        return count + 1;
    }
    double L[16], R[16];
    halves(q, L, R);
    const double um = 0.5 * (u0 + u1);
    count = split_rec(L, level + 1, max_level, u0, um, pieces, pu0, pu1, pmask, count, max_pieces);
    return split_rec(R, level + 1, max_level, um, u1, pieces, pu0, pu1, pmask, count, max_pieces);
}

/* Pieces of one fiber (see the header); returns their number (pieces past
 * max_pieces are counted, not written). */
int fv_presplit(const double q[16], int max_level, double *pieces, double *pu0, double *pu1, int32_t *pmask,
                int max_pieces)
{
    return split_rec(q, 0, max_level, 0.0, 1.0, pieces, pu0, pu1, pmask, 0, max_pieces);
}

/* Batch over a fiber table (16 rows of n floats): masks and excesses */
void fv_validate_batch(const float *fibers, int64_t stride, int64_t n, int32_t *mask_out, double *ex_out,
                       int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double q[16];
        for (int k = 0; k < 16; ++k) q[k] = fibers[k * stride + i];
        double e0, e1;
        mask_out[i] = fv_validate(q, &e0, &e1);
        if (ex_out) { ex_out[2 * i] = e0; ex_out[2 * i + 1] = e1; }
    }
}
