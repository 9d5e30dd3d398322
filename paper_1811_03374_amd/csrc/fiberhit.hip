// fiberhit: ray/fiber intersection for AMD MI355X (gfx950).
//
// Method: Binder & Keller, "Fast, High Precision Ray/Fiber Intersection using
// Tight, Disjoint Bounding Volumes" (arXiv 1811.03374). One lane owns one
// (ray, fiber) pair. The fiber is moved into the frame of the ray once
// (Section 3.3), held in the {p, d, t0, t1} form of Section 3.1, and
// subdivided at the parametric centre inside bounding cylinders cropped by
// end-cap and split planes (Sections 3.2, 3.3). The recursion is iterated with
// one bit per level (Section 3.3); a backtrack rebuilds the pending sibling by
// replaying the split rules from the root along the integer path, which gives
// bit-for-bit the node that the descent produced (no cancellation from
// re-evaluating the curve at absolute parameters).
//
// Arithmetic notes for gfx950:
//  * everything is FP32 VALU work (no MFMA: nothing here is a contraction);
//  * the ray-frame projection runs once per pair in FP64 (full VALU rate on
//    CDNA4) from exact differences of the float32 inputs, so the root's
//    {p, d, t0, t1} components are each correctly rounded to float32 -- the
//    traversal never forms a difference of rounded absolute coordinates;
//  * the file is compiled with -ffp-contract=off: every FMA is written out, so
//    the descent and the replay round identically.
//
// Readings where the paper is silent or its listings disagree are the same as
// those of the FP64 CPU oracle (visibility needs a non-empty cropped
// interval, the leaf t is the entry into the capped leaf cylinder, planes
// parallel to the ray and axes parallel to the ray get explicit rules, zero
// tangents fall back to the next non-negligible control-polygon edge).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fiberhit.h"

namespace {

constexpr int kWave = 64;                     // gfx950 wavefront
#ifndef FIBERHIT_QUEUE
#define FIBERHIT_QUEUE 64                     // build knob: queue entries per wave
#endif
constexpr int kQueue = FIBERHIT_QUEUE;        // prepared roots per wave (LDS queue)

// Entry x of the queue ring, for 0 <= x < 3 kQueue.
__device__ __forceinline__ int qslot(int x)
{
    x = x >= kQueue ? x - kQueue : x;
    return x >= kQueue ? x - kQueue : x;
}
constexpr int kQWords = 21;                   // root node (16), lo, hi, tmax, pair, scene * 64 + stall * 32 + depth
constexpr uint32_t kRootSize = 1u << 23;      // parametric domain [0, 1) in units of 2^-23
constexpr uint32_t kStallBit = 1u << 31;       // flag bit kept in a lane's interval start
constexpr uint32_t kStartMask = kRootSize - 1u;
constexpr int kMaxTrips = 1 << 16;            // hang guard; real pairs need < 200 trips
#ifndef FIBERHIT_PARENT_CACHE
#define FIBERHIT_PARENT_CACHE 1
#endif
constexpr bool kParentCache = FIBERHIT_PARENT_CACHE != 0;   // cache the latest both-hit parent in LDS
#ifndef FIBERHIT_FUSED_REFILL
#define FIBERHIT_FUSED_REFILL 1                    // free lanes that take queued roots (single calls)
#endif
#ifndef FIBERHIT_REFINE_REFILL
#define FIBERHIT_REFINE_REFILL 1                   // the same for refined calls
#endif

struct V4 { float x, y, z, w; };
struct Node { V4 p, d, t0, t1; };             // Section 3.1: p = p0, d = p3-p0, t0 = p1-p0, t1 = p3-p2

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float vsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// A tangent whose squared length is at most 2^-40 of the squared chord (cc)
// has no reliable direction: at a cusp or a vanishing end tangent its
// components are rounding noise of the control points. The cap and split
// planes then take the next control-polygon edge or the chord instead. With
// a zero chord only the zero vector is negligible.
__device__ __forceinline__ bool negligible(float x, float y, float z, float cc)
{
    return fmaf(x, x, fmaf(y, y, z * z)) <= 0x1p-40f * cc;
}

// ---------------------------------------------------------------------------
// Ray frame (Section 3.3)
// ---------------------------------------------------------------------------

// 1/sqrt(x) and 1/x in double: hardware estimates refined by two Newton
// steps each (quadratic convergence from ~2^-22 to full double precision).
__device__ __forceinline__ double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    y = fma(fma(-x, y, 1.0), y, y);
    return y;
}

// Orthonormal basis (u, v) completing the unit w: Duff et al. 2017, the
// revision of Frisvad's construction cited in Section 3.3.
__device__ __forceinline__ void make_onb(double wx, double wy, double wz,
                                         double u[3], double v[3])
{
    const double s = copysign(1.0, wz);
    const double a = -rcp64(s + wz);
    const double b = wx * wy * a;
    u[0] = fma(s * wx * wx, a, 1.0);
    u[1] = s * b;
    u[2] = -s * wx;
    v[0] = b;
    v[1] = fma(wy * wy, a, s);
    v[2] = -wy;
}


// ---------------------------------------------------------------------------
// Node geometry
// ---------------------------------------------------------------------------

// t interval between the node's two end-cap planes (Section 3.3, cropping),
// intersected with [0, tmax]. Start cap: plane through p, normal t0, curve on
// the positive side. End cap: plane through p + d, normal t1, curve on the
// negative side. A negligible end tangent falls back to the next
// control-polygon edge from that end (p2 - p0, resp. p3 - p1), then the chord.
__device__ __forceinline__ void cap_interval(const Node &c, float tmax, float &lo, float &hi)
{
    float n0x = c.t0.x, n0y = c.t0.y, n0z = c.t0.z;
    float n1x = c.t1.x, n1y = c.t1.y, n1z = c.t1.z;
    const float cc = dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z);
    if (negligible(n0x, n0y, n0z, cc) || negligible(n1x, n1y, n1z, cc)) {
        // rare (a vanishing end tangent): kept out of the common path
        if (negligible(n0x, n0y, n0z, cc)) { n0x = c.d.x - c.t1.x; n0y = c.d.y - c.t1.y; n0z = c.d.z - c.t1.z; }
        if (negligible(n0x, n0y, n0z, cc)) { n0x = c.d.x; n0y = c.d.y; n0z = c.d.z; }
        if (negligible(n1x, n1y, n1z, cc)) { n1x = c.d.x - c.t0.x; n1y = c.d.y - c.t0.y; n1z = c.d.z - c.t0.z; }
        if (negligible(n1x, n1y, n1z, cc)) { n1x = c.d.x; n1y = c.d.y; n1z = c.d.z; }
    }

    // both crossings are computed and selected by the signs of the normals'
    // z (no divergent branches); a plane parallel to the ray keeps the whole
    // ray or none of it
    const float c0 = dot3(c.p.x, c.p.y, c.p.z, n0x, n0y, n0z);
    const float q0 = c0 * rcp(n0z);
    const float ex = c.p.x + c.d.x, ey = c.p.y + c.d.y, ez = c.p.z + c.d.z;
    const float c1 = dot3(ex, ey, ez, n1x, n1y, n1z);
    const float q1 = c1 * rcp(n1z);
    float l = n0z > 0.0f ? fmaxf(0.0f, q0) : 0.0f;
    float h = n0z < 0.0f ? fminf(tmax, q0) : tmax;
    h = n1z > 0.0f ? fminf(h, q1) : h;
    l = n1z < 0.0f ? fmaxf(l, q1) : l;
    const bool empty = (n0z == 0.0f && c0 > 0.0f) || (n1z == 0.0f && c1 < 0.0f);
    lo = empty ? INFINITY : l;
    hi = empty ? -INFINITY : h;
}

// Conservative cylinder radius (Section 3.3): largest distance of the inner
// control points (t0 and -t1 relative to the chord ends) to the chord line,
// plus the largest radius control value (convex hull of the radius Bezier).
// QUAD: the node is the exact cubic elevation of a quadratic (Appendix B.1:
// q1 = (p0 + 2 p1) / 3, q2 = (2 p1 + p2) / 3): the same curve, halves and
// planes. Its bound is the quadratic's: the middle control point p1 lies at
// 3/2 of the elevated inner points' distance from the chord, and the middle
// radius value is r0 + 3/2 t0.w = r2 - 3/2 t1.w.
template <bool QUAD = false>
__device__ __forceinline__ float conservative_radius(const Node &c)
{
    const float cc = dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z);
    const float ic = cc > 0.0f ? rcp(cc) : 0.0f;
    const float b0 = dot3(c.t0.x, c.t0.y, c.t0.z, c.d.x, c.d.y, c.d.z) * ic;
    const float e0x = fmaf(-b0, c.d.x, c.t0.x), e0y = fmaf(-b0, c.d.y, c.t0.y), e0z = fmaf(-b0, c.d.z, c.t0.z);
    const float b1 = dot3(c.t1.x, c.t1.y, c.t1.z, c.d.x, c.d.y, c.d.z) * ic;
    const float e1x = fmaf(-b1, c.d.x, c.t1.x), e1y = fmaf(-b1, c.d.y, c.t1.y), e1z = fmaf(-b1, c.d.z, c.t1.z);
    const float l0 = dot3(e0x, e0y, e0z, e0x, e0y, e0z);
    const float l1 = dot3(e1x, e1y, e1z, e1x, e1y, e1z);
    if constexpr (QUAD) {
        const float r1 = fmaxf(fmaf(1.5f, c.t0.w, 0.0f), fmaf(-1.5f, c.t1.w, c.d.w));
        const float rmax = c.p.w + fmaxf(fmaxf(0.0f, c.d.w), r1);
        return 1.5f * vsqrt(fmaxf(l0, l1)) + rmax;
    }
    const float rmax = c.p.w + fmaxf(fmaxf(0.0f, c.t0.w), fmaxf(c.d.w, c.d.w - c.t1.w));
    return vsqrt(fmaxf(l0, l1)) + rmax;
}

// Unit ray (origin, +z) against the infinite cylinder of radius r about the
// line through o along a (Appendix A). False on a miss.
__device__ __forceinline__ bool unit_ray_cylinder(const V4 &o, const V4 &a, float r, float &te, float &tx)
{
    // both cases are evaluated and selected: no divergent branch. The axis
    // counts as parallel to the ray when its across-ray part is below 2^-50
    // of its along-ray part (or zero): beyond that the general formula's
    // terms (up to a.z^2 / g) would leave the float range, while the
    // cylinder it describes already spans the whole ray. The test is relative:
    // the chord of a node next to a cusp or a stalled end shrinks like 4^-level,
    // and an absolute threshold took such nodes for parallel ones.
    const float g = fmaf(a.x, a.x, a.y * a.y);
    const bool parallel = g <= 0x1p-100f * (a.z * a.z);
    const float dd = fmaf(a.x, o.y, -(a.y * o.x));
    const float h = rcp(g);
    const float e = fmaf(-(dd * dd), h, r * r);
    const float tc = fmaf(-a.z, fmaf(a.x, o.x, a.y * o.y) * h, o.z);
    const float s = vsqrt(e * fmaf(a.z, a.z, g) * h);
    const bool inside = fmaf(o.x, o.x, o.y * o.y) < r * r;
    te = parallel ? -INFINITY : tc - s;
    tx = parallel ? INFINITY : tc + s;
    return parallel ? inside : e >= 0.0f;
}

// Split quantities of Section 3.1: centre offset dp and split tangent tc
// (1/8 of -q0 - q1 + q2 + q3, the children's tangent at the split point).
// A negligible split tangent is rounding noise of the exact value zero: the
// split point is a cusp, and the children take a zero tangent there (xyz;
// the radius channel keeps its slope), as if the curve had been split at the
// cusp beforehand. Returns whether that happened.
__device__ __forceinline__ bool split_terms(const Node &c, V4 &dp, V4 &tc)
{
    dp.x = fmaf(0.375f, c.t0.x - c.t1.x, 0.5f * c.d.x);
    dp.y = fmaf(0.375f, c.t0.y - c.t1.y, 0.5f * c.d.y);
    dp.z = fmaf(0.375f, c.t0.z - c.t1.z, 0.5f * c.d.z);
    dp.w = fmaf(0.375f, c.t0.w - c.t1.w, 0.5f * c.d.w);
    tc.x = fmaf(-0.125f, c.t0.x + c.t1.x, 0.25f * c.d.x);
    tc.y = fmaf(-0.125f, c.t0.y + c.t1.y, 0.25f * c.d.y);
    tc.z = fmaf(-0.125f, c.t0.z + c.t1.z, 0.25f * c.d.z);
    tc.w = fmaf(-0.125f, c.t0.w + c.t1.w, 0.25f * c.d.w);
    const bool cusp = negligible(tc.x, tc.y, tc.z, dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z));
    tc.x = cusp ? 0.0f : tc.x;
    tc.y = cusp ? 0.0f : tc.y;
    tc.z = cusp ? 0.0f : tc.z;
    return cusp;
}

// Keep one half (Section 3.1): left (p, dp, t0/2, tc) or right (p+dp, d-dp, tc, t1/2).
__device__ __forceinline__ void take_child(Node &c, const V4 &dp, const V4 &tc, bool right)
{
#define FI_TAKE(k)                                                    \
    {                                                                 \
        const float pr = c.p.k + dp.k, dr = c.d.k - dp.k;             \
        const float h0 = 0.5f * c.t0.k, h1 = 0.5f * c.t1.k;           \
        c.p.k = right ? pr : c.p.k;                                   \
        c.d.k = right ? dr : dp.k;                                    \
        c.t0.k = right ? tc.k : h0;                                   \
        c.t1.k = right ? h1 : tc.k;                                   \
    }
    FI_TAKE(x) FI_TAKE(y) FI_TAKE(z) FI_TAKE(w)
#undef FI_TAKE
}

// ---------------------------------------------------------------------------
// Per-lane traversal state
// ---------------------------------------------------------------------------

struct Args {
    const float *rays; int64_t ray_stride; int64_t n_rays;
    const float *fibers; int64_t fiber_stride; int64_t n_fibers;
    const int32_t *pair_ray; const int32_t *pair_fiber; const uint8_t *pair_depth;
    int32_t depth; int64_t n_pairs;
    float *t_out; float *u_out; uint8_t *hit_out;
    int32_t *counts;                       // counting mode
    double *t64_out; double *u64_out;      // refinement
    float *normal_out;                     // normals (3 rows of n_pairs), or null
    // candidate lists: pair i is ray i against its candidate number
    // cand_round (cand_fiber[cand_off[i] + cand_round]), tested against the
    // ray shortened to the nearest hit so far; pair_depth then indexes the
    // candidates. Null cand_off: plain pairs.
    const int64_t *cand_off; const int32_t *cand_fiber; int32_t cand_round; int64_t n_cand;
    int32_t *fiber_out;                    // the fiber of each ray's nearest hit
};

// ---------------------------------------------------------------------------
// FP64 surface solve inside a leaf (FI_FP64_REFINE)
// ---------------------------------------------------------------------------
//
// The leaf cylinders converge to the solid swept by a disc of radius r(u)
// centred on C(u) in the plane normal to C'(u) (Sec. 3.2: the limit surface
// of the cylinders maps the intersection to the closest point on the curve),
// closed by the end discs. With refinement, a pair of depth > 16 runs the
// traversal with every pruning test enlarged by a bound on its FP32 rounding,
// so that no leaf holding part of that solid along the ray is pruned, and each
// leaf the search reaches is checked in FP64: the first point of the solid
// along the ray whose disc parameter u lies in the leaf's interval. A leaf
// with no such point counts as missed and the search goes on; leaves are
// reached front to back, so the first leaf that holds the solid gives the hit.
// In the ray frame (ray point P = (0, 0, t)):
//   the ray meets the disc plane of u at   t(u) = <C, C'> / C'_z
//   it lies in that disc when              phi(u) = |P(t(u)) - C(u)|^2 - r(u)^2 <= 0
//   boundary points solve                  f1 = <P - C, C'> = 0, f2 = |P - C|^2 - r^2 = 0
// Candidates: Newton's method on (f1, f2) from the FP32 leaf hit; roots of
// phi on the leaf interval (sampled, bracketed, then polished by Newton);
// the end discs when the leaf touches u = 0 or 1; t = 0 when the origin lies
// in one of the leaf's discs. The smallest candidate in [0, tmax) is the hit.

constexpr int kRefineAbove = 16;         // refine pairs of depth > 16
constexpr double kNewtonTol = 1e-9;      // relative residuals of an accepted Newton point
constexpr int kCurveSamples = 64;        // phi samples over the whole curve (local minima are searched)

struct Curve64 {
    double q[4][4];                      // control points in the FP64 ray frame (x, y, z, r)
    double scale;                        // largest control-point coordinate
};

// quad: F is a quadratic table (12 rows), taken as its exact cubic elevation
__device__ __forceinline__ bool curve_in_ray_frame(const float *R, int64_t rs, const float *F,
                                                   int64_t fs, Curve64 &c, double *frame = nullptr,
                                                   bool quad = false)
{
    const double ox = R[0], oy = R[rs], oz = R[2 * rs];
    const double dx = R[3 * rs], dy = R[4 * rs], dz = R[5 * rs];
    const double n2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(n2 > 0.0) || !(n2 < INFINITY)) return false;
    const double il = 1.0 / sqrt(n2);
    const double w[3] = {dx * il, dy * il, dz * il};
    double u[3], v[3];
    make_onb(w[0], w[1], w[2], u, v);
    if (frame) {
#pragma unroll
        for (int k = 0; k < 3; ++k) { frame[k] = u[k]; frame[3 + k] = v[k]; frame[6 + k] = w[k]; }
    }
    double P[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = quad ? 4 * (k == 3 ? 2 : k) + j : 4 * k + j;
            P[k][j] = (double)F[row * fs];
        }
    if (quad) {                      // P holds p0, p1, p2, p2: elevate
        double e1[4], e2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            e1[j] = (P[0][j] + 2.0 * P[1][j]) / 3.0;
            e2[j] = (2.0 * P[1][j] + P[2][j]) / 3.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) { P[1][j] = e1[j]; P[2][j] = e2[j]; }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double ex = P[k][0] - ox;
        const double ey = P[k][1] - oy;
        const double ez = P[k][2] - oz;
        c.q[k][0] = fma(ex, u[0], fma(ey, u[1], ez * u[2]));
        c.q[k][1] = fma(ex, v[0], fma(ey, v[1], ez * v[2]));
        c.q[k][2] = fma(ex, w[0], fma(ey, w[1], ez * w[2]));
        c.q[k][3] = P[k][3];
    }
    c.scale = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c.scale = fmax(c.scale, fmax(fabs(c.q[k][0]), fmax(fabs(c.q[k][1]), fabs(c.q[k][2]))));
    return true;
}

// A boundary point needs a disc plane: where C'(u) vanishes (a zero end
// tangent, a cusp) <P - C, C'> = 0 holds for every P, and |P - C| = r(u)
// would describe a sphere, not the swept solid.
__device__ __forceinline__ bool has_disc(const Curve64 &c, const double D[4])
{
    return sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) > 1e-12 * c.scale;
}

// C(u) (with radius), D = C'(u)/3 (with r'/3) and E = C''(u)/6 (xyz)
__device__ __forceinline__ void eval_curve(const Curve64 &c, double u, double C[4], double D[4], double E[3])
{
    const double v = 1.0 - u;
    const double b0 = v * v * v, b1 = 3.0 * u * v * v, b2 = 3.0 * u * u * v, b3 = u * u * u;
    const double e0 = v * v, e1 = 2.0 * u * v, e2 = u * u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        C[k] = fma(b0, c.q[0][k], fma(b1, c.q[1][k], fma(b2, c.q[2][k], b3 * c.q[3][k])));
        D[k] = fma(e0, c.q[1][k] - c.q[0][k], fma(e1, c.q[2][k] - c.q[1][k], e2 * (c.q[3][k] - c.q[2][k])));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        E[k] = fma(v, c.q[2][k] - 2.0 * c.q[1][k] + c.q[0][k], u * (c.q[3][k] - 2.0 * c.q[2][k] + c.q[1][k]));
}

// Normal of the disc at an end of the curve whose tangent vanishes (squared
// length at most 2^-40 of the squared chord; p1 = p0 or p2 = p3): the disc
// planes of the nearby u converge to the plane normal to the next
// control-polygon edge from that end (p2 - p0, resp. p3 - p1), or to the
// chord if that vanishes too. D (C'/3 at u) is replaced by that direction;
// elsewhere it is left alone.
__device__ __forceinline__ void end_disc_normal(const Curve64 &c, double u, double D[4])
{
    if (u != 0.0 && u != 1.0) return;
    const double ax = c.q[3][0] - c.q[0][0], ay = c.q[3][1] - c.q[0][1], az = c.q[3][2] - c.q[0][2];
    const double lim = 0x1p-40 * (ax * ax + ay * ay + az * az);
    if (D[0] * D[0] + D[1] * D[1] + D[2] * D[2] > lim) return;
    const int from = u == 0.0 ? 0 : 1, to = u == 0.0 ? 2 : 3;     // p2 - p0 or p3 - p1
    double nx = c.q[to][0] - c.q[from][0], ny = c.q[to][1] - c.q[from][1], nz = c.q[to][2] - c.q[from][2];
    if (nx * nx + ny * ny + nz * nz <= lim) { nx = ax; ny = ay; nz = az; }
    D[0] = nx;
    D[1] = ny;
    D[2] = nz;
}

// Ray point in the disc plane at u, and its signed excess |P-C|^2 - r^2.
__device__ __forceinline__ bool disc_point(const Curve64 &c, double u, double &t, double &phi)
{
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    end_disc_normal(c, u, D);
    if (D[2] == 0.0) return false;
    t = (C[0] * D[0] + C[1] * D[1] + C[2] * D[2]) / D[2];
    const double h = t - C[2];
    phi = C[0] * C[0] + C[1] * C[1] + h * h - C[3] * C[3];
    return true;
}

// phi(u) D_z^2 without the division: (C_x^2 + C_y^2 - r^2) D_z^2 +
// (C_x D_x + C_y D_y)^2 (the ray point's offset from the disc centre along
// the ray is (C_x D_x + C_y D_y) / D_z). Same sign as phi where the disc
// plane crosses the ray (D_z != 0); for the root search, which needs the
// sign and, within a narrow bracket where D_z barely changes, the shape.
__device__ __forceinline__ bool disc_excess_scaled(const Curve64 &c, double u, double &g)
{
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    end_disc_normal(c, u, D);
    if (D[2] == 0.0) return false;
    const double a = C[0] * D[0] + C[1] * D[1];
    g = (C[0] * C[0] + C[1] * C[1] - C[3] * C[3]) * (D[2] * D[2]) + a * a;
    return true;
}

// Does phi have a minimum inside the sample interval next to the end u (0 or
// 1), given that the end sample is the lower of the two? Only if phi turns
// there: it falls from u = 0, or rises into u = 1. From the slope of phi at
// the end (t = N / D_z with N = <C, D>, D = C'/3, D' = 2E):
//   phi' = 6 (C_x D_x + C_y D_y) + 2 (t - C_z)(t' - 3 D_z) - 6 r D_r,
//   t'   = ((3 |D|^2 + 2 <C, E>) D_z - 2 N E_z) / D_z^2.
// At a vanishing end tangent (no disc plane of its own; the limit plane
// serves) the slope is not formed and the interval is searched.
__device__ __forceinline__ bool end_turns(const Curve64 &c, double u)
{
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    const double ax = c.q[3][0] - c.q[0][0], ay = c.q[3][1] - c.q[0][1], az = c.q[3][2] - c.q[0][2];
    if (D[0] * D[0] + D[1] * D[1] + D[2] * D[2] <= 0x1p-40 * (ax * ax + ay * ay + az * az)) return true;
    if (D[2] == 0.0) return true;
    const double N = C[0] * D[0] + C[1] * D[1] + C[2] * D[2];
    const double t = N / D[2];
    const double dN = 3.0 * (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) + 2.0 * (C[0] * E[0] + C[1] * E[1] + C[2] * E[2]);
    const double dt = (dN * D[2] - 2.0 * N * E[2]) / (D[2] * D[2]);
    const double dphi = 6.0 * (C[0] * D[0] + C[1] * D[1]) + 2.0 * (t - C[2]) * (dt - 3.0 * D[2]) - 6.0 * C[3] * D[3];
    return u == 0.0 ? !(dphi >= 0.0) : !(dphi <= 0.0);       // NaN: searched
}

// t of a boundary point known to lie on the circle of the disc at u (C, D
// from eval_curve) whose plane crossing is t_plane = <C, D> / D_z. On the
// circle the same point is also C_z +- sqrt(r^2 - C_x^2 - C_y^2). The plane
// form loses about |C| |D| / |D_z| units of rounding as the disc plane turns
// towards the ray (D_z -> 0, near-collinear curves seen along their normal);
// the circle form loses about r^2 / sqrt(r^2 - C_x^2 - C_y^2) as the ray
// grazes the circle. The better conditioned form is returned, its sign
// taken from the plane form.
__device__ __forceinline__ double circle_t(const double C[4], const double D[4], double t_plane)
{
    const double rest = C[3] * C[3] - C[0] * C[0] - C[1] * C[1];
    if (!(rest > 0.0)) return t_plane;
    const double sr = sqrt(rest);
    const double e_plane = sqrt((C[0] * C[0] + C[1] * C[1] + C[2] * C[2]) * (D[0] * D[0] + D[1] * D[1] + D[2] * D[2])) /
                           fabs(D[2]);
    const double e_circle = C[3] * C[3] / sr;
    if (!(e_circle < e_plane)) return t_plane;
    return t_plane >= C[2] ? C[2] + sr : C[2] - sr;
}

// Newton's method on (f1, f2) from (t, u): true when it converges to a
// boundary point of the swept solid (entry or exit).
__device__ __forceinline__ bool newton_surface(const Curve64 &c, double &t, double &u)
{
    for (int it = 0; it < 10; ++it) {
        double C[4], D[4], E[3];
        eval_curve(c, u, C, D, E);
        const double h = t - C[2];
        const double f1 = h * D[2] - C[0] * D[0] - C[1] * D[1];
        const double f2 = C[0] * C[0] + C[1] * C[1] + h * h - C[3] * C[3];
        const double dd = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
        const double a11 = D[2];
        const double a12 = -3.0 * dd + 2.0 * (-C[0] * E[0] - C[1] * E[1] + h * E[2]);
        const double a21 = 2.0 * h;
        const double a22 = -6.0 * f1 - 6.0 * C[3] * D[3];
        const double det = a11 * a22 - a12 * a21;
        if (!(fabs(det) > 0.0)) return false;
        const double dt = (-f1 * a22 + f2 * a12) / det;
        const double du = (-f2 * a11 + f1 * a21) / det;
        t += dt;
        u += du;
        if (!(fabs(u) < 4.0) || !isfinite(t)) return false;
        if (fabs(du) <= 4e-16 && fabs(dt) <= 4e-16 * fabs(t)) break;
    }
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    const double h = t - C[2];
    const double scale = fmax(C[3] * C[3], 1e-300);
    const double f1 = h * D[2] - C[0] * D[0] - C[1] * D[1];
    const double f2 = C[0] * C[0] + C[1] * C[1] + h * h - C[3] * C[3];
    const double dn = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    // the residual floor is set by cancellation in C (control points far
    // from the ray), so the test is loose; near a tangent ray a point that
    // passes it can still lie measurably off the surface (see bracket_polish)
    return has_disc(c, D) && fabs(f2) <= kNewtonTol * scale && fabs(f1) <= kNewtonTol * C[3] * dn;
}

// Narrow a sign change of phi on [lo, hi] (lo_in: phi(lo) <= 0) to a
// bracket of at most 2^-53, then polish the root by Newton's method, kept
// only if it stays within a few final brackets (a polish that wanders
// further follows the residual's rounding, not the root); returns the
// boundary point in (t, u).
// The bracket is narrowed by the ITP method (interpolate, truncate, project;
// Oliveira and Takahashi, ACM Trans. Math. Softw. 47(1), 2020): each step
// takes the false-position estimate from the end values, moves it towards
// the midpoint by 0.2 (width)^2 / (initial width) (at least the final
// bracket), and keeps it within a distance of the midpoint that shrinks as
// the step budget is used up. It never takes more than one step beyond
// bisection, and on the simple roots that phi has where the ray crosses the
// boundary it takes about ten (a wave runs the steps of its slowest lane;
// bisection took 44).
__device__ __forceinline__ bool boundary_root(const Curve64 &c, double lo, double hi, bool lo_in, double &t,
                                              double &u)
{
    constexpr double kEps = 0x1p-54;                // half the final bracket
    // g = phi with the sign that makes g(lo) <= 0 <= g(hi). It only places
    // the estimate (the bracket follows the sign of phi, as in bisection),
    // so it is kept in FP32, which saves registers: the estimate's relative
    // error of about 2^-24 still shrinks the bracket by about that factor a
    // step near the root.
    const float sg = lo_in ? 1.0f : -1.0f;
    float gl = 0.0f, gh = 0.0f;
    {
        double pl, ph;
        if (disc_excess_scaled(c, lo, pl) && disc_excess_scaled(c, hi, ph)) {
            gl = sg * (float)pl;
            gh = sg * (float)ph;
        }
    }
    const float k1 = 0.2f / (float)(hi - lo);
    const int nmax = ilogb((hi - lo) / (2.0 * kEps)) + 2;       // bisection's steps, rounded up, plus one
    for (int j = 0; j <= nmax && hi - lo > 2.0 * kEps; ++j) {
        const double w = hi - lo, mid = 0.5 * (lo + hi);
        double xf = mid;
        if (gl <= 0.0f && gh >= 0.0f && gh > gl) xf = lo + w * (double)(gl / (gl - gh));
        const double s = mid >= xf ? 1.0 : -1.0;
        // at least the final bracket: an estimate that lands on the root
        // then still steps past it, and the far end moves as well
        const double delta = fmax((double)k1 * w * w, 2.0 * kEps);
        const double xt = delta <= fabs(mid - xf) ? xf + s * delta : mid;
        const double r = ldexp(kEps, nmax - j) - 0.5 * w;
        double x = fabs(xt - mid) <= r ? xt : mid - s * r;
        if (!(x > lo && x < hi)) x = mid;
        if (!(x > lo && x < hi)) break;
        double xphi;
        if (!disc_excess_scaled(c, x, xphi)) return false;
        if ((xphi <= 0.0) == lo_in) {
            lo = x;
            gl = sg * (float)xphi;
        } else {
            hi = x;
            gh = sg * (float)xphi;
        }
    }
    u = 0.5 * (lo + hi);
    double phi;
    if (!disc_point(c, u, t, phi)) return false;
    {
        double C[4], D[4], E[3];
        eval_curve(c, u, C, D, E);
        if (!has_disc(c, D)) return false;
        t = circle_t(C, D, t);
    }
    double tn = t, un = u;
    if (newton_surface(c, tn, un) && fabs(un - u) <= 4.0 * (hi - lo) + 0x1p-50) {
        t = tn;
        u = un;
    }
    return true;
}

// A Newton point re-derived from a sign change of phi around it. Near a
// tangent ray the boundary point is ill-conditioned: a residual small enough
// to pass Newton's test still moves t by far more than rounding (a residual
// e * r^2 moves t by about e * r / sqrt(2 * penetration / r)). Brackets of
// growing width around u are tried; the first with a sign change is
// narrowed to its root. Without one the point is kept.
__device__ __forceinline__ void bracket_polish(const Curve64 &c, double &t, double &u)
{
    double w = 0x1p-32;
    for (int it = 0; it < 8; ++it, w *= 8.0) {
        double ta, pa, tb, pb;
        if (!disc_point(c, u - w, ta, pa) || !disc_point(c, u + w, tb, pb)) return;
        if ((pa <= 0.0) != (pb <= 0.0)) {
            double tt, uu;
            if (boundary_root(c, u - w, u + w, pa <= 0.0, tt, uu)) {
                t = tt;
                u = uu;
            }
            return;
        }
    }
}

// Boundary points of the swept solid along the ray with u in [ua, ub]; the
// earliest with t in [tlo, thi] (the part of the ray the leaf owns) and below
// tmax is kept in (t_best, u_best). (t0, u0) is the FP32 leaf hit. Also the
// end discs when the interval reaches u = 0 or 1, and t = 0 when the origin
// lies in one of the discs. The earliest boundary point of the solid is its
// entry (or the origin, when inside), so no entry/exit classification is
// needed.
// The search runs in two passes so that the lanes of a wave stay together:
// the first samples phi at the NS + 1 parameters and records, per sample
// interval, the events that need a search (a sign change of phi, a local
// minimum of phi above zero, a crossing of the disc plane through the origin)
// as bit masks; the second searches the recorded events one after another.
// A wave then runs one search per event of its busiest lane, not the union
// of every lane's searches at every sample.
template <int NS>
__device__ __forceinline__ void leaf_candidates(const Curve64 &c, double ua, double ub, double tlo, double thi,
                                                double tmax, double t0, double u0, double &t_best,
                                                double &u_best)
{
    constexpr int kWords = (NS + 1 + 31) / 32;
    auto take = [&](double t, double u) {
        if (t >= tlo && t <= thi && t < tmax && t < t_best) { t_best = t; u_best = u; }
    };
    {
        double t = t0, u = u0;
        if (newton_surface(c, t, u)) {
            bracket_polish(c, t, u);
            if (u >= ua && u <= ub) take(t, u);
        }
    }
    const double h = (ub - ua) / NS;
    auto at = [&](int k) { return k == NS ? ub : ua + h * k; };
    // sample k (0..NS): inside (phi <= 0) and t <= 0 flags; events on (k-1, k]
    uint32_t in_m[kWords], tneg_m[kWords], sign_m[kWords], min_m[kWords], org_m[kWords];
#pragma unroll
    for (int q = 0; q < kWords; ++q) in_m[q] = tneg_m[q] = sign_m[q] = min_m[q] = org_m[q] = 0u;
    // the first sample counts as a minimum (event 1) only where phi turns
    // inside the first interval
    double pt = 0.0, pphi = 0.0, ppphi = ua == 0.0 && !end_turns(c, 0.0) ? -INFINITY : INFINITY;
    bool pok = disc_point(c, ua, pt, pphi);
    if (pok && pphi <= 0.0) in_m[0] |= 1u;
    if (pok && pt <= 0.0) tneg_m[0] |= 1u;
    for (int k = 1; k <= NS; ++k) {
        double ct = 0.0, cphi = 0.0;
        const bool cok = disc_point(c, at(k), ct, cphi);
        const uint32_t bit = 1u << (k & 31);
        if (cok && cphi <= 0.0) in_m[k >> 5] |= bit;
        if (cok && ct <= 0.0) tneg_m[k >> 5] |= bit;
        if (pok && cok) {
            if ((pphi <= 0.0) != (cphi <= 0.0)) sign_m[k >> 5] |= bit;
            else if (pphi > 0.0 && cphi > pphi && ppphi > pphi) min_m[k >> 5] |= bit;
            if ((pt <= 0.0) != (ct <= 0.0) && (pphi <= 0.0 || cphi <= 0.0) && tlo <= 0.0) org_m[k >> 5] |= bit;
        }
        ppphi = pok ? pphi : INFINITY;
        pt = ct; pphi = cphi; pok = cok;
    }
    // phi still falling at the last sample: a dip can sit between the last
    // two samples (as at a stalled end, where the disc planes turn fast as
    // u -> 1), where phi turns before the end; recorded as the event of a
    // minimum at sample NS - 1 (searched on (u[NS-2], u[NS]), which holds it)
    if (pok && pphi > 0.0 && ppphi > pphi && (ub < 1.0 || end_turns(c, 1.0)))
        min_m[NS >> 5] |= 1u << (NS & 31);
    // masks are indexed with unrolled selects (no dynamic register indexing)
    auto flag = [&](const uint32_t *m, int k) {
        uint32_t w = 0u;
#pragma unroll
        for (int q = 0; q < kWords; ++q) w = q == (k >> 5) ? m[q] : w;
        return ((w >> (k & 31)) & 1u) != 0u;
    };
    auto next_event = [&](uint32_t *m) {       // lowest recorded event, removed from the mask
        int k = -1;
#pragma unroll
        for (int q = kWords - 1; q >= 0; --q)
            if (m[q]) k = 32 * q + __builtin_ctz(m[q]);
#pragma unroll
        for (int q = 0; q < kWords; ++q)
            if (k >= 0 && q == (k >> 5)) m[q] &= m[q] - 1u;
        return k;
    };
    // sign changes: one boundary point between the samples
    for (int k; (k = next_event(sign_m)) >= 0;) {
        {
            double t, u;
            if (boundary_root(c, at(k - 1), at(k), flag(in_m, k - 1), t, u)) take(t, u);
        }
    }
    // a local minimum of phi above zero at sample k-1: a dip below zero
    // narrower than the sampling has two boundary points in (u[k-2], u[k]).
    // The dip is searched by Brent's minimisation (Brent, Algorithms for
    // Minimization without Derivatives, 1973, ch. 5): a parabola through
    // the three best points so far, replaced by a golden-section step
    // whenever its step is not acceptable, from the lowest sample. It stops
    // at the first point with phi <= 0, or once the bracket around the best
    // point is 2^-33 of the initial one (where 48 golden-section steps end,
    // 0.618^48), in about a third of their evaluations.
    for (int k; (k = next_event(min_m)) >= 0;) {
        {
            constexpr double g = 0.38196601125010515;         // golden-section step
            double a = at(k >= 2 ? k - 2 : 0), b = at(k), tt;
            const double tol = (b - a) * 0x1p-35;
            double x = at(k - 1), fx = 0.0;
            bool ok = disc_point(c, x, tt, fx);
            double xw = x, xv = x, fw = fx, fv = fx, d = 0.0, e = 0.0;
            for (int it = 0; ok && it < 64 && fx > 0.0; ++it) {
                const double m = 0.5 * (a + b);
                if (fabs(x - m) <= 2.0 * tol - 0.5 * (b - a)) break;
                bool gold = true;
                if (fabs(e) > tol) {
                    const double r = (x - xw) * (fx - fv);
                    double q = (x - xv) * (fx - fw);
                    double p = (x - xv) * q - (x - xw) * r;
                    q = 2.0 * (q - r);
                    if (q > 0.0) p = -p;
                    else q = -q;
                    const double e_old = e;
                    e = d;
                    if (fabs(p) < fabs(0.5 * q * e_old) && p > q * (a - x) && p < q * (b - x)) {
                        d = p / q;                               // the parabola's step
                        const double un = x + d;
                        if (un - a < 2.0 * tol || b - un < 2.0 * tol) d = m >= x ? tol : -tol;
                        gold = false;
                    }
                }
                if (gold) {
                    e = (x >= m ? a : b) - x;
                    d = g * e;
                }
                const double un = fabs(d) >= tol ? x + d : x + (d > 0.0 ? tol : -tol);
                double fu;
                ok = disc_point(c, un, tt, fu);
                if (!ok) break;
                if (fu <= fx) {
                    if (un >= x) a = x;
                    else b = x;
                    xv = xw; fv = fw;
                    xw = x; fw = fx;
                    x = un; fx = fu;
                } else {
                    if (un < x) a = un;
                    else b = un;
                    if (fu <= fw || xw == x) {
                        xv = xw; fv = fw;
                        xw = un; fw = fu;
                    } else if (fu <= fv || xv == x || xv == xw) {
                        xv = un; fv = fu;
                    }
                }
            }
            if (ok && fx <= 0.0) {
                // the minimisation's bracket ends lie above zero (samples,
                // or points it evaluated before the first one at or below
                // zero), so they bracket the two boundary points more
                // tightly than the samples
                const double um = x;
                double t, u;
                if (boundary_root(c, a, um, false, t, u)) take(t, u);
                if (boundary_root(c, um, b, true, t, u)) take(t, u);
            }
        }
    }
    // the disc plane sweeps through the origin: is the origin in that disc?
    for (int k; (k = next_event(org_m)) >= 0;) {
        {
            double lo = at(k - 1), hi = at(k);
            const bool lo_neg = flag(tneg_m, k - 1);
            for (int it = 0; it < 64; ++it) {
                const double mid = 0.5 * (lo + hi);
                double mt, mphi;
                if (!disc_point(c, mid, mt, mphi)) break;
                if ((mt <= 0.0) == lo_neg) lo = mid; else hi = mid;
            }
            const double uz = 0.5 * (lo + hi);
            double C[4], D[4], E[3];
            eval_curve(c, uz, C, D, E);
            if (C[0] * C[0] + C[1] * C[1] + C[2] * C[2] <= C[3] * C[3]) take(0.0, uz);
        }
    }
    // end discs
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        if ((e == 0 && ua > 0.0) || (e == 1 && ub < 1.0)) continue;
        double C[4], D[4], E[3];
        eval_curve(c, (double)e, C, D, E);
        end_disc_normal(c, (double)e, D);      // a vanishing end tangent: the limit plane
        if (D[2] == 0.0) continue;
        const double tc = (C[0] * D[0] + C[1] * D[1] + C[2] * D[2]) / D[2];
        const double hz = tc - C[2];
        if (C[0] * C[0] + C[1] * C[1] + hz * hz <= C[3] * C[3]) take(tc, (double)e);
    }
}

struct Lane {
    Node c;                       // current node, {p, d, t0, t1} in the ray frame
    Node root;                    // the pair's root (replays of the split rules start here)
    float lo, hi;                 // cropped t interval of the current node
    float tmax, t;                // ray tmax; hit distance once found
    uint32_t bits, start, size;   // Section 3.3: pending-sibling bits, integer interval (start:
                                  // bits 0..22; bit 31 set when the pair's end nodes may stall,
                                  // see stall_possible)
    uint32_t min_size;            // leaf size 2^(23 - depth)
    uint32_t cached;              // size of the pending children whose parent is cached (0: none)
    int32_t waiting;              // refinement: parked at its first leaf until the wave decides it
    float ru;                     //   the FP32 u of the leaf hit (Newton's start)
    int32_t scene;                // batched: the problem this pair belongs to
    int32_t pair;                 // index of the pair within its problem
    float slack;                  // conservative mode: bound on across-ray rounding of any node
                                  // (negative: a pair of depth <= 16, searched by the plain rules)
    int32_t trips, splits, backtracks;
    float u;                      // u of a leaf hit
    int32_t level;                // level of a leaf hit
};

enum { kGoOn = 0, kHit = 1, kMiss = 2 };

// Traversal variants: plain, counting, and conservative (for FP64 refinement:
// every pruning test is enlarged by a bound on its FP32 rounding error, so no
// surface point within that error is pruned; FP64 then decides).
enum { kPlain = 0, kCount = 1, kConservative = 2 };

// Per-lane LDS column (conflict-free: lane-contiguous rows of 64 floats) that
// caches the parent of the most recent split that left a sibling pending, so
// that the usual backtrack (to that sibling) rebuilds it with one split. Other
// backtracks replay the split rules from the root, re-read from the lane's
// root slot.
__device__ __forceinline__ void lds_put(float *col, const Node &r)
{
    const float *f = &r.p.x;
#pragma unroll
    for (int k = 0; k < 16; ++k) col[k * kWave] = f[k];
}

__device__ __forceinline__ void lds_get(const float *col, Node &r)
{
    float *f = &r.p.x;
#pragma unroll
    for (int k = 0; k < 16; ++k) f[k] = col[k * kWave];
}


// Each split rounds a node's position at the magnitude of its partial sum,
// which starts at the root's across-ray extent, so deep nodes inherit errors
// of a few ulp of that extent; 2^-18 of it is a generous bound.
__device__ __forceinline__ float root_slack(const Node &r)
{
    return (fabsf(r.p.x) + fabsf(r.p.y) + fabsf(r.d.x) + fabsf(r.d.y) +
            fabsf(r.t0.x) + fabsf(r.t0.y) + fabsf(r.t1.x) + fabsf(r.t1.y)) * 0x1p-18f;
}

// Pruning test of a node (Section 3.2): does the ray meet the conservative
// cylinder inside the node's cropped interval? `lo_used` / `hi_used` are the
// interval the test used (enlarged in conservative mode); a leaf's t is taken
// from its start.
template <int MODE, bool QUAD = false>
__device__ __forceinline__ bool node_visible(const Node &c, float lo, float hi, float slack, float &te,
                                             float &tx, float &lo_used, float &hi_used)
{
    float rad = conservative_radius<QUAD>(c);
    if (MODE == kConservative && slack >= 0.0f) {
        rad += slack + rad * 0x1p-18f;
        // an interval emptied on purpose (a parked lane, a cap plane parallel
        // to the ray that excludes it) must stay empty: no slack, since
        // infinite bounds would turn it into NaN, which fmaxf/fminf ignore
        const bool open = lo < INFINITY && hi > -INFINITY;
        const float tslack = open ? (fabsf(lo) + fabsf(hi < INFINITY ? hi : lo)) * 0x1p-17f : 0.0f;
        lo -= tslack;
        hi += tslack;
    }
    lo_used = lo;
    hi_used = hi;
    return unit_ray_cylinder(c.p, c.d, rad, te, tx) && fmaxf(te, lo) <= fminf(tx, hi);
}

// Bound on the rounding of a ray-plane distance c / n_z with c = <point, n>:
// the products' magnitudes over |n_z| (obliquity amplifies), plus the size
// of the result, at 2^-18 (64 ulp).
__device__ __forceinline__ float plane_slack(float px, float py, float pz, float nx, float ny, float nz, float t)
{
    return (fabsf(px * nx) + fabsf(py * ny) + fabsf(pz * nz)) * rcp(fabsf(nz)) * 0x1p-18f +
           fabsf(t) * 0x1p-18f;
}

// u of a leaf hit (Section 3.3): the hit point projected onto the leaf chord.
__device__ __forceinline__ float leaf_u(const Lane &L)
{
    const float cc = dot3(L.c.d.x, L.c.d.y, L.c.d.z, L.c.d.x, L.c.d.y, L.c.d.z);
    float ul = 0.0f;
    if (cc > 0.0f) {
        ul = dot3(-L.c.p.x, -L.c.p.y, L.t - L.c.p.z, L.c.d.x, L.c.d.y, L.c.d.z) * rcp(cc);
        ul = fminf(1.0f, fmaxf(0.0f, ul));
    }
    return fmaf(ul, (float)L.size * 0x1p-23f, (float)(L.start & kStartMask) * 0x1p-23f);
}

// FP64 decision of a pair of depth > 16 once the conservative search reaches
// its first leaf: the earliest boundary point of the swept solid along the
// ray over the whole curve, t in [0, tmax), from kCurveSamples samples of the
// disc excess (with the FP32 leaf hit as Newton's start). A leaf-local check
// (three leaves around the FP32 hit, then the whole curve if it failed) was
// measured first: at hair scale almost every leaf check failed (the FP32
// leaf lies more than a leaf from the entry), so it only added work.
// Arguments and result go by value: a reference to the caller's lane state
// or to the kernel's arguments would keep them in scratch memory for the
// whole kernel (the call is not inlined), every trip included.
struct Refined {
    double t = INFINITY, u = __builtin_nan("");
    bool hit = false;
    float nx = __builtin_nanf(""), ny = __builtin_nanf(""), nz = __builtin_nanf("");   // world space
};

// Outward unit normal of the swept solid at a refined hit (ray frame):
// at an end disc (u = 0 or 1) minus the start tangent or the end tangent
// (their limits where they vanish); on the side, where the surface is
// C(u) + r(u) e with e a unit vector normal to C'(u), the unit direction e
// from C(u) to the hit, tilted against the tangent T by the taper:
// e - r' / (|C'| - r <e, C''> / |C'|) T (the disc's normal plane turns with
// the curve, hence the curvature term). In the units of eval_curve (D = C'/3
// with r'/3, E = C''/6) the tilt is 3 D_r / (3 |D| - 2 r <e, E> / |D|). The
// origin inside the solid (t = 0) has no surface crossing: NaN.
__device__ __forceinline__ void solid_normal(const Curve64 &c, double t, double u, double n[3])
{
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    if (t == 0.0) {
        n[0] = n[1] = n[2] = __builtin_nan("");
        return;
    }
    if (u == 0.0 || u == 1.0) {
        end_disc_normal(c, u, D);
        const double s = (u == 0.0 ? -1.0 : 1.0) * rsqrt64(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        n[0] = s * D[0];
        n[1] = s * D[1];
        n[2] = s * D[2];
        return;
    }
    double ex = -C[0], ey = -C[1], ez = t - C[2];
    const double ie = rsqrt64(ex * ex + ey * ey + ez * ez);
    ex *= ie; ey *= ie; ez *= ie;
    const double dl = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    const double tilt = -3.0 * D[3] / (3.0 * dl - 2.0 * C[3] * (ex * E[0] + ey * E[1] + ez * E[2]) / dl);
    n[0] = ex + tilt * D[0] / dl;
    n[1] = ey + tilt * D[1] / dl;
    n[2] = ez + tilt * D[2] / dl;
}

// `fiber` >= 0 names the fiber directly (candidate lists); `tmax` is the
// FP64 limit of the search.
__device__ __noinline__ Refined refine_whole_curve(const float *rays, int64_t ray_stride, const float *fibers,
                                                   int64_t fiber_stride, const int32_t *pair_ray,
                                                   const int32_t *pair_fiber, int64_t i, int64_t fiber,
                                                   double tmax, float t0, float u0, bool normal, bool quad)
{
    Refined r;
    const int64_t ri = pair_ray ? (int64_t)pair_ray[i] : i;
    const int64_t fi = fiber >= 0 ? fiber : pair_fiber ? (int64_t)pair_fiber[i] : i;
    Curve64 cv;
    double frame[9];
    if (!curve_in_ray_frame(rays + ri, ray_stride, fibers + fi, fiber_stride, cv, frame, quad)) return r;
    double t = INFINITY, u = __builtin_nan("");
    leaf_candidates<kCurveSamples>(cv, 0.0, 1.0, 0.0, tmax, tmax, (double)t0, (double)u0, t, u);
    if (t < INFINITY) {
        r.t = t;
        r.u = u;
        r.hit = true;
        if (normal) {
            double n[3];
            solid_normal(cv, t, u, n);
            // back to world space: n.x u + n.y v + n.z w, unit length
            const double wx = n[0] * frame[0] + n[1] * frame[3] + n[2] * frame[6];
            const double wy = n[0] * frame[1] + n[1] * frame[4] + n[2] * frame[7];
            const double wz = n[0] * frame[2] + n[1] * frame[5] + n[2] * frame[8];
            const double il = rsqrt64(wx * wx + wy * wy + wz * wz);
            r.nx = (float)(wx * il);
            r.ny = (float)(wy * il);
            r.nz = (float)(wz * il);
        }
    }
    return r;
}

// One loop trip of the paper's iteration (Appendix C, final listing): a
// pruning test of the current node, then a descent, a leaf hit, a miss, or a
// jump to the deepest pending sibling.
// The descent (split, ordering, child) is straight-line code computed for
// every continuing lane; a lane that backtracks then overwrites its result
// with the rebuilt sibling. The new node thus has a single definition point,
// which spares the copies of the whole lane state that a merge of separately
// computed nodes costs, and a backtracking lane only adds the rebuild.
// The split of the current node (Section 3.1 / 3.2): centre offset and split
// tangent, the split plane's crossing tp with the ray, whether the ray meets
// both halves inside [te, tx], which half it meets first, and the interval
// of that half (narrowed at tp).
struct Split {
    V4 dp, tc;
    float nlo, nhi;
    bool both, near_right, oblique;
};

template <int MODE>
__device__ __forceinline__ void split_plane(const Lane &L, float te, float tx, Split &sp)
{
    // at a cusp (no split tangent) the split plane is normal to the chord
    const bool cusp = split_terms(L.c, sp.dp, sp.tc);
    const float nx = cusp ? L.c.d.x : sp.tc.x;
    const float ny = cusp ? L.c.d.y : sp.tc.y;
    const float nz = cusp ? L.c.d.z : sp.tc.z;
    const float qx = L.c.p.x + sp.dp.x, qy = L.c.p.y + sp.dp.y, qz = L.c.p.z + sp.dp.z;
    const float cs = dot3(qx, qy, qz, nx, ny, nz);
    const float tp = cs * rcp(nz);
    sp.oblique = nz != 0.0f;
    sp.nlo = L.lo;
    sp.nhi = L.hi;
    if (MODE == kConservative && L.slack >= 0.0f) {
        // visit both halves unless the crossing is clearly outside [te, tx];
        // narrow by the far side of tp's rounding bound
        const float ep = plane_slack(qx, qy, qz, nx, ny, nz, tp);
        sp.both = sp.oblique ? (te - ep < tp && tp < tx + ep)
                             : (cs == 0.0f || fabsf(cs) <= L.slack * (fabsf(nx) + fabsf(ny)));
        if (tp > te) sp.nhi = fminf(sp.nhi, tp + ep);
        else         sp.nlo = fmaxf(sp.nlo, tp - ep);
    } else {
        sp.both = sp.oblique ? (te < tp && tp < tx) : cs == 0.0f;
        if (tp > te) sp.nhi = fminf(sp.nhi, tp);
        else         sp.nlo = fmaxf(sp.nlo, tp);
    }
    // a plane parallel to the ray leaves the whole ray on the side of sign(-cs)
    sp.near_right = sp.oblique ? ((tp > te) != (nz > 0.0f)) : cs < 0.0f;
}

// Bookkeeping of a descent into the near half (Section 3.3: one level down,
// the far half pending when the ray meets both).
template <bool PC>
__device__ __forceinline__ void descend_state(Lane &L, const Split &sp)
{
    if (sp.oblique) { L.lo = sp.nlo; L.hi = sp.nhi; }
    L.size >>= 1;
    if (sp.both) {
        L.bits ^= L.size;
        if (PC) L.cached = L.size;
    }
    if (sp.near_right) L.start ^= L.size;
}

// Where a backtrack that misses the parent cache finds its pair's root: in
// the lane's registers (16 more VGPRs per lane, which the occupancy that
// the LDS queue allows can hold), so a replay starts without a memory
// access.
struct RegRoot {
    __device__ __forceinline__ void get(const Lane &L, Node &n) const { n = L.root; }
};

// What the normal of a leaf hit needs from the leaf, taken before the trip
// moves on to a child: the ray-frame vector from the leaf chord's point at
// the hit's projection to the hit point, and whether the hit entered the
// leaf through a plane (the interval's start) rather than the cylinder's
// side.
struct HitGeo {
    float vx, vy, vz;
    bool plane;
};

__device__ __forceinline__ HitGeo hit_geo(const Node &c, float t, bool plane)
{
    const float cc = dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z);
    float ul = 0.0f;
    if (cc > 0.0f) {
        ul = dot3(-c.p.x, -c.p.y, t - c.p.z, c.d.x, c.d.y, c.d.z) * rcp(cc);
        ul = fminf(1.0f, fmaxf(0.0f, ul));
    }
    return HitGeo{-fmaf(ul, c.d.x, c.p.x), -fmaf(ul, c.d.y, c.p.y), t - fmaf(ul, c.d.z, c.p.z), plane};
}

// Stalled end nodes. Where an end tangent vanishes the curve leaves that end
// with vanishing speed, and the end nodes' chords shrink like 4^-level: from
// some level on, all their control points coincide to FP32 precision, every
// test on them is rounding noise, and a search through them can visit
// thousands of nodes. A node that holds an end of the curve (u = 0 or u = 1)
// and whose extent -- the largest squared length of its chord and end
// tangents -- is at most (2^-20 X)^2 (X: the largest ray-frame coordinate of
// the root's control points) and at most 2^-16 of the root's extent times
// 4^-level, is therefore a leaf. Near a vanishing end tangent the curve keeps
// a fixed direction, so such a node's end planes stay perpendicular to its
// chord and its cylinder stays closed. Cusps (interior stalls, where the
// direction reverses) are not cut short.
__device__ __forceinline__ float node_extent(const Node &c)
{
    const float cc = dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z);
    const float a0 = dot3(c.t0.x, c.t0.y, c.t0.z, c.t0.x, c.t0.y, c.t0.z);
    const float a1 = dot3(c.t1.x, c.t1.y, c.t1.z, c.t1.x, c.t1.y, c.t1.z);
    return fmaxf(cc, fmaxf(a0, a1));
}

// The end nodes' outer tangents shrink exactly like 2^-level (halving is
// exact), so their extents stay at least |t0|^2 4^-level (start) and
// |t1|^2 4^-level (end): a pair whose root end tangents both exceed 2^-15 of
// the root's extent (a factor 2 above the bound, against rounding) can never
// stall, and its lanes skip the test. Decided in the setup round, with the
// root's other tests.
__device__ __forceinline__ bool stall_possible(const Node &r)
{
    const float a0 = dot3(r.t0.x, r.t0.y, r.t0.z, r.t0.x, r.t0.y, r.t0.z);
    const float a1 = dot3(r.t1.x, r.t1.y, r.t1.z, r.t1.x, r.t1.y, r.t1.z);
    const float ext = node_extent(r);
    return a0 <= 0x1p-15f * ext || a1 <= 0x1p-15f * ext;
}

// (2^-20 X)^2 of the pair's root (X: its largest ray-frame coordinate)
__device__ __forceinline__ float stall_abs(const Node &r)
{
    const float ex = r.p.x + r.d.x, ey = r.p.y + r.d.y, ez = r.p.z + r.d.z;     // p3
    float X = fmaxf(fabsf(r.p.x), fmaxf(fabsf(r.p.y), fabsf(r.p.z)));
    X = fmaxf(X, fmaxf(fabsf(r.p.x + r.t0.x), fmaxf(fabsf(r.p.y + r.t0.y), fabsf(r.p.z + r.t0.z))));
    X = fmaxf(X, fmaxf(fabsf(ex - r.t1.x), fmaxf(fabsf(ey - r.t1.y), fabsf(ez - r.t1.z))));
    X = fmaxf(X, fmaxf(fabsf(ex), fmaxf(fabsf(ey), fabsf(ez))));
    return 0x1p-40f * X * X;
}

__device__ __forceinline__ bool stalled_end(const Lane &L)
{
    if (!(L.start & kStallBit)) return false;
    const float s = (float)L.size * 0x1p-23f;                 // 2^-level
    const float rel = 0x1p-16f * node_extent(L.root) * s * s;
    // the chord alone fails the relative bound at every regular node: the
    // extent (at least the chord) is only formed where it passes
    const float cc = dot3(L.c.d.x, L.c.d.y, L.c.d.z, L.c.d.x, L.c.d.y, L.c.d.z);
    if (!(cc <= rel)) return false;
    const float e = node_extent(L.c);
    const uint32_t start = L.start & kStartMask;
    const bool end = start == 0u || start + L.size == kRootSize;
    return end && e <= rel && e <= stall_abs(L.root);
}

// PC: the parent cache in LDS (else every backtrack replays from the root)
template <int MODE, bool QUAD, bool PC, class Root>
__device__ __forceinline__ int trip(Lane &L, const Root &root, float *col, HitGeo &hg)
{
    float te, tx, lo, hi;
    bool vis = node_visible<MODE, QUAD>(L.c, L.lo, L.hi, L.slack, te, tx, lo, hi);
    const bool leaf = L.size <= L.min_size || stalled_end(L);
    if (MODE == kConservative && vis && leaf && L.slack >= 0.0f) {
        // refinement: the first leaf reached means the solid may be hit; park
        // the lane (empty interval, no pending sibling) until the wave decides
        // its parked pairs in FP64, keeping the leaf hit as Newton's start
        L.t = fmaxf(te, lo);
        L.ru = leaf_u(L);
        L.bits = 0;
        L.lo = INFINITY;
        L.hi = -INFINITY;
        L.waiting = 1;
        vis = false;
    }
    // A lane that stops here still runs the rest of the trip (its state is
    // not used again): without early returns the lane state keeps one set of
    // registers across the loop instead of being copied at every exit.
    int st = kGoOn;
    if (vis && leaf) {
        L.t = fmaxf(te, lo);
        hg = hit_geo(L.c, L.t, te < lo);
        L.u = leaf_u(L);
        L.level = 23 - (31 - __builtin_clz(L.size));
        st = kHit;
    }
    const bool over = ++L.trips > kMaxTrips;          // hang guard (each trip is a test)
    if ((!vis && L.bits == 0) || over) st = kMiss;
    // A backtracking lane first rebuilds the parent of its pending sibling
    // (Section 3.3: the deepest level with a pending sibling) -- the cached
    // parent, or a replay of the split rules from the root along the integer
    // path -- and then takes the same split as a descending lane: one split
    // per trip for every continuing lane.
    const bool back = !vis && st == kGoOn;
    if (back) {
        L.size = L.bits & (0u - L.bits);
        L.start ^= L.size;
        L.bits ^= L.size;
        L.start &= ~(L.size - 1u);
        if (PC && L.cached == L.size) {
            lds_get(col, L.c);
        } else {
            root.get(L, L.c);
            for (uint32_t b = kRootSize >> 1; b > L.size; b >>= 1) {
                V4 rdp, rtc;
                split_terms(L.c, rdp, rtc);
                take_child(L.c, rdp, rtc, (L.start & b) != 0u);
            }
        }
        L.cached = 0;
    }
    // Section 3.1 / 3.2: split plane through the centre, normal to the split
    // tangent; a descending lane goes to the half the ray meets first
    Split sp;
    split_plane<MODE>(L, te, tx, sp);
    const bool descend = vis && st == kGoOn;
    if (PC && descend && sp.both) lds_put(col, L.c);
    const bool right = back ? (L.start & L.size) != 0u : sp.near_right;
    take_child(L.c, sp.dp, sp.tc, right);
    if (back) {
        cap_interval(L.c, L.tmax, L.lo, L.hi);
    } else if (descend) {
        descend_state<PC>(L, sp);
    }
    // work counters (counting variant only), branch-free
    if (MODE == kCount) {
        L.splits += descend ? 1 : 0;
        L.backtracks += back ? 1 : 0;
    }
    return st;
}

// Normal at a leaf hit (Appendix C, the final computation of an
// intersection). A hit through the leaf cylinder's side gets the direction
// from the leaf chord's point at the hit's projection to the hit point. A hit
// through a plane (the start of the leaf's interval) whose point lies on the
// curve's start or end cap plane -- within (8 + 2 level) 2^-24 X, the node
// error bound of the leaf's level plus this test's own rounding, X the
// largest ray-frame coordinate of the control points -- gets that cap's
// outward normal: minus the start tangent, the end tangent, with the cap
// planes' fallbacks where a tangent vanishes (the nearer plane when both
// qualify). Other plane entries keep the radial direction. At depth 22 a
// leaf is shorter than FP32 resolves along the ray, so the first leaf can
// look empty and hand its hit to the next one through their common split
// plane: the tolerance keeps such hits on the cap. The vector is formed in
// the ray frame and turned back into world space with the frame of the
// pair's ray (rebuilt in FP64, as for the projection).
template <bool CAND>
__device__ __forceinline__ void leaf_normal(const Args &a, int64_t i, const Lane &L, const HitGeo &hg, float &nx,
                                            float &ny, float &nz)
{
    float vx = hg.vx, vy = hg.vy, vz = hg.vz;
    if (hg.plane) {
        const Node &r = L.root;
        const float cc = dot3(r.d.x, r.d.y, r.d.z, r.d.x, r.d.y, r.d.z);
        // cap normals: p1 - p0, else p2 - p0, else p3 - p0; p3 - p2, else p3 - p1, else p3 - p0
        float ax = r.t0.x, ay = r.t0.y, az = r.t0.z;
        if (negligible(ax, ay, az, cc)) { ax = r.d.x - r.t1.x; ay = r.d.y - r.t1.y; az = r.d.z - r.t1.z; }
        if (negligible(ax, ay, az, cc)) { ax = r.d.x; ay = r.d.y; az = r.d.z; }
        float bx = r.t1.x, by = r.t1.y, bz = r.t1.z;
        if (negligible(bx, by, bz, cc)) { bx = r.d.x - r.t0.x; by = r.d.y - r.t0.y; bz = r.d.z - r.t0.z; }
        if (negligible(bx, by, bz, cc)) { bx = r.d.x; by = r.d.y; bz = r.d.z; }
        const float ex = r.p.x + r.d.x, ey = r.p.y + r.d.y, ez = r.p.z + r.d.z;     // p3
        const float d0 = fabsf(L.t * az - dot3(r.p.x, r.p.y, r.p.z, ax, ay, az)) * rcp(vsqrt(dot3(ax, ay, az, ax, ay, az)));
        const float d1 = fabsf(L.t * bz - dot3(ex, ey, ez, bx, by, bz)) * rcp(vsqrt(dot3(bx, by, bz, bx, by, bz)));
        float X = 0.0f;
        X = fmaxf(X, fmaxf(fabsf(r.p.x), fmaxf(fabsf(r.p.y), fabsf(r.p.z))));
        X = fmaxf(X, fmaxf(fabsf(r.p.x + r.t0.x), fmaxf(fabsf(r.p.y + r.t0.y), fabsf(r.p.z + r.t0.z))));
        X = fmaxf(X, fmaxf(fabsf(ex - r.t1.x), fmaxf(fabsf(ey - r.t1.y), fabsf(ez - r.t1.z))));
        X = fmaxf(X, fmaxf(fabsf(ex), fmaxf(fabsf(ey), fabsf(ez))));
        const float tol = (float)(8 + 2 * L.level) * 0x1p-24f * X;
        const bool near1 = d1 < d0;
        if (fminf(d0, d1) <= tol) {
            vx = near1 ? bx : -ax;
            vy = near1 ? by : -ay;
            vz = near1 ? bz : -az;
        }
    }
    const int64_t ri = a.pair_ray && !CAND ? (int64_t)a.pair_ray[i] : i;
    const float *R = a.rays + ri;
    const int64_t rs = a.ray_stride;
    const double dx = R[3 * rs], dy = R[4 * rs], dz = R[5 * rs];
    const double il = rsqrt64(fma(dx, dx, fma(dy, dy, dz * dz)));
    const double w[3] = {dx * il, dy * il, dz * il};
    double u[3], v[3];
    make_onb(w[0], w[1], w[2], u, v);
    const double wx = fma((double)vx, u[0], fma((double)vy, v[0], (double)vz * w[0]));
    const double wy = fma((double)vx, u[1], fma((double)vy, v[1], (double)vz * w[1]));
    const double wz = fma((double)vx, u[2], fma((double)vy, v[2], (double)vz * w[2]));
    const double in = rsqrt64(fma(wx, wx, fma(wy, wy, wz * wz)));
    nx = (float)(wx * in);
    ny = (float)(wy * in);
    nz = (float)(wz * in);
}

// Write the result of pair i (Section 3.3: u from projecting the hit point
// onto the leaf chord; hit when t < tmax). A refined pair (depth > 16 under
// FI_FP64_REFINE) reports its FP64 surface hit, decided in FP64.
// `hg` is the leaf geometry of a plain hit; `ref` the FP64 result of a
// refined pair (used when `reached`). CAND: candidate lists (see Args).
template <int MODE, bool CAND = false>
__device__ __forceinline__ void finish(const Args &a, int64_t i, const Lane &L, bool reached,
                                       HitGeo hg = HitGeo{}, Refined ref = Refined{})
{
    float t = INFINITY, u = __builtin_nanf("");
    double t64 = INFINITY, u64 = __builtin_nan("");
    bool hit = false;
    if (MODE == kConservative && L.slack >= 0.0f) {
        if (reached) {
            t64 = ref.t;
            u64 = ref.u;
            t = (float)t64;
            u = (float)u64;
            hit = true;
        }
    } else if (reached && L.t < L.tmax) {
        t = L.t;
        u = L.u;
        t64 = t;
        u64 = u;
        hit = true;
    }
    if constexpr (CAND) {
        // candidate lists: a miss leaves the ray's nearest hit so far; a
        // hit (nearer by construction: tmax was shortened to it) replaces it
        if (!hit) return;
        a.fiber_out[i] = a.cand_fiber[a.cand_off[i] + a.cand_round];
    }
    a.t_out[i] = t;
    a.u_out[i] = u;
    a.hit_out[i] = hit ? 1 : 0;
    if (MODE == kConservative) {
        a.t64_out[i] = t64;
        a.u64_out[i] = u64;
    }
    if (MODE != kCount && a.normal_out) {
        float nx = __builtin_nanf(""), ny = nx, nz = nx;
        if (MODE == kConservative && L.slack >= 0.0f) {
            if (hit) { nx = ref.nx; ny = ref.ny; nz = ref.nz; }
        } else if (hit) {
            leaf_normal<CAND>(a, i, L, hg, nx, ny, nz);
        }
        a.normal_out[i] = nx;
        a.normal_out[a.n_pairs + i] = ny;
        a.normal_out[2 * a.n_pairs + i] = nz;
    }
    if (MODE == kCount) {
        int32_t *cn = a.counts + 4 * i;
        cn[0] = L.trips;
        cn[1] = L.splits;
        cn[2] = L.backtracks;
        cn[3] = hit ? L.level : -1;
    }
}

template <int MODE>
__device__ __forceinline__ void finish_invalid(const Args &a, int64_t i)
{
    a.t_out[i] = INFINITY;
    a.u_out[i] = __builtin_nanf("");
    a.hit_out[i] = 0;
    if (MODE == kConservative) {
        a.t64_out[i] = INFINITY;
        a.u64_out[i] = __builtin_nan("");
    }
    if (MODE != kCount && a.normal_out) {
        a.normal_out[i] = __builtin_nanf("");
        a.normal_out[a.n_pairs + i] = __builtin_nanf("");
        a.normal_out[2 * a.n_pairs + i] = __builtin_nanf("");
    }
    if (MODE == kCount) {
        int32_t *cn = a.counts + 4 * i;
        cn[0] = 0; cn[1] = 0; cn[2] = 0; cn[3] = -1;
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Scene of global pair g: offsets[s] <= g < offsets[s + 1] (empty scenes skipped).
__device__ __forceinline__ int find_scene(const int64_t *offsets, int n_scenes, int64_t g)
{
    int lo = 0, hi = n_scenes;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Load pair i and move it into the ray frame: the root node in the
// {p, d, t0, t1} form (Section 3.1), written to q[k * kQueue] (k = 0..15: p,
// d, t0, t1, each x, y, z, w) as each part is computed, so that the FP64
// frame and the finished root never take registers at the same time. False
// when the pair is a definite miss (bad index, depth, direction, tmax or a
// non-finite root).
// The projection runs once per pair in FP64 (full rate on this chip): the
// differences of the float32 control points and of the origin are exact in
// double, so p is the rounded frame position of p0 and d, t0, t1 are the
// rounded frame images of p3-p0, p1-p0, p3-p2 -- each component accurate to
// its own float32 ulp, including the tiny across-ray or along-ray parts of
// nearly parallel or nearly perpendicular tangents.
// `aos`, when given, holds the fibers as 16 consecutive floats each (see
// k_fibers_aos): a gathered fiber is then one or two cache lines instead of
// one line per coordinate row.
// In candidate mode (cand_off given) pair i is ray i against its candidate
// number cand_round; a ray without that candidate, or with an invalid one,
// is a definite miss too (its callers then leave the ray's nearest hit so far
// as it is), and tmax is the ray's tmax shortened to that hit.
// QUAD: the fiber table holds quadratics (12 rows: p0, p1, p2), loaded as
// their exact cubic elevation (t0 = 2/3 (p1 - p0), t1 = 2/3 (p2 - p1)).
template <bool CAND, bool QUAD = false>
__device__ __forceinline__ bool load_pair(const Args &a, int64_t i, float *q, float &tmax, uint32_t &depth,
                                          const float *aos)
{
    int64_t ri, fi;
    if constexpr (CAND) {
        const int64_t o = a.cand_off[i] + a.cand_round;
        if (o >= a.cand_off[i + 1] || o < 0 || o >= a.n_cand) return false;
        ri = i;
        fi = a.cand_fiber[o];
        depth = a.pair_depth ? (uint32_t)a.pair_depth[o] : (uint32_t)a.depth;
    } else {
        ri = a.pair_ray ? (int64_t)a.pair_ray[i] : i;
        fi = a.pair_fiber ? (int64_t)a.pair_fiber[i] : i;
        depth = a.pair_depth ? (uint32_t)a.pair_depth[i] : (uint32_t)a.depth;
    }
    if (ri < 0 || ri >= a.n_rays || fi < 0 || fi >= a.n_fibers || depth > FI_MAX_DEPTH) return false;
    const float *R = a.rays + ri;
    const int64_t rs = a.ray_stride;
    tmax = R[6 * rs];
    if (!(tmax == tmax)) return false;
    if constexpr (CAND) {
        if (a.t64_out) {
            // refined candidates: the FP64 nearest hit so far, rounded up
            // (the FP32 search prunes conservatively; FP64 decides)
            const double b = a.t64_out[i];
            float f = (float)b;
            if ((double)f < b) f = __uint_as_float(__float_as_uint(f) + 1u);     // b >= 0: one ulp up
            tmax = fminf(tmax, f);
        } else {
            tmax = fminf(tmax, a.t_out[i]);
        }
    }
    const float *F = aos ? aos + 16 * fi : a.fibers + fi;
    const int64_t fs = aos ? 1 : a.fiber_stride;
    const double dx = R[3 * rs], dy = R[4 * rs], dz = R[5 * rs];
    const double n2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(n2 > 0.0) || !(n2 < INFINITY)) return false;
    const double il = rsqrt64(n2);
    const double w[3] = {dx * il, dy * il, dz * il};
    double u[3], v[3];
    make_onb(w[0], w[1], w[2], u, v);
    bool finite = true;
    auto proj = [&](double ex, double ey, double ez, double ew, int k, bool check) {
        const float x = (float)fma(ex, u[0], fma(ey, u[1], ez * u[2]));
        const float y = (float)fma(ex, v[0], fma(ey, v[1], ez * v[2]));
        const float z = (float)fma(ex, w[0], fma(ey, w[1], ez * w[2]));
        if (check) finite = finite && isfinite(x) && isfinite(y) && isfinite(z);
        q[(4 * k) * kQueue] = x;
        q[(4 * k + 1) * kQueue] = y;
        q[(4 * k + 2) * kQueue] = z;
        q[(4 * k + 3) * kQueue] = (float)ew;
    };
    const float p0x = F[0], p0y = F[fs], p0z = F[2 * fs], p0w = F[3 * fs];
    proj((double)p0x - (double)R[0], (double)p0y - (double)R[rs], (double)p0z - (double)R[2 * rs], (double)p0w, 0,
         true);
    if constexpr (QUAD) {
        const float p2x = F[8 * fs], p2y = F[9 * fs], p2z = F[10 * fs], p2w = F[11 * fs];
        const float p1x = F[4 * fs], p1y = F[5 * fs], p1z = F[6 * fs], p1w = F[7 * fs];
        constexpr double k23 = 2.0 / 3.0;
        proj((double)p2x - p0x, (double)p2y - p0y, (double)p2z - p0z, (double)p2w - p0w, 1, true);
        proj(((double)p1x - p0x) * k23, ((double)p1y - p0y) * k23, ((double)p1z - p0z) * k23,
             ((double)p1w - p0w) * k23, 2, false);
        proj(((double)p2x - p1x) * k23, ((double)p2y - p1y) * k23, ((double)p2z - p1z) * k23,
             ((double)p2w - p1w) * k23, 3, false);
        return finite;
    }
    const float p3x = F[12 * fs], p3y = F[13 * fs], p3z = F[14 * fs], p3w = F[15 * fs];
    proj((double)p3x - p0x, (double)p3y - p0y, (double)p3z - p0z, (double)p3w - p0w, 1, true);
    proj((double)F[4 * fs] - p0x, (double)F[5 * fs] - p0y, (double)F[6 * fs] - p0z, (double)F[7 * fs] - p0w, 2,
         false);
    proj((double)p3x - F[8 * fs], (double)p3y - F[9 * fs], (double)p3z - F[10 * fs], (double)p3w - F[11 * fs], 3,
         false);
    return finite;
}

// The kernel of every call: each persistent 64-lane wave takes an even share
// of the call's pairs (of the whole scene table for a batch), contiguous so
// that its loads are coalesced. Pairs reach the lanes through a queue of
// prepared roots in LDS:
//  * a setup round, run by the whole wave when the queue cannot serve its
//    free lanes, loads up to 64 pairs (one per lane), moves them into the
//    ray frame in FP64 and tests their roots; pairs decided there (a miss, a
//    root that is the leaf, a bad pair) are written out at once, the others
//    are appended to the queue (root node, its cap interval, tmax, pair);
//  * at every trip, each free lane takes the next queued root (copying it to
//    its root slot for the backtracks that miss the parent cache), and its
//    first trip tests the root and takes the first split.
// Setup rounds thus run with every lane busy and pay their load latency
// once per up to 64 pairs, while a lane that finishes a pair waits no more
// than one trip for the next (a round of loads, the FP64 frame and the root
// test costs about three trips' time). The attribute sets the register
// budget; the LDS (queue and parent cache, 9.5 KiB) allows 16 waves per CU.

// A scene descriptor's fields that pair loading and finishing read, as
// wave-uniform values.
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x)
{
    return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32)) << 32) |
                     __builtin_amdgcn_readfirstlane((uint32_t)x));
}

__device__ __forceinline__ void uniform_scene(const Args &s, Args &o)
{
    o.rays = uniform_ptr(s.rays);
    o.ray_stride = uniform_i64(s.ray_stride);
    o.n_rays = uniform_i64(s.n_rays);
    o.fibers = uniform_ptr(s.fibers);
    o.fiber_stride = uniform_i64(s.fiber_stride);
    o.n_fibers = uniform_i64(s.n_fibers);
    o.pair_ray = uniform_ptr(s.pair_ray);
    o.pair_fiber = uniform_ptr(s.pair_fiber);
    o.pair_depth = uniform_ptr(s.pair_depth);
    o.depth = __builtin_amdgcn_readfirstlane(s.depth);
    o.t_out = uniform_ptr(s.t_out);
    o.u_out = uniform_ptr(s.u_out);
    o.hit_out = uniform_ptr(s.hit_out);
    o.counts = uniform_ptr(s.counts);
    o.t64_out = uniform_ptr(s.t64_out);
    o.u64_out = uniform_ptr(s.u64_out);
    o.normal_out = uniform_ptr(s.normal_out);
    o.n_pairs = uniform_i64(s.n_pairs);
}

// The wave's contiguous range of the call's pairs (an even share).
__device__ __forceinline__ void wave_range(int64_t w, int64_t waves, int64_t count, int64_t &begin, int64_t &end)
{
    const int64_t share = (count + waves - 1) / waves;
    begin = w * share < count ? w * share : count;
    end = (w + 1) * share < count ? (w + 1) * share : count;
}

#ifndef FIBERHIT_WAVES
#define FIBERHIT_WAVES 4                      // build knob: register budget (waves per SIMD)
#endif
template <int MODE, bool BATCHED, bool CAND = false, bool QUAD = false, bool PC = kParentCache>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(MODE == kConservative ? 4 : FIBERHIT_WAVES, 8)))
void k_fused(Args a0, const Args *scenes, const int64_t *offsets, int n_scenes, int64_t count, int refill,
             const float *aos)
{
    __shared__ float s_cache[16 * kWave];
    __shared__ float s_queue[kQWords * kQueue];
    const int lane = (int)threadIdx.x;
    float *col = s_cache + lane;
    const int64_t w = blockIdx.x, waves = gridDim.x;
    int64_t next, end;                                                  // wave-uniform range
    wave_range(w, waves, count, next, end);
    const RegRoot root{};
    // batched: pairs are numbered across the scene table; the wave's share
    // is contiguous, so the scene of its next pair only moves forward
    int scene0 = 0;                      // scene of the wave's next pair (wave-uniform)
    Args cur = a0;                       // batched: scene0's descriptor, read once per change
    int64_t base0 = 0, bound0 = count;   // batched: scene0's first pair, and the next scene's
    if constexpr (BATCHED) {
        scene0 = __builtin_amdgcn_readfirstlane(next < count ? find_scene(offsets, n_scenes, next) : 0);
        uniform_scene(scenes[scene0], cur);
        base0 = uniform_i64(offsets[scene0]);
        bound0 = uniform_i64(offsets[scene0 + 1]);
    }
    int q_head = 0, q_count = 0;         // the queue: entries q_head .. q_head + q_count - 1 (mod kQueue)
    Lane L = {};
    L.lo = INFINITY;                                                   // an empty interval: no work
    L.hi = -INFINITY;
    bool active = false;
    for (;;) {
        const uint64_t free_mask = __ballot(!active);
        const int n_free = __popcll(free_mask);
        if (next < end && q_count < n_free) {
            // setup round: lane k prepares pair next + k
            const int take = end - next < kQueue - q_count ? (int)(end - next) : kQueue - q_count;
            bool queued = false;
            Node r = {};
            float rlo = 0.0f, rhi = 0.0f, rtmax = 0.0f;
            uint32_t depth = 0;
            int64_t idx = next + lane;
            int sc = scene0;
            // each preparing lane stages its root in the queue entry after the
            // current tail plus its lane number; survivors then move to
            // consecutive entries (every lane has read its own entry back
            // before any lane writes)
            float *stage = s_queue + qslot(q_head + q_count + lane);
            if (lane < take) {
                Args a = a0;
                if constexpr (BATCHED) {
                    if (idx < bound0) {
                        idx -= base0;
                        a = cur;
                    } else {
                        while (sc + 1 < n_scenes && offsets[sc + 1] <= idx) ++sc;
                        idx -= offsets[sc];
                        a = scenes[sc];
                    }
                }
                const bool ok = load_pair<CAND, QUAD>(a, idx, stage, rtmax, depth, aos);
                asm volatile("" ::: "memory");
                float *f = &r.p.x;
#pragma unroll
                for (int k = 0; k < 16; ++k) f[k] = stage[k * kQueue];
                if (!ok) {
                    if (!CAND) finish_invalid<MODE>(a, idx);
                } else {
                    cap_interval(r, rtmax, rlo, rhi);
                    float te, tx, lu, hu;
                    const float slack = MODE == kConservative && depth > kRefineAbove ? root_slack(r) : -1.0f;
                    const bool vis = node_visible<MODE, QUAD>(r, rlo, rhi, slack, te, tx, lu, hu);
                    if (vis && depth > 0) {
                        queued = true;
                    } else {
                        // decided at the root: a miss, or the root is the leaf
                        Lane D = {};
                        D.c = r;
                        D.root = r;
                        D.tmax = rtmax;
                        D.t = fmaxf(te, lu);

                        D.start = 0;
                        D.size = kRootSize;
                        D.u = leaf_u(D);
                        D.level = 0;
                        D.trips = 1;
                        D.slack = slack;
                        finish<MODE, CAND>(a, idx, D, vis, hit_geo(r, D.t, te < lu));
                    }
                }
            }
            asm volatile("" ::: "memory");
            const uint64_t qm = __ballot(queued);
            if (queued) {
                const int e = qslot(q_head + q_count + (int)lanes_below(qm));
                float *q = s_queue + e;
                if (q != stage) {
                    const float *f = &r.p.x;
#pragma unroll
                    for (int k = 0; k < 16; ++k) q[k * kQueue] = f[k];
                }
                q[16 * kQueue] = rlo;
                q[17 * kQueue] = rhi;
                q[18 * kQueue] = rtmax;
                q[19 * kQueue] = __int_as_float((int)idx);
                q[20 * kQueue] = __int_as_float((sc << 6) | (stall_possible(r) ? 32 : 0) | (int)depth);
            }
            q_count += __popcll(qm);
            next += take;
            if constexpr (BATCHED) {
                if (next < count && next >= bound0) {
                    while (scene0 + 1 < n_scenes && offsets[scene0 + 1] <= next) ++scene0;
                    scene0 = __builtin_amdgcn_readfirstlane(scene0);
                    uniform_scene(scenes[scene0], cur);
                    base0 = uniform_i64(offsets[scene0]);
                    bound0 = uniform_i64(offsets[scene0 + 1]);
                }
            }
        }
        if (q_count > 0 && n_free >= (refill < q_count ? refill : q_count)) {
            // free lanes take the next queued roots
            const int k = n_free < q_count ? n_free : q_count;
            if (!active) {
                const int rank = (int)lanes_below(free_mask);
                if (rank < k) {
                    const float *q = s_queue + qslot(q_head + rank);
                    float *f = &L.c.p.x;
#pragma unroll
                    for (int j = 0; j < 16; ++j) f[j] = q[j * kQueue];
                    L.lo = q[16 * kQueue];
                    L.hi = q[17 * kQueue];
                    L.tmax = q[18 * kQueue];
                    L.pair = __float_as_int(q[19 * kQueue]);
                    const int ds = __float_as_int(q[20 * kQueue]);
                    const uint32_t depth = (uint32_t)ds & 31u;
                    L.scene = ds >> 6;
                    L.root = L.c;
                    L.min_size = kRootSize >> depth;
                    L.slack = MODE == kConservative && depth > kRefineAbove ? root_slack(L.c) : -1.0f;
                    L.start = (ds & 32) ? kStallBit : 0u;
                    L.size = kRootSize;
                    L.bits = 0;
                    L.cached = 0;
                    L.waiting = 0;
                    L.trips = 0;
                    L.splits = L.backtracks = 0;
                    active = true;
                }
            }
            q_head = qslot(q_head + k);
            q_count -= k;
        }
        // No edge back to the setup that bypasses the trip: a wave whose
        // fresh pairs were all decided at the root runs one idle trip instead.
        // With a single path around the loop the lane state keeps one set of
        // registers; a bypass edge had made the compiler copy the node and
        // the traversal state at every trip (about 45 moves, measured 12-14 %
        // of the call).
        if (__ballot(active) == 0 && next >= end && q_count == 0) break;
        HitGeo hg;
        const int st = trip<MODE, QUAD, PC>(L, root, col, hg);
        if (active && st != kGoOn && !(MODE == kConservative && L.waiting)) {
            if constexpr (BATCHED) {
                // lanes of the wave's current scene read its output
                // pointers with uniform loads; others (a scene boundary
                // inside the wave) load their scene's
                if (L.scene == scene0) finish<MODE>(cur, L.pair, L, st == kHit, hg);
                else finish<MODE>(scenes[L.scene], L.pair, L, st == kHit, hg);
            } else {
                finish<MODE, CAND>(a0, L.pair, L, st == kHit, hg);
            }
            active = false;
        }
        if constexpr (MODE == kConservative) {
            // the FP64 searches run for all parked lanes at once (SIMD lanes
            // of one call) when no busy lane is left: every lane of the wave
            // then shares the search's passes (measured: 2x faster on hair
            // than batches of 16 parked lanes)
            const uint64_t parked = __ballot(L.waiting != 0);
            if (parked != 0 && __ballot(active && !L.waiting) == 0) {
                if (L.waiting) {
                    L.waiting = 0;
                    // plain values, not references (see refine_whole_curve)
                    const float *rays = a0.rays, *fibers = a0.fibers;
                    int64_t rs = a0.ray_stride, fs = a0.fiber_stride;
                    const int32_t *pr = a0.pair_ray, *pf = a0.pair_fiber;
                    bool want_n = a0.normal_out != nullptr;
                    if constexpr (BATCHED) {
                        const Args *sc = scenes + L.scene;
                        rays = sc->rays; fibers = sc->fibers;
                        rs = sc->ray_stride; fs = sc->fiber_stride;
                        pr = sc->pair_ray; pf = sc->pair_fiber;
                        want_n = sc->normal_out != nullptr;
                    }
                    int64_t fi = -1;
                    double tlim = L.tmax;
                    if (CAND) {
                        // candidate lists: the ray's tmax shortened to its
                        // FP64 nearest hit so far
                        fi = a0.cand_fiber[a0.cand_off[L.pair] + a0.cand_round];
                        tlim = fmin((double)rays[6 * rs + L.pair], a0.t64_out[L.pair]);
                    }
                    const int32_t pair = L.pair, scene = L.scene;
                    const Refined r = refine_whole_curve(rays, rs, fibers, fs, pr, pf, pair, fi, tlim, L.t, L.ru,
                                                         want_n, QUAD);
                    // the output pointers are read after the call (not kept
                    // live across it); a refined pair's finish reads only the
                    // search's result from the lane (slack >= 0)
                    Lane R = {};
                    if constexpr (BATCHED) finish<MODE>(scenes[scene], pair, R, r.hit, HitGeo{}, r);
                    else finish<MODE, CAND>(a0, pair, R, r.hit, HitGeo{}, r);
                    active = false;
                }
                // every lane is free now. Its traversal state is reset, so
                // that none of it is live across the searches (kept, it
                // had to be saved and restored around the call)
                L = Lane{};
            }
        }
        if (!active) {
            L.lo = INFINITY;
            L.hi = -INFINITY;
            L.bits = 0;
        }
    }
}

// Fibers transposed to 16 consecutive floats each, for calls that gather them
// through pair indices (one lane per fiber: coalesced row reads, 64-byte
// records written as four 16-byte stores).
__global__ __launch_bounds__(256) void k_fibers_aos(const float *F, int64_t fs, int64_t nf, float4 *out)
{
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= nf) return;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        out[4 * f + k] = make_float4(F[(4 * k) * fs + f], F[(4 * k + 1) * fs + f], F[(4 * k + 2) * fs + f],
                                     F[(4 * k + 3) * fs + f]);
}

// Candidate lists start as misses (each round then writes the hits).
__global__ __launch_bounds__(256) void k_cand_init(int64_t n, float *t, float *u, uint8_t *hit, int32_t *fiber,
                                                   double *t64, double *u64, float *nrm)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    t[i] = INFINITY;
    u[i] = __builtin_nanf("");
    hit[i] = 0;
    fiber[i] = -1;
    if (t64) {
        t64[i] = INFINITY;
        u64[i] = __builtin_nan("");
    }
    if (nrm) {
        nrm[i] = __builtin_nanf("");
        nrm[n + i] = __builtin_nanf("");
        nrm[2 * n + i] = __builtin_nanf("");
    }
}

int check_common(const float *rays, int64_t ray_stride, int64_t n_rays,
                 const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                 const int32_t *pair_ray, const int32_t *pair_fiber,
                 int32_t depth, int64_t n_pairs, uint32_t flags,
                 const void *t_out, const void *u_out, const void *hit_out)
{
    if (n_pairs < 0 || n_rays < 0 || n_fibers < 0) return FI_ERR_RANGE;
    if (depth < 0 || depth > FI_MAX_DEPTH) return FI_ERR_RANGE;
    if ((flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ | FI_QUADRATIC)) != 0u) return FI_ERR_RANGE;
    if (n_pairs == 0) return FI_OK;
    if (!rays || !fibers || !t_out || !u_out || !hit_out) return FI_ERR_NULL;
    if (ray_stride < n_rays || fiber_stride < n_fibers) return FI_ERR_RANGE;
    if (!pair_ray && n_pairs > n_rays) return FI_ERR_RANGE;
    if (!pair_fiber && n_pairs > n_fibers) return FI_ERR_RANGE;
    if (n_pairs > (int64_t)0x7fffffff - 64) return FI_ERR_RANGE;   // int32 pair indices in the lanes
    return FI_OK;
}

// ---------------------------------------------------------------------------
// Kernel variants and per-device state
// ---------------------------------------------------------------------------

using FusedFn = void (*)(Args, const Args *, const int64_t *, int, int64_t, int, const float *);
// [0] plain, [1] counting, [2] conservative (single calls), [3] plain and
// [4] conservative over a scene table, [5] plain and [6] conservative over
// candidate lists, [7..9] plain, counting and conservative on quadratic
// fibers, [10] plain and [11] conservative over a scene table without the
// parent cache (a tuning choice: every backtrack replays from the root)
constexpr int kVariants = 12;
const FusedFn kFused[kVariants] = {k_fused<kPlain, false>, k_fused<kCount, false>, k_fused<kConservative, false>,
                                   k_fused<kPlain, true>, k_fused<kConservative, true>,
                                   k_fused<kPlain, false, true>, k_fused<kConservative, false, true>,
                                   k_fused<kPlain, false, false, true>, k_fused<kCount, false, false, true>,
                                   k_fused<kConservative, false, false, true>,
                                   k_fused<kPlain, true, false, false, false>,
                                   k_fused<kConservative, true, false, false, false>};
constexpr int kBatchedVariant = 3;
constexpr int kBatchedRefineVariant = 4;
constexpr int kCandVariant = 5;              // + 1: refined
constexpr int kQuadVariant = 7;              // + kPlain, kCount, kConservative: quadratic fibers
constexpr int kBatchedReplayVariant = 10;    // + 1: refined

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kMaxRecordBytes = (size_t)1 << 30;                 // fiber records, largest table

constexpr int kMaxDevices = 64;
constexpr int kStageSlots = 4;                 // pinned staging for batched scene tables
constexpr size_t kStageBytes = 1u << 20;

// Fiber records of fiber_intersect_pairs_noalloc, for callers that cannot
// allocate: a fixed array in the code object, one copy per device, of
// kScratchBytes (32 MiB: the records of 524,288 fibers). Host code never
// passes the array's name to a kernel: each device's copy is reached through
// the address hipGetSymbolAddress gives for it (DeviceInfo::scratch).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

struct DeviceInfo {
    std::atomic<bool> ready;
    int cus;
    char arch[64];                             // architecture name (gfx950...), without feature flags
    int fused_resident[kVariants];             // resident waves per CU, per variant (as kFused)
    float *scratch;                            // this device's copy of `scratch`
    std::mutex stage_mutex;
    void *stage[kStageSlots];                  // pinned host buffers for scene tables
    hipEvent_t stage_done[kStageSlots];
    int stage_next;
};
DeviceInfo g_dev[kMaxDevices];
std::mutex g_dev_mutex;

int current_device(int &dev)
{
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FI_ERR_HIP;
    return FI_OK;
}

// Set-up of the current device, once: unit counts, occupancy of every kernel
// variant, the address of this device's scratch array and the pinned staging
// buffers of batched calls. Every entry point runs it on its first call on a
// device (fi_init_device runs it ahead).
int device_info(DeviceInfo *&out)
{
    int dev = 0;
    if (current_device(dev) != FI_OK) return FI_ERR_HIP;
    DeviceInfo &d = g_dev[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(g_dev_mutex);
        if (!d.ready.load(std::memory_order_relaxed)) {
            if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                return FI_ERR_HIP;
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FI_ERR_HIP;
            size_t n = 0;
            while (n + 1 < sizeof d.arch && prop.gcnArchName[n] && prop.gcnArchName[n] != ':') {
                d.arch[n] = prop.gcnArchName[n];
                ++n;
            }
            d.arch[n] = '\0';
            for (int m = 0; m < kVariants; ++m) {
                int nb = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)kFused[m], kWave, 0) != hipSuccess)
                    return FI_ERR_HIP;
                d.fused_resident[m] = nb > 0 ? nb : 1;
            }
            // the device address of this device's copy of the static
            // scratch array (taken with the device current)
            d.scratch = nullptr;
            if (hipGetSymbolAddress((void **)&d.scratch, HIP_SYMBOL(scratch)) != hipSuccess || !d.scratch)
                return FI_ERR_HIP;
            for (int k = 0; k < kStageSlots; ++k) {
                if (hipHostMalloc(&d.stage[k], kStageBytes, hipHostMallocDefault) != hipSuccess) return FI_ERR_HIP;
                if (hipEventCreateWithFlags(&d.stage_done[k], hipEventDisableTiming) != hipSuccess) return FI_ERR_HIP;
            }
            d.stage_next = 0;
            d.ready.store(true, std::memory_order_release);
        }
    }
    out = &d;
    return FI_OK;
}

// Fiber records of a single call: when it gathers fibers through pair_fiber
// and reads each fiber about once or more, the fibers are first copied to
// 16-float records (one pass over the table): a gathered fiber is then one
// or two cache lines instead of one line per coordinate row.
size_t record_bytes(int64_t n_pairs, int64_t n_fibers, bool gathered)
{
    const size_t need = (size_t)(n_fibers > 0 ? n_fibers : 0) * 16 * sizeof(float);
    return gathered && n_fibers > 0 && n_pairs >= n_fibers && need <= kMaxRecordBytes ? align256(need) : 0;
}

// Launch defaults of single-problem calls (and of batches without a tuned
// entry); measured choices, overridable when building.
#ifndef FIBERHIT_DEFAULT_REFILL
#define FIBERHIT_DEFAULT_REFILL 1
#endif
#ifndef FIBERHIT_DEFAULT_WAVES_PER_SIMD
#define FIBERHIT_DEFAULT_WAVES_PER_SIMD 0
#endif
fi_tuning default_tuning(bool refine)
{
    return fi_tuning{refine ? FIBERHIT_REFINE_REFILL : FIBERHIT_DEFAULT_REFILL, FIBERHIT_DEFAULT_WAVES_PER_SIMD, 0};
}

// Autotune results: keyed by the GPU architecture, the refinement flag and
// the batch's class -- log2 of its total pairs, log2 of its problem count and
// a depth bucket of its largest depth (<= 9, <= 16, deeper). A batch launched
// without an explicit tuning uses the entry of its class if one exists. The
// table lives for the process; fiber_tuning_save / fiber_tuning_load keep it
// in a text file across processes.
using TuneKey = std::tuple<std::string, int, int, int, int>;
std::mutex g_tune_mutex;
std::map<TuneKey, fi_tuning> g_tune_cache;

int log2_floor(int64_t x)
{
    int l = 0;
    while (l < 62 && ((int64_t)1 << (l + 1)) <= x) ++l;
    return l;
}

int depth_bucket(int max_depth) { return max_depth <= 9 ? 0 : max_depth <= 16 ? 1 : 2; }

TuneKey tune_key(const std::string &arch, int64_t total, int n_scenes, int max_depth, bool refine)
{
    return TuneKey{arch, refine ? 1 : 0, log2_floor(total), log2_floor(n_scenes), depth_bucket(max_depth)};
}

int check_tuning(const fi_tuning &t)
{
    if (t.refill < 1 || t.refill > kWave || t.waves_per_simd < 0 || t.waves_per_simd > 16 || t.stack < 0 ||
        t.stack > 1)
        return FI_ERR_RANGE;
    return FI_OK;
}

int max_scene_depth(const fi_scene *sc, int32_t n)
{
    int d = 0;
    for (int k = 0; k < n; ++k) d = sc[k].depth > d ? sc[k].depth : d;
    return d;
}

int64_t total_pairs(const fi_scene *sc, int32_t n)
{
    int64_t t = 0;
    for (int k = 0; k < n; ++k) t += sc[k].n_pairs > 0 ? sc[k].n_pairs : 0;
    return t;
}

// The remembered tuning of this batch's class on the current device, else
// the defaults.
fi_tuning tuned_or_default(const fi_scene *sc, int32_t n, bool refine)
{
    DeviceInfo *d = nullptr;
    if (device_info(d) != FI_OK) return default_tuning(refine);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it = g_tune_cache.find(tune_key(d->arch, total_pairs(sc, n), n, max_scene_depth(sc, n), refine));
    return it == g_tune_cache.end() ? default_tuning(refine) : it->second;
}

void remember_tuning(const fi_scene *sc, int32_t n, bool refine, const fi_tuning &t)
{
    DeviceInfo *d = nullptr;
    if (device_info(d) != FI_OK) return;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[tune_key(d->arch, total_pairs(sc, n), n, max_scene_depth(sc, n), refine)] = t;
}


// Persistent waves of a single call: twice the resident waves, each with
// half the share. The second half starts as waves of the first finish, so
// waves whose pairs happened to need few trips take more of the work and
// the call's tail shrinks. Measured against the resident waves alone (A/B
// on one box, 2^20 pairs): depth 22 198 against 232 us, depth 9 123
// against 115 us, the two calls overlapped on two streams 228.5 against
// 230 us; hair (2^24 pairs) 1.23 / 1.90 against 1.26 / 1.96 ms; refined
// hair 3.93 against 4.13 ms per 2^22 pairs. Four times the resident waves
// was slower (overlapped 283 us), and so were twice the waves for deep
// calls only (overlapped 250 us: the shallow call's waves then wait behind
// the deep call's), a grid skewed towards the waves that start first on
// each SIMD, and issue priority by progress through the share. The rounds
// of candidate lists keep the resident waves: most of their pairs end at
// the root, and twice the waves made them 15 % (refined 39 %) slower.
int64_t single_call_waves(const DeviceInfo &d, int mode, const Args &)
{
    const bool cand = mode == kCandVariant || mode == kCandVariant + 1;
    return (cand ? 1 : 2) * (int64_t)d.fused_resident[mode] * d.cus;
}

// Enqueue one single call on `s`: the fiber records (when `aos` is given and
// `convert`), then one persistent launch of about one wave per 64 pairs, at
// most `max_waves`.
int launch(int mode, const Args &a, int64_t max_waves, float *aos, hipStream_t s, bool convert = true)
{
    if (aos && convert)
        hipLaunchKernelGGL(k_fibers_aos, dim3((unsigned)((a.n_fibers + 255) / 256)), dim3(256), 0, s,
                           a.fibers, a.fiber_stride, a.n_fibers, (float4 *)aos);
    int64_t g = (a.n_pairs + kWave - 1) / kWave;
    if (g > max_waves) g = max_waves;
    if (g > 0)
        hipLaunchKernelGGL(kFused[mode], dim3((unsigned)g), dim3(kWave), 0, s, a, nullptr, nullptr, 0,
                           a.n_pairs,
                           mode == kConservative || mode == kCandVariant + 1 ||
                                   mode == kQuadVariant + kConservative
                               ? FIBERHIT_REFINE_REFILL
                               : FIBERHIT_FUSED_REFILL,
                           aos);
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

// A single call with the fiber records (if it gathers fibers) in the
// caller's workspace, room permitting.
int launch_with_workspace(int mode, const Args &a, void *workspace, size_t workspace_bytes, void *stream,
                          bool quad = false)
{
    if (workspace && ((uintptr_t)workspace & 255u) != 0u) return FI_ERR_WORKSPACE;
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    const int st = device_info(d);
    if (st != FI_OK) return st;
    // quadratic tables are read in place (the records hold cubic rows)
    const size_t rec = quad ? 0 : record_bytes(a.n_pairs, a.n_fibers, a.pair_fiber != nullptr);
    float *aos = rec && workspace && workspace_bytes >= rec ? (float *)workspace : nullptr;
    return launch(mode, a, single_call_waves(*d, mode, a), aos, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Batched problems
// ---------------------------------------------------------------------------

size_t scene_table_bytes(int n) { return align256((size_t)n * sizeof(Args)) + align256((size_t)(n + 1) * sizeof(int64_t)); }

int scenes_to_table(const fi_scene *sc, int32_t n, uint32_t flags, Args *tab, int64_t *off)
{
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    off[0] = 0;
    for (int k = 0; k < n; ++k) {
        const fi_scene &x = sc[k];
        const int st = check_common(x.rays, x.ray_stride, x.n_rays, x.fibers, x.fiber_stride, x.n_fibers,
                                    x.pair_ray, x.pair_fiber, x.depth, x.n_pairs, flags, x.t_out, x.u_out, x.hit_out);
        if (st != FI_OK) return st;
        if (refine && x.n_pairs > 0 && (!x.t64_out || !x.u64_out)) return FI_ERR_NULL;
        tab[k] = Args{x.rays, x.ray_stride, x.n_rays, x.fibers, x.fiber_stride, x.n_fibers,
                      x.pair_ray, x.pair_fiber, x.pair_depth, x.depth, x.n_pairs,
                      x.t_out, x.u_out, x.hit_out, nullptr,
                      refine ? x.t64_out : nullptr, refine ? x.u64_out : nullptr, x.normal_out};
        off[k + 1] = off[k] + x.n_pairs;
    }
    if (off[n] > (int64_t)0x7fffffff - 64) return FI_ERR_RANGE;
    return FI_OK;
}

// Layout of a batched workspace: scene table, pair offsets.
struct BatchLayout {
    Args *scenes;
    int64_t *offsets;
};

BatchLayout layout_of(void *ws, int n)
{
    char *p = (char *)ws;
    BatchLayout L;
    L.scenes = (Args *)p;
    L.offsets = (int64_t *)(p + align256((size_t)n * sizeof(Args)));
    return L;
}

// One persistent launch over all scenes of a batch: about one wave per 64
// pairs, at most the resident waves, or the tuning's waves per SIMD (fewer
// or more than fit).
void launch_batched(const DeviceInfo &d, const fi_tuning &t, const BatchLayout &L, int n_scenes, int64_t total,
                    bool refine, hipStream_t s)
{
    const int variant = t.stack == 1 ? kBatchedReplayVariant + (refine ? 1 : 0)
                                     : (refine ? kBatchedRefineVariant : kBatchedVariant);
    int per_cu = d.fused_resident[variant];
    // below the resident waves per SIMD: fewer waves; above: the grid holds
    // more waves than fit, and the dispatcher starts them as others end
    if (t.waves_per_simd > 0) per_cu = 4 * t.waves_per_simd;
    int64_t g = (total + kWave - 1) / kWave;
    if (g > (int64_t)per_cu * d.cus) g = (int64_t)per_cu * d.cus;
    if (g > 0)
        hipLaunchKernelGGL(kFused[variant], dim3((unsigned)g), dim3(kWave), 0, s, Args{}, L.scenes, L.offsets,
                           n_scenes, total, t.refill, nullptr);
}

int batched_enqueue(const fi_scene *scenes, int32_t n_scenes, uint32_t flags, const fi_tuning &t, void *workspace,
                    size_t workspace_bytes, hipStream_t s)
{
    DeviceInfo *d = nullptr;
    int st = device_info(d);
    if (st != FI_OK) return st;
    const size_t tb = scene_table_bytes(n_scenes);
    if (tb > kStageBytes) return FI_ERR_RANGE;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0u || workspace_bytes < tb) return FI_ERR_WORKSPACE;
    std::lock_guard<std::mutex> lock(d->stage_mutex);
    const int k = d->stage_next;
    // the staging buffer's previous upload must have left it (rarely waits:
    // four buffers in turn)
    if (hipEventSynchronize(d->stage_done[k]) != hipSuccess) return FI_ERR_HIP;
    char *host = (char *)d->stage[k];
    int64_t *off = (int64_t *)(host + align256((size_t)n_scenes * sizeof(Args)));
    st = scenes_to_table(scenes, n_scenes, flags, (Args *)host, off);
    if (st != FI_OK) return st;
    const int64_t total = off[n_scenes];
    const BatchLayout L = layout_of(workspace, n_scenes);
    if (hipMemcpyAsync(workspace, host, tb, hipMemcpyHostToDevice, s) != hipSuccess) return FI_ERR_HIP;
    if (hipEventRecord(d->stage_done[k], s) != hipSuccess) return FI_ERR_HIP;
    d->stage_next = (k + 1) % kStageSlots;
    launch_batched(*d, t, L, n_scenes, total, (flags & FI_FP64_REFINE) != 0u, s);
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

}  // namespace

struct fi_batch_plan {
    int device;
    void *mem;                 // device copy of the scene table and offsets
    int n_scenes;
    int64_t total;
    uint32_t flags;
    fi_tuning tuning;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {
int fi_version(void) { return (0 << 16) | (9 << 8) | 0; }

const char *fi_strerror(int status)
{
    switch (status) {
    case FI_OK: return "ok";
    case FI_ERR_NULL: return "a required pointer is NULL";
    case FI_ERR_RANGE: return "a count, stride, depth or flag is out of range";
    case FI_ERR_HIP: return "the HIP runtime reported an error";
    case FI_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case FI_ERR_SCRATCH: return "the call needs more scratch than the no-allocation entry point holds";
    case FI_ERR_IO: return "a tuning table file could not be opened or written";
    default: return "unknown status";
    }
}

int fi_init_device(void)
{
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    return device_info(d);
}

size_t fiber_pairs_workspace_bytes(int64_t n_pairs, int64_t n_fibers, int32_t gathered, uint32_t flags)
{
    if (n_pairs < 0 || n_fibers < 0 || (flags & FI_QUADRATIC) != 0u) return 0;
    return record_bytes(n_pairs, n_fibers, gathered != 0);
}

int fiber_intersect_pairs(const float *rays, int64_t ray_stride, int64_t n_rays,
                          const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                          const int32_t *pair_ray, const int32_t *pair_fiber,
                          const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                          uint32_t flags,
                          float *t_out, float *u_out, uint8_t *hit_out,
                          double *t64_out, double *u64_out, float *normal_out,
                          void *workspace, size_t workspace_bytes, void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    if (refine && (!t64_out || !u64_out)) return FI_ERR_NULL;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, nullptr,
           refine ? t64_out : nullptr, refine ? u64_out : nullptr, normal_out};
    const bool quad = (flags & FI_QUADRATIC) != 0u;
    return launch_with_workspace((refine ? kConservative : kPlain) + (quad ? kQuadVariant : 0), a, workspace,
                                 workspace_bytes, stream, quad);
}

int fiber_intersect_pairs_noalloc(const float *rays, int64_t ray_stride, int64_t n_rays,
                                  const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                                  const int32_t *pair_ray, const int32_t *pair_fiber,
                                  const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                                  uint32_t flags,
                                  float *t_out, float *u_out, uint8_t *hit_out,
                                  double *t64_out, double *u64_out, float *normal_out,
                                  void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    if (refine && (!t64_out || !u64_out)) return FI_ERR_NULL;
    const bool quad = (flags & FI_QUADRATIC) != 0u;
    const size_t rec = quad ? 0 : record_bytes(n_pairs, n_fibers, pair_fiber != nullptr);
    if (rec > kScratchBytes) return FI_ERR_SCRATCH;
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    const int ds = device_info(d);
    if (ds != FI_OK) return ds;
    const int mode = (refine ? kConservative : kPlain) + (quad ? kQuadVariant : 0);
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, nullptr,
           refine ? t64_out : nullptr, refine ? u64_out : nullptr, normal_out};
    // the fiber records of a gathered call go to this device's copy of the
    // scratch array (through its device address, never the array's name)
    return launch(mode, a, single_call_waves(*d, mode, a), rec ? d->scratch : nullptr, (hipStream_t)stream);
}

int fiber_intersect_counts(const float *rays, int64_t ray_stride, int64_t n_rays,
                           const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                           const int32_t *pair_ray, const int32_t *pair_fiber,
                           const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                           uint32_t flags,
                           float *t_out, float *u_out, uint8_t *hit_out,
                           int32_t *counts_out, void *workspace, size_t workspace_bytes, void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    if (!counts_out) return FI_ERR_NULL;
    if ((flags & FI_FP64_REFINE) != 0u) return FI_ERR_RANGE;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, counts_out, nullptr, nullptr,
           nullptr};
    const bool quad = (flags & FI_QUADRATIC) != 0u;
    return launch_with_workspace(kCount + (quad ? kQuadVariant : 0), a, workspace, workspace_bytes, stream, quad);
}

size_t fiber_candidates_workspace_bytes(int64_t n_candidates, int64_t n_fibers, uint32_t flags)
{
    (void)flags;
    if (n_candidates < 0 || n_fibers < 0) return 0;
    return record_bytes(n_candidates, n_fibers, true);
}

int fiber_intersect_candidates(const float *rays, int64_t ray_stride, int64_t n_rays,
                               const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                               const int64_t *cand_offsets, const int32_t *cand_fiber,
                               const uint8_t *cand_depth, int32_t depth, int32_t max_candidates,
                               int64_t n_candidates, uint32_t flags,
                               float *t_out, float *u_out, uint8_t *hit_out, int32_t *fiber_out,
                               double *t64_out, double *u64_out, float *normal_out,
                               void *workspace, size_t workspace_bytes, void *stream)
{
    if (n_rays < 0 || n_fibers < 0 || n_candidates < 0 || max_candidates < 0) return FI_ERR_RANGE;
    if (depth < 0 || depth > FI_MAX_DEPTH) return FI_ERR_RANGE;
    if ((flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ)) != 0u) return FI_ERR_RANGE;
    if (n_rays == 0) return FI_OK;
    if (!rays || !fibers || !cand_offsets || !t_out || !u_out || !hit_out || !fiber_out) return FI_ERR_NULL;
    if (n_candidates > 0 && !cand_fiber) return FI_ERR_NULL;
    if (ray_stride < n_rays || fiber_stride < n_fibers) return FI_ERR_RANGE;
    if (n_rays > (int64_t)0x7fffffff - 64) return FI_ERR_RANGE;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    if (refine && (!t64_out || !u64_out)) return FI_ERR_NULL;
    if (workspace && ((uintptr_t)workspace & 255u) != 0u) return FI_ERR_WORKSPACE;
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    const int ds = device_info(d);
    if (ds != FI_OK) return ds;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_cand_init, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, s, n_rays, t_out, u_out,
                       hit_out, fiber_out, refine ? t64_out : nullptr, refine ? u64_out : nullptr, normal_out);
    if (hipGetLastError() != hipSuccess) return FI_ERR_HIP;
    const int mode = refine ? kCandVariant + 1 : kCandVariant;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           nullptr, nullptr, cand_depth, depth, n_rays, t_out, u_out, hit_out, nullptr,
           refine ? t64_out : nullptr, refine ? u64_out : nullptr, normal_out,
           cand_offsets, cand_fiber, 0, n_candidates, fiber_out};
    const size_t rec = record_bytes(n_candidates, n_fibers, true);
    float *aos = rec && workspace && workspace_bytes >= rec ? (float *)workspace : nullptr;
    // one launch per list position, in order: round k tests every ray's k-th
    // candidate against the ray shortened to its nearest hit of rounds < k
    for (int32_t k = 0; k < max_candidates; ++k) {
        a.cand_round = k;
        const int st = launch(mode, a, single_call_waves(*d, mode, a), aos, s, k == 0);
        if (st != FI_OK) return st;
    }
    return FI_OK;
}

size_t fiber_batched_workspace_bytes(int32_t n_scenes, int64_t total_pairs)
{
    if (n_scenes < 0 || total_pairs < 0) return 0;
    return scene_table_bytes(n_scenes);
}

int fiber_intersect_batched(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, void *workspace, size_t workspace_bytes, void *stream)
{
    if (n_scenes < 0 || (flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ)) != 0u) return FI_ERR_RANGE;
    if (n_scenes == 0) return FI_OK;
    if (!scenes) return FI_ERR_NULL;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    const fi_tuning t = tuning ? *tuning : tuned_or_default(scenes, n_scenes, refine);
    if (check_tuning(t) != FI_OK) return FI_ERR_RANGE;
    (void)hipGetLastError();
    return batched_enqueue(scenes, n_scenes, flags, t, workspace, workspace_bytes, (hipStream_t)stream);
}

int fiber_batch_plan_create(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, fi_batch_plan **plan_out)
{
    if (!plan_out) return FI_ERR_NULL;
    *plan_out = nullptr;
    if (n_scenes <= 0 || (flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ)) != 0u) return FI_ERR_RANGE;
    if (!scenes) return FI_ERR_NULL;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    const fi_tuning t = tuning ? *tuning : tuned_or_default(scenes, n_scenes, refine);
    if (check_tuning(t) != FI_OK) return FI_ERR_RANGE;
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    int st = device_info(d);
    if (st != FI_OK) return st;
    const size_t tb = scene_table_bytes(n_scenes);
    char *host = (char *)malloc(tb);
    if (!host) return FI_ERR_RANGE;
    int64_t *off = (int64_t *)(host + align256((size_t)n_scenes * sizeof(Args)));
    st = scenes_to_table(scenes, n_scenes, flags, (Args *)host, off);
    if (st != FI_OK) { free(host); return st; }
    fi_batch_plan *p = new fi_batch_plan();
    p->n_scenes = n_scenes;
    p->total = off[n_scenes];
    p->flags = flags;
    p->tuning = t;
    current_device(p->device);
    hipStream_t cs = nullptr;
    const size_t bytes = tb;
    bool ok = hipMalloc(&p->mem, bytes) == hipSuccess &&
              hipMemcpy(p->mem, host, tb, hipMemcpyHostToDevice) == hipSuccess &&
              hipStreamCreate(&cs) == hipSuccess;
    free(host);
    if (ok) {
        const BatchLayout L = layout_of(p->mem, n_scenes);
        ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            launch_batched(*d, t, L, n_scenes, p->total, refine, cs);
            ok = hipStreamEndCapture(cs, &p->graph) == hipSuccess &&
                 hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
        }
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (!ok) {
        (void)hipGetLastError();
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->mem) (void)hipFree(p->mem);
        delete p;
        return FI_ERR_HIP;
    }
    *plan_out = p;
    return FI_OK;
}

int fiber_batch_plan_launch(fi_batch_plan *plan, void *stream)
{
    if (!plan) return FI_ERR_NULL;
    (void)hipGetLastError();
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_ERR_HIP;
}

int fiber_batch_plan_destroy(fi_batch_plan *plan)
{
    if (!plan) return FI_OK;
    int st = FI_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) st = FI_ERR_HIP;
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) st = FI_ERR_HIP;
    if (plan->mem && hipFree(plan->mem) != hipSuccess) st = FI_ERR_HIP;
    delete plan;
    return st;
}

int fiber_batch_plan_tuning(const fi_batch_plan *plan, fi_tuning *tuning_out)
{
    if (!plan || !tuning_out) return FI_ERR_NULL;
    *tuning_out = plan->tuning;
    return FI_OK;
}

int fiber_batch_autotune(const fi_scene *scenes, int32_t n_scenes, uint32_t flags, void *workspace,
                         size_t workspace_bytes, void *stream, int32_t repeats,
                         fi_tuning *best, float *best_ms)
{
    if (!best) return FI_ERR_NULL;
    if (n_scenes <= 0 || (flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ)) != 0u || repeats < 1)
        return FI_ERR_RANGE;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FI_ERR_HIP;
    // refining waves park lanes until the wave decides them together, so
    // they refill early; plain waves refill late
    const int plain_refills[] = {32, 48, 56};
    const int refine_refills[] = {4, 8, 16};
    const int *refills = refine ? refine_refills : plain_refills;
    const int occ[] = {0, 8, 16};         // as many as fit (4), twice, four times
    float best_t = INFINITY;
    fi_tuning bt = default_tuning(refine);
    int st = FI_OK;
    for (int sk = 0; sk < 2 && st == FI_OK; ++sk)
    for (int oi = 0; oi < 3 && st == FI_OK; ++oi)
        for (int ri = 0; ri < 3 && st == FI_OK; ++ri) {
            const fi_tuning t{refills[ri], occ[oi], sk};
            float tmin = INFINITY;
            for (int r = 0; r <= repeats && st == FI_OK; ++r) {       // first run warms up
                if (hipEventRecord(e0, s) != hipSuccess) { st = FI_ERR_HIP; break; }
                st = fiber_intersect_batched(scenes, n_scenes, &t, flags, workspace, workspace_bytes, stream);
                if (st == FI_OK && hipEventRecord(e1, s) != hipSuccess) st = FI_ERR_HIP;
                if (st == FI_OK && hipEventSynchronize(e1) != hipSuccess) st = FI_ERR_HIP;
                float ms = 0.0f;
                if (st == FI_OK && r > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < tmin)
                    tmin = ms;
            }
            if (tmin < best_t) { best_t = tmin; bt = t; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FI_OK) return st;
    *best = bt;
    if (best_ms) *best_ms = best_t;
    remember_tuning(scenes, n_scenes, refine, bt);
    return FI_OK;
}

// Tuning table files: a header line, then one entry per line --
// arch refine log2_pairs log2_scenes depth_bucket refill waves_per_simd stack
int fiber_tuning_save(const char *path)
{
    if (!path) return FI_ERR_NULL;
    std::vector<std::pair<TuneKey, fi_tuning>> rows;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        rows.assign(g_tune_cache.begin(), g_tune_cache.end());
    }
    FILE *f = fopen(path, "w");
    if (!f) return FI_ERR_IO;
    bool ok = fprintf(f, "fiberhit-tuning 1\n") > 0;
    for (const auto &r : rows)
        ok = ok && fprintf(f, "%s %d %d %d %d %d %d %d\n", std::get<0>(r.first).c_str(), std::get<1>(r.first),
                           std::get<2>(r.first), std::get<3>(r.first), std::get<4>(r.first), r.second.refill,
                           r.second.waves_per_simd, r.second.stack) > 0;
    ok = (fclose(f) == 0) && ok;
    return ok ? FI_OK : FI_ERR_IO;
}

int fiber_tuning_load(const char *path)
{
    if (!path) return FI_ERR_NULL;
    FILE *f = fopen(path, "r");
    if (!f) return FI_ERR_IO;
    std::vector<std::pair<TuneKey, fi_tuning>> rows;
    char line[256];
    bool ok = fgets(line, sizeof line, f) && strcmp(line, "fiberhit-tuning 1\n") == 0;
    while (ok && fgets(line, sizeof line, f)) {
        char arch[64];
        int rf, lt, ls, db;
        fi_tuning t;
        char tail;
        if (sscanf(line, "%63s %d %d %d %d %d %d %d %c", arch, &rf, &lt, &ls, &db, &t.refill, &t.waves_per_simd,
                   &t.stack, &tail) != 8 ||
            rf < 0 || rf > 1 || lt < 0 || lt > 62 || ls < 0 || ls > 31 || db < 0 || db > 2 ||
            check_tuning(t) != FI_OK) {
            ok = false;
            break;
        }
        rows.push_back({TuneKey{arch, rf, lt, ls, db}, t});
    }
    fclose(f);
    if (!ok) return FI_ERR_RANGE;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const auto &r : rows) g_tune_cache[r.first] = r.second;
    return FI_OK;
}

int fiber_tuning_lookup(const char *arch, uint32_t flags, int64_t total_pairs, int32_t n_scenes, int32_t max_depth,
                        fi_tuning *out)
{
    if (!arch || !out) return FI_ERR_NULL;
    if (total_pairs < 0 || n_scenes < 1 || max_depth < 0 || max_depth > FI_MAX_DEPTH ||
        (flags & ~(uint32_t)(FI_FP64_REFINE | FI_COMPENSATED_PROJ)) != 0u)
        return FI_ERR_RANGE;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it =
        g_tune_cache.find(tune_key(arch, total_pairs, n_scenes, max_depth, (flags & FI_FP64_REFINE) != 0u));
    if (it == g_tune_cache.end()) return FI_ERR_RANGE;
    *out = it->second;
    return FI_OK;
}

int fiber_tuning_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache.clear();
    return FI_OK;
}

}  // extern "C"
