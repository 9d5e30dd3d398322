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
// tangents fall back to the next non-zero control-polygon edge).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "fiberhit.h"

namespace {

constexpr int kWave = 64;                     // gfx950 wavefront
constexpr uint32_t kRootSize = 1u << 23;      // parametric domain [0, 1) in units of 2^-23
constexpr int kMaxTrips = 1 << 16;            // hang guard; real pairs need < 200 trips
constexpr float kParallelG = 1e-30f;          // axis treated as parallel to the ray below this
#ifndef FIBERHIT_PARENT_CACHE
#define FIBERHIT_PARENT_CACHE 1
#endif
constexpr bool kParentCache = FIBERHIT_PARENT_CACHE != 0;   // cache the latest both-hit parent in LDS

struct V4 { float x, y, z, w; };
struct Node { V4 p, d, t0, t1; };             // Section 3.1: p = p0, d = p3-p0, t0 = p1-p0, t1 = p3-p2

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float vsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

__device__ __forceinline__ bool zero3(float x, float y, float z)
{
    return x == 0.0f && y == 0.0f && z == 0.0f;
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

// Root node of one pair in the ray frame, in the {p, d, t0, t1} form.
// The projection runs once per pair in FP64 (full rate on this chip): the
// differences of the float32 control points and of the origin are exact in
// double, so p is the rounded frame position of p0 and d, t0, t1 are the
// rounded frame images of p3-p0, p1-p0, p3-p2 -- each component accurate to
// its own float32 ulp, including the tiny across-ray or along-ray parts of
// nearly parallel or nearly perpendicular tangents. Returns false for a zero
// or non-finite direction.
__device__ __forceinline__ bool root_in_ray_frame(const float *R, int64_t rs, const float *F,
                                                  int64_t fs, Node &root)
{
    const double ox = R[0], oy = R[rs], oz = R[2 * rs];
    const double dx = R[3 * rs], dy = R[4 * rs], dz = R[5 * rs];
    const double n2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(n2 > 0.0) || !(n2 < INFINITY)) return false;
    const double il = rsqrt64(n2);
    const double w[3] = {dx * il, dy * il, dz * il};
    double u[3], v[3];
    make_onb(w[0], w[1], w[2], u, v);

    double P[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) P[k][c] = F[(4 * k + c) * fs];

    auto proj = [&](double ex, double ey, double ez, double ew) {
        V4 q;
        q.x = (float)fma(ex, u[0], fma(ey, u[1], ez * u[2]));
        q.y = (float)fma(ex, v[0], fma(ey, v[1], ez * v[2]));
        q.z = (float)fma(ex, w[0], fma(ey, w[1], ez * w[2]));
        q.w = (float)ew;
        return q;
    };
    root.p = proj(P[0][0] - ox, P[0][1] - oy, P[0][2] - oz, P[0][3]);
    root.d = proj(P[3][0] - P[0][0], P[3][1] - P[0][1], P[3][2] - P[0][2], P[3][3] - P[0][3]);
    root.t0 = proj(P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2], P[1][3] - P[0][3]);
    root.t1 = proj(P[3][0] - P[2][0], P[3][1] - P[2][1], P[3][2] - P[2][2], P[3][3] - P[2][3]);
    return isfinite(root.p.x) && isfinite(root.p.y) && isfinite(root.p.z) &&
           isfinite(root.d.x) && isfinite(root.d.y) && isfinite(root.d.z);
}

// ---------------------------------------------------------------------------
// Node geometry
// ---------------------------------------------------------------------------

// t interval between the node's two end-cap planes (Section 3.3, cropping),
// intersected with [0, tmax]. Start cap: plane through p, normal t0, curve on
// the positive side. End cap: plane through p + d, normal t1, curve on the
// negative side. A zero tangent falls back to the next control-polygon edge.
__device__ __forceinline__ void cap_interval(const Node &c, float tmax, float &lo, float &hi)
{
    float n0x = c.t0.x, n0y = c.t0.y, n0z = c.t0.z;
    if (zero3(n0x, n0y, n0z)) { n0x = c.d.x - c.t1.x; n0y = c.d.y - c.t1.y; n0z = c.d.z - c.t1.z; }
    if (zero3(n0x, n0y, n0z)) { n0x = c.d.x; n0y = c.d.y; n0z = c.d.z; }
    float n1x = c.t1.x, n1y = c.t1.y, n1z = c.t1.z;
    if (zero3(n1x, n1y, n1z)) { n1x = c.d.x - c.t0.x; n1y = c.d.y - c.t0.y; n1z = c.d.z - c.t0.z; }
    if (zero3(n1x, n1y, n1z)) { n1x = c.d.x; n1y = c.d.y; n1z = c.d.z; }

    float l = 0.0f, h = tmax;
    const float c0 = dot3(c.p.x, c.p.y, c.p.z, n0x, n0y, n0z);
    if (n0z > 0.0f)      l = fmaxf(l, c0 * rcp(n0z));
    else if (n0z < 0.0f) h = fminf(h, c0 * rcp(n0z));
    else if (c0 > 0.0f)  { l = INFINITY; h = -INFINITY; }
    const float ex = c.p.x + c.d.x, ey = c.p.y + c.d.y, ez = c.p.z + c.d.z;
    const float c1 = dot3(ex, ey, ez, n1x, n1y, n1z);
    if (n1z > 0.0f)      h = fminf(h, c1 * rcp(n1z));
    else if (n1z < 0.0f) l = fmaxf(l, c1 * rcp(n1z));
    else if (c1 < 0.0f)  { l = INFINITY; h = -INFINITY; }
    lo = l;
    hi = h;
}

// Conservative cylinder radius (Section 3.3): largest distance of the inner
// control points (t0 and -t1 relative to the chord ends) to the chord line,
// plus the largest radius control value (convex hull of the radius Bezier).
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
    const float rmax = c.p.w + fmaxf(fmaxf(0.0f, c.t0.w), fmaxf(c.d.w, c.d.w - c.t1.w));
    return vsqrt(fmaxf(l0, l1)) + rmax;
}

// Unit ray (origin, +z) against the infinite cylinder of radius r about the
// line through o along a (Appendix A). False on a miss.
__device__ __forceinline__ bool unit_ray_cylinder(const V4 &o, const V4 &a, float r, float &te, float &tx)
{
    // both cases are evaluated and selected: no divergent branch
    const float g = fmaf(a.x, a.x, a.y * a.y);
    const bool parallel = g < kParallelG;
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

// Split quantities of Section 3.1: centre offset dp and split tangent tc.
__device__ __forceinline__ void split_terms(const Node &c, V4 &dp, V4 &tc)
{
    dp.x = fmaf(0.375f, c.t0.x - c.t1.x, 0.5f * c.d.x);
    dp.y = fmaf(0.375f, c.t0.y - c.t1.y, 0.5f * c.d.y);
    dp.z = fmaf(0.375f, c.t0.z - c.t1.z, 0.5f * c.d.z);
    dp.w = fmaf(0.375f, c.t0.w - c.t1.w, 0.5f * c.d.w);
    tc.x = fmaf(-0.125f, c.t0.x + c.t1.x, 0.25f * c.d.x);
    tc.y = fmaf(-0.125f, c.t0.y + c.t1.y, 0.25f * c.d.y);
    tc.z = fmaf(-0.125f, c.t0.z + c.t1.z, 0.25f * c.d.z);
    tc.w = fmaf(-0.125f, c.t0.w + c.t1.w, 0.25f * c.d.w);
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
    int32_t *counts;
};

struct Lane {
    Node c;                       // current node, {p, d, t0, t1} in the ray frame
    float lo, hi;                 // cropped t interval of the current node
    float tmax, t;                // ray tmax; hit distance once found
    uint32_t bits, start, size;   // Section 3.3: pending-sibling bits, integer interval
    uint32_t min_size;            // leaf size 2^(23 - depth)
    uint32_t cached;              // size of the pending children whose parent is cached (0: none)
    float slack;                  // conservative mode: bound on across-ray rounding of any node
    int32_t trips, splits, backtracks;
};

// Per-lane node storage for backtracking. The root is read only when a
// backtrack replays the path from it; the parent of the most recent split
// that left a sibling pending is cached so that the usual backtrack (to that
// sibling) rebuilds it with one split instead of a replay. Both layouts keep
// the cache in an LDS column per lane (conflict-free); the root lives in LDS
// as well (frees 16 VGPRs) or in registers -- a tuning choice.
template <bool LDS> struct RootStore;

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

template <> struct RootStore<true> {
    float *col;                               // this lane's column of a [32][64] tile
    __device__ __forceinline__ void put(const Node &r) { lds_put(col, r); }
    __device__ __forceinline__ void get(Node &r) const { lds_get(col, r); }
    __device__ __forceinline__ void put_parent(const Node &r) { lds_put(col + 16 * kWave, r); }
    __device__ __forceinline__ void get_parent(Node &r) const { lds_get(col + 16 * kWave, r); }
};

template <> struct RootStore<false> {
    Node root;
    float *col;                               // this lane's column of a [16][64] tile
    __device__ __forceinline__ void put(const Node &r) { root = r; }
    __device__ __forceinline__ void get(Node &r) const { r = root; }
    __device__ __forceinline__ void put_parent(const Node &r) { lds_put(col, r); }
    __device__ __forceinline__ void get_parent(Node &r) const { lds_get(col, r); }
};

// Load pair i, move it into the ray frame and start the search. False when
// the pair is a definite miss (bad index, depth, direction or tmax).
template <class Store>
__device__ __forceinline__ bool start_pair(const Args &a, int64_t i, Lane &L, Store &store)
{
    const int64_t ri = a.pair_ray ? (int64_t)a.pair_ray[i] : i;
    const int64_t fi = a.pair_fiber ? (int64_t)a.pair_fiber[i] : i;
    const uint32_t depth = a.pair_depth ? (uint32_t)a.pair_depth[i] : (uint32_t)a.depth;
    if (ri < 0 || ri >= a.n_rays || fi < 0 || fi >= a.n_fibers || depth > FI_MAX_DEPTH) return false;
    const float *R = a.rays + ri;
    L.tmax = R[6 * a.ray_stride];
    if (!(L.tmax == L.tmax)) return false;
    Node root;
    if (!root_in_ray_frame(R, a.ray_stride, a.fibers + fi, a.fiber_stride, root)) return false;
    store.put(root);
    L.c = root;
    cap_interval(L.c, L.tmax, L.lo, L.hi);
    L.bits = 0;
    L.start = 0;
    L.size = kRootSize;
    L.min_size = kRootSize >> depth;
    L.cached = 0;
    // Each split rounds a node's position at the magnitude of its partial sum,
    // which starts at the root's across-ray extent, so deep nodes inherit
    // errors of a few ulp of that extent; 2^-18 of it is a generous bound.
    L.slack = (fabsf(root.p.x) + fabsf(root.p.y) + fabsf(root.d.x) + fabsf(root.d.y) +
               fabsf(root.t0.x) + fabsf(root.t0.y) + fabsf(root.t1.x) + fabsf(root.t1.y)) * 0x1p-18f;
    L.trips = L.splits = L.backtracks = 0;
    return true;
}

enum { kGoOn = 0, kHit = 1, kMiss = 2 };

// Traversal variants: plain, counting, and conservative (for FP64 refinement:
// every pruning test is enlarged by a bound on its FP32 rounding error, so no
// surface point within that error is pruned; FP64 then decides).
enum { kPlain = 0, kCount = 1, kConservative = 2 };

// Bound on the rounding of a ray-plane distance c / n_z with c = <point, n>:
// the products' magnitudes over |n_z| (obliquity amplifies), plus the size
// of the result, at 2^-18 (64 ulp).
__device__ __forceinline__ float plane_slack(float px, float py, float pz, float nx, float ny, float nz, float t)
{
    return (fabsf(px * nx) + fabsf(py * ny) + fabsf(pz * nz)) * rcp(fabsf(nz)) * 0x1p-18f +
           fabsf(t) * 0x1p-18f;
}

// One loop trip of the paper's iteration (Appendix C, final listing): a
// pruning test of the current node, then a descent, a leaf hit, a miss, or a
// jump to the deepest pending sibling.
// The common case (test, split, ordering, descent) is straight-line code for
// every active lane: a lane that will stop still computes the split, which
// costs nothing on a SIMD that runs it for its neighbours anyway, and avoids
// divergent branches. Only the jump to a pending sibling branches.
template <int MODE, class Store>
__device__ __forceinline__ int trip(Lane &L, Store &store)
{
    float te, tx;
    float rad = conservative_radius(L.c);
    float lo = L.lo, hi = L.hi;
    if (MODE == kConservative) {
        rad += L.slack + rad * 0x1p-18f;
        const float tslack = (fabsf(lo) + fabsf(hi < INFINITY ? hi : lo)) * 0x1p-17f;
        lo -= tslack;
        hi += tslack;
    }
    const bool vis = unit_ray_cylinder(L.c.p, L.c.d, rad, te, tx) && fmaxf(te, lo) <= fminf(tx, hi);
    const bool leaf = L.size <= L.min_size;
    if (++L.trips > kMaxTrips) return kMiss;
    if (!vis) {
        if (L.bits == 0) return kMiss;
        // Section 3.3: jump to the deepest level with a pending sibling and
        // rebuild its parent -- the cached node, or a replay of the split
        // rules along the integer path from the root
        L.size = L.bits & (0u - L.bits);
        L.start ^= L.size;
        L.bits ^= L.size;
        L.start &= ~(L.size - 1u);
        if (kParentCache && L.cached == L.size) {
            store.get_parent(L.c);
        } else {
            store.get(L.c);
            for (uint32_t b = kRootSize >> 1; b > L.size; b >>= 1) {
                V4 dp, tc;
                split_terms(L.c, dp, tc);
                take_child(L.c, dp, tc, (L.start & b) != 0u);
            }
        }
        L.cached = 0;
        V4 dp, tc;
        split_terms(L.c, dp, tc);
        take_child(L.c, dp, tc, (L.start & L.size) != 0u);
        cap_interval(L.c, L.tmax, L.lo, L.hi);
        L.backtracks++;
        return kGoOn;
    }
    // Section 3.2: split plane through the centre, normal to the split tangent
    V4 dp, tc;
    split_terms(L.c, dp, tc);
    float nx = tc.x, ny = tc.y, nz = tc.z;
    const bool flat = zero3(nx, ny, nz);
    nx = flat ? L.c.d.x : nx;
    ny = flat ? L.c.d.y : ny;
    nz = flat ? L.c.d.z : nz;
    const float qx = L.c.p.x + dp.x, qy = L.c.p.y + dp.y, qz = L.c.p.z + dp.z;
    const float cs = dot3(qx, qy, qz, nx, ny, nz);
    const float tp = cs * rcp(nz);
    const bool oblique = nz != 0.0f;
    bool right, both;
    float nlo = L.lo, nhi = L.hi;
    if (MODE == kConservative) {
        // visit both halves unless the crossing is clearly outside [te, tx];
        // narrow by the far side of tp's rounding bound
        const float ep = plane_slack(qx, qy, qz, nx, ny, nz, tp);
        both = oblique ? (te - ep < tp && tp < tx + ep)
                       : (cs == 0.0f || fabsf(cs) <= L.slack * (fabsf(nx) + fabsf(ny)));
        if (tp > te) nhi = fminf(nhi, tp + ep);
        else         nlo = fmaxf(nlo, tp - ep);
    } else {
        both = oblique ? (te < tp && tp < tx) : cs == 0.0f;
        if (tp > te) nhi = fminf(nhi, tp);
        else         nlo = fmaxf(nlo, tp);
    }
    // the whole ray lies on the side of sign(-cs) when the plane is parallel
    right = oblique ? ((tp > te) != (nz > 0.0f)) : cs < 0.0f;
    if (oblique) { L.lo = nlo; L.hi = nhi; }
    if (leaf) { L.t = fmaxf(te, lo); return kHit; }
    if (kParentCache && both) store.put_parent(L.c);
    take_child(L.c, dp, tc, right);
    L.size >>= 1;
    if (both) {
        L.bits ^= L.size;
        if (kParentCache) L.cached = L.size;
    }
    if (right) L.start ^= L.size;
    L.splits++;
    return kGoOn;
}

// Write the result of pair i (Section 3.3: u from projecting the hit point
// onto the leaf chord; hit when t < tmax).
template <int MODE>
__device__ __forceinline__ void finish(const Args &a, int64_t i, const Lane &L, bool reached)
{
    float t = INFINITY, u = __builtin_nanf("");
    bool hit = false;
    if (reached && L.t < L.tmax) {
        const float cc = dot3(L.c.d.x, L.c.d.y, L.c.d.z, L.c.d.x, L.c.d.y, L.c.d.z);
        float ul = 0.0f;
        if (cc > 0.0f) {
            ul = dot3(-L.c.p.x, -L.c.p.y, L.t - L.c.p.z, L.c.d.x, L.c.d.y, L.c.d.z) * rcp(cc);
            ul = fminf(1.0f, fmaxf(0.0f, ul));
        }
        t = L.t;
        u = fmaf(ul, (float)L.size * 0x1p-23f, (float)L.start * 0x1p-23f);
        hit = true;
    }
    a.t_out[i] = t;
    a.u_out[i] = u;
    a.hit_out[i] = hit ? 1 : 0;
    if (MODE == kCount) {
        int32_t *cn = a.counts + 4 * i;
        cn[0] = L.trips;
        cn[1] = L.splits;
        cn[2] = L.backtracks;
        cn[3] = hit ? (int32_t)(23 - (31 - __builtin_clz(L.size))) : -1;
    }
}

template <int MODE>
__device__ __forceinline__ void finish_invalid(const Args &a, int64_t i)
{
    a.t_out[i] = INFINITY;
    a.u_out[i] = __builtin_nanf("");
    a.hit_out[i] = 0;
    if (MODE == kCount) {
        int32_t *cn = a.counts + 4 * i;
        cn[0] = 0; cn[1] = 0; cn[2] = 0; cn[3] = -1;
    }
}

// ---------------------------------------------------------------------------
// Persistent kernel: each 64-lane wave pulls pairs from a device queue and
// refills finished lanes in batches, so lanes of uneven trip counts (a miss
// ends after one or a few trips, a hit needs depth + 1 or more) keep the SIMD
// busy instead of idling until the slowest lane of a fixed batch finishes.
// ---------------------------------------------------------------------------

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

// queue[0]: next unclaimed pair; queue[1]: waves finished. The last wave to
// finish returns both to zero, so the slot is ready for the next launch.
// BATCHED: pairs are numbered across a table of scenes (one persistent
// launch for many independent problems); otherwise the single problem a0.
// Work distribution: wave w first owns the static range [w S, (w + 1) S)
// (no atomics), then pulls dynamic chunks of `chunk` pairs from queue[0]
// (one device-scope atomic per chunk, offset past all static ranges). Lanes
// are refilled from the wave's current range, held in scalar registers.
struct Sched {
    int64_t static_per_wave;     // S
    int32_t chunk;               // dynamic chunk, pairs
    int32_t refill;              // refill once this many lanes are free
};

template <int MODE, bool BATCHED, bool ROOT_LDS>
__global__ __launch_bounds__(kWave) void k_traverse(Args a0, const Args *scenes, const int64_t *offsets,
                                                    int n_scenes, int64_t total, uint32_t *queue, Sched sc)
{
    __shared__ float s_nodes[((ROOT_LDS ? 16 : 0) + (kParentCache ? 16 : 0) + 1) * kWave];
    const int lane = threadIdx.x;
    RootStore<ROOT_LDS> store;
    store.col = s_nodes + lane;
    Lane L;
    int64_t idx = 0;
    int scene = 0;
    bool active = false;
    bool exhausted = false;
    const int64_t dyn0 = (int64_t)gridDim.x * sc.static_per_wave;     // first dynamic pair
    int64_t next = (int64_t)blockIdx.x * sc.static_per_wave;           // wave-uniform range
    int64_t end = next + sc.static_per_wave < total ? next + sc.static_per_wave : total;
    for (;;) {
        const uint64_t free_mask = __ballot(!active);
        const int n_free = __popcll(free_mask);
        if (!exhausted && (n_free >= sc.refill || n_free == kWave)) {
            if (next >= end && dyn0 >= total) {
                exhausted = true;                  // static ranges cover every pair
            } else if (next >= end) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&queue[0], (uint32_t)sc.chunk);
                base = __builtin_amdgcn_readfirstlane(base);
                next = dyn0 + (int64_t)base;
                end = next + sc.chunk < total ? next + sc.chunk : total;
                if (next >= total) exhausted = true;
            }
            if (!exhausted) {
                const int64_t avail = end - next;
                const int take = avail < n_free ? (int)avail : n_free;
                if (!active) {
                    const int rank = (int)lanes_below(free_mask);
                    if (rank < take) {
                        const int64_t g = next + rank;
                        if constexpr (BATCHED) {
                            scene = find_scene(offsets, n_scenes, g);
                            idx = g - offsets[scene];
                            const Args a = scenes[scene];
                            active = start_pair(a, idx, L, store);
                            if (!active) finish_invalid<MODE>(a, idx);
                        } else {
                            idx = g;
                            active = start_pair(a0, idx, L, store);
                            if (!active) finish_invalid<MODE>(a0, idx);
                        }
                    }
                }
                next += take;
            }
        }
        if (__ballot(active) == 0) {
            if (exhausted) break;
            continue;
        }
        if (active) {
            const int st = trip<MODE>(L, store);
            if (st != kGoOn) {
                if constexpr (BATCHED) {
                    const Args a = scenes[scene];
                    finish<MODE>(a, idx, L, st == kHit);
                } else {
                    finish<MODE>(a0, idx, L, st == kHit);
                }
                active = false;
            }
        }
    }
    if (lane == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

// Zero a queue slot from inside a stream or graph (a kernel, not a memset
// node, so that graph replays see a fresh queue).
__global__ void k_reset_queue(uint32_t *queue)
{
    if (threadIdx.x < 2) queue[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// FP64 refinement of a hit onto the swept-disc surface
// ---------------------------------------------------------------------------
//
// The leaf cylinders converge to the surface swept by a disc of radius r(u)
// centred on C(u) and normal to C'(u) (Sec. 3.2: the limit surface of the
// cylinders maps the intersection to the closest point on the curve). At
// depth > 16 the FP32 leaf locates the entry to within a few leaf widths;
// this step solves for the surface point in FP64:
//   f1(t, u) = <P - C(u), C'(u)> = 0      (P = (0, 0, t): the ray point)
//   f2(t, u) = |P - C(u)|^2 - r(u)^2 = 0
// by Newton's method from the FP32 (t, u), accepts the root if it is an entry
// (the signed distance decreases along the ray) close to the FP32 estimate,
// and otherwise brackets the entry on a window of leaves around the FP32 u.
// The end discs at u = 0 and u = 1 are candidates when the window reaches
// them. No surface point near the leaf means the exact surface is missed.

constexpr int kRefineAbove = 16;         // refine hits at depth > 16

struct Curve64 { double q[4][4]; };      // control points in the FP64 ray frame (x, y, z, r)

__device__ __forceinline__ bool curve_in_ray_frame(const float *R, int64_t rs, const float *F,
                                                   int64_t fs, Curve64 &c)
{
    const double ox = R[0], oy = R[rs], oz = R[2 * rs];
    const double dx = R[3 * rs], dy = R[4 * rs], dz = R[5 * rs];
    const double n2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(n2 > 0.0) || !(n2 < INFINITY)) return false;
    const double il = 1.0 / sqrt(n2);
    const double w[3] = {dx * il, dy * il, dz * il};
    double u[3], v[3];
    make_onb(w[0], w[1], w[2], u, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double ex = (double)F[(4 * k) * fs] - ox;
        const double ey = (double)F[(4 * k + 1) * fs] - oy;
        const double ez = (double)F[(4 * k + 2) * fs] - oz;
        c.q[k][0] = fma(ex, u[0], fma(ey, u[1], ez * u[2]));
        c.q[k][1] = fma(ex, v[0], fma(ey, v[1], ez * v[2]));
        c.q[k][2] = fma(ex, w[0], fma(ey, w[1], ez * w[2]));
        c.q[k][3] = F[(4 * k + 3) * fs];
    }
    return true;
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

// Ray point in the disc plane at u, and its signed excess |P-C|^2 - r^2.
__device__ __forceinline__ bool disc_point(const Curve64 &c, double u, double &t, double &phi)
{
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    if (D[2] == 0.0) return false;
    t = (C[0] * D[0] + C[1] * D[1] + C[2] * D[2]) / D[2];
    const double h = t - C[2];
    phi = C[0] * C[0] + C[1] * C[1] + h * h - C[3] * C[3];
    return true;
}

// Derivative along the ray of the signed excess at a surface point: negative
// at an entry.
__device__ __forceinline__ double entry_slope(const double C[4], const double D[4], const double E[3], double t)
{
    const double h = t - C[2];
    const double pe = -C[0] * E[0] - C[1] * E[1] + h * E[2];
    const double dd = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    const double den = 9.0 * dd - 6.0 * pe;
    return 2.0 * h - (den != 0.0 ? 2.0 * C[3] * 9.0 * D[3] * D[2] / den : 0.0);
}

__device__ __forceinline__ bool newton_surface(const Curve64 &c, double &t, double &u)
{
    for (int it = 0; it < 8; ++it) {
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
        if (fabs(du) <= 1e-16 && fabs(dt) <= 1e-16 * fabs(t)) break;
    }
    double C[4], D[4], E[3];
    eval_curve(c, u, C, D, E);
    const double h = t - C[2];
    const double scale = fmax(C[3] * C[3], 1e-300);
    const double f1 = h * D[2] - C[0] * D[0] - C[1] * D[1];
    const double f2 = C[0] * C[0] + C[1] * C[1] + h * h - C[3] * C[3];
    const double dn = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    return fabs(f2) <= 1e-9 * scale && fabs(f1) <= 1e-9 * C[3] * dn && entry_slope(C, D, E, t) < 0.0;
}

// Bracketed search of the entry on [ua, ub]: sample the disc excess, take the
// first sign change towards smaller t, bisect it.
__device__ __forceinline__ bool bracket_surface(const Curve64 &c, double ua, double ub, double tmax,
                                                double &t_best, double &u_best)
{
    constexpr int kSamples = 48;
    bool found = false;
    double pu = ua, pt = 0.0, pphi = 0.0;
    bool pok = disc_point(c, pu, pt, pphi);
    for (int k = 1; k <= kSamples; ++k) {
        const double cu = ua + (ub - ua) * k / kSamples;
        double ct, cphi;
        const bool cok = disc_point(c, cu, ct, cphi);
        if (pok && cok && ((pphi <= 0.0) != (cphi <= 0.0))) {
            double lo = pu, hi = cu;
            const bool lo_inside = pphi <= 0.0;
            for (int it = 0; it < 60; ++it) {
                const double mid = 0.5 * (lo + hi);
                double mt, mphi;
                if (!disc_point(c, mid, mt, mphi)) break;
                if ((mphi <= 0.0) == lo_inside) lo = mid; else hi = mid;
            }
            const double ur = 0.5 * (lo + hi);
            double tr, phir;
            if (disc_point(c, ur, tr, phir)) {
                double C[4], D[4], E[3];
                eval_curve(c, ur, C, D, E);
                if (tr >= 0.0 && tr < tmax && tr < t_best && entry_slope(C, D, E, tr) < 0.0) {
                    t_best = tr;
                    u_best = ur;
                    found = true;
                }
            }
        }
        pu = cu; pt = ct; pphi = cphi; pok = cok;
    }
    return found;
}

__global__ __launch_bounds__(256) void k_refine(Args a, double *t64, double *u64)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n_pairs) return;
    const uint32_t depth = a.pair_depth ? (uint32_t)a.pair_depth[i] : (uint32_t)a.depth;
    const bool hit = a.hit_out[i] != 0;
    const float t32 = a.t_out[i], u32 = a.u_out[i];
    if (!hit || depth <= (uint32_t)kRefineAbove) {
        t64[i] = hit ? (double)t32 : INFINITY;
        u64[i] = hit ? (double)u32 : __builtin_nan("");
        return;
    }
    const int64_t ri = a.pair_ray ? (int64_t)a.pair_ray[i] : i;
    const int64_t fi = a.pair_fiber ? (int64_t)a.pair_fiber[i] : i;
    const float *R = a.rays + ri;
    const double tmax = R[6 * a.ray_stride];
    Curve64 c;
    double t_best = INFINITY, u_best = __builtin_nan("");
    if (curve_in_ray_frame(R, a.ray_stride, a.fibers + fi, a.fiber_stride, c)) {
        double t = t32, u = u32;
        const double leaf = ldexp(1.0, -(int)depth);
        if (newton_surface(c, t, u) && u >= 0.0 && u <= 1.0 && t >= 0.0 && t < tmax &&
            fabs(t - (double)t32) <= 1e-5 * fmax(1.0, fabs((double)t32)) && fabs(u - (double)u32) <= 256.0 * leaf + 1e-4) {
            t_best = t;
            u_best = u;
        } else {
            const double w = fmax(256.0 * leaf, 1e-4);
            bracket_surface(c, fmax(0.0, (double)u32 - w), fmin(1.0, (double)u32 + w), tmax, t_best, u_best);
        }
        // end discs within reach of the FP32 estimate
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double ue = (double)e;
            if (fabs(ue - (double)u32) > fmax(256.0 * leaf, 1e-4)) continue;
            double C[4], D[4], E[3];
            eval_curve(c, ue, C, D, E);
            if (D[2] == 0.0) continue;
            const double tc = (C[0] * D[0] + C[1] * D[1] + C[2] * D[2]) / D[2];
            const double h = tc - C[2];
            if (C[0] * C[0] + C[1] * C[1] + h * h <= C[3] * C[3] && tc >= 0.0 && tc < tmax && tc < t_best) {
                t_best = tc;
                u_best = ue;
            }
        }
    }
    const bool ok = t_best < INFINITY;
    t64[i] = t_best;
    u64[i] = u_best;
    a.hit_out[i] = ok ? 1 : 0;
    a.t_out[i] = ok ? (float)t_best : INFINITY;
    a.u_out[i] = ok ? (float)u_best : __builtin_nanf("");
}

int check_common(const float *rays, int64_t ray_stride, int64_t n_rays,
                 const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                 const int32_t *pair_ray, const int32_t *pair_fiber,
                 int32_t depth, int64_t n_pairs, uint32_t flags,
                 const void *t_out, const void *u_out, const void *hit_out)
{
    if (n_pairs < 0 || n_rays < 0 || n_fibers < 0) return FI_ERR_RANGE;
    if (depth < 0 || depth > FI_MAX_DEPTH) return FI_ERR_RANGE;
    if ((flags & ~(uint32_t)FI_FP64_REFINE) != 0u) return FI_ERR_RANGE;
    if (n_pairs == 0) return FI_OK;
    if (!rays || !fibers || !t_out || !u_out || !hit_out) return FI_ERR_NULL;
    if (ray_stride < n_rays || fiber_stride < n_fibers) return FI_ERR_RANGE;
    if (!pair_ray && n_pairs > n_rays) return FI_ERR_RANGE;
    if (!pair_fiber && n_pairs > n_fibers) return FI_ERR_RANGE;
    if (n_pairs > (int64_t)0x7fffffff - 64) return FI_ERR_RANGE;   // 32-bit work queue
    return FI_OK;
}

// ---------------------------------------------------------------------------
// Kernel variants, work-queue slots and launch shape
// ---------------------------------------------------------------------------

using TraverseFn = void (*)(Args, const Args *, const int64_t *, int, int64_t, uint32_t *, Sched);

// [mode][batched][root in LDS]
const TraverseFn kTraverse[3][2][2] = {
    {{k_traverse<kPlain, false, false>, k_traverse<kPlain, false, true>},
     {k_traverse<kPlain, true, false>, k_traverse<kPlain, true, true>}},
    {{k_traverse<kCount, false, false>, k_traverse<kCount, false, true>},
     {k_traverse<kCount, true, false>, k_traverse<kCount, true, true>}},
    {{k_traverse<kConservative, false, false>, k_traverse<kConservative, false, true>},
     {k_traverse<kConservative, true, false>, k_traverse<kConservative, true, true>}},
};

// Queue slots in a file-scope device array (zero at load; each launch leaves
// its slot zero). Launches take slots round-robin, so up to kSlots launches
// may be in flight at once on one device without sharing a slot.
constexpr int kSlots = 256;
__device__ __align__(256) uint32_t g_queue_slots[kSlots * 2];

constexpr int kMaxDevices = 64;
constexpr int kStageSlots = 4;                 // pinned staging for batched scene tables
constexpr size_t kStageBytes = 1u << 20;

struct DeviceInfo {
    std::atomic<bool> ready;
    uint32_t *slots;                           // device address of g_queue_slots on this device
    int cus;
    int resident[3][2][2];                     // resident 64-lane workgroups per CU, per variant
    std::mutex stage_mutex;
    void *stage[kStageSlots];                  // pinned host buffers (allocated on first batched call)
    hipEvent_t stage_done[kStageSlots];
    int stage_next;
};
DeviceInfo g_dev[kMaxDevices];
std::mutex g_dev_mutex;
std::atomic<uint32_t> g_next_slot{0};

int current_device(int &dev)
{
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FI_ERR_HIP;
    return FI_OK;
}

int device_info(DeviceInfo *&out)
{
    int dev = 0;
    if (current_device(dev) != FI_OK) return FI_ERR_HIP;
    DeviceInfo &d = g_dev[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(g_dev_mutex);
        if (!d.ready.load(std::memory_order_relaxed)) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_queue_slots)) != hipSuccess || !p) return FI_ERR_HIP;
            if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                return FI_ERR_HIP;
            for (int m = 0; m < 3; ++m)
                for (int b = 0; b < 2; ++b)
                    for (int l = 0; l < 2; ++l) {
                        int nb = 0;
                        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)kTraverse[m][b][l],
                                                                         kWave, 0) != hipSuccess)
                            return FI_ERR_HIP;
                        d.resident[m][b][l] = nb > 0 ? nb : 1;
                    }
            d.slots = (uint32_t *)p;
            d.stage_next = 0;
            d.ready.store(true, std::memory_order_release);
        }
    }
    out = &d;
    return FI_OK;
}

// Launch defaults of single-problem calls (and of batches without a tuned
// entry); measured choices, overridable when building.
#ifndef FIBERHIT_DEFAULT_REFILL
#define FIBERHIT_DEFAULT_REFILL 32
#endif
#ifndef FIBERHIT_DEFAULT_WAVES_PER_SIMD
#define FIBERHIT_DEFAULT_WAVES_PER_SIMD 0
#endif
#ifndef FIBERHIT_DEFAULT_ROOT_IN_LDS
#define FIBERHIT_DEFAULT_ROOT_IN_LDS 0
#endif
#ifndef FIBERHIT_DEFAULT_CHUNK
#define FIBERHIT_DEFAULT_CHUNK 128
#endif
#ifndef FIBERHIT_DEFAULT_STATIC_PCT
#define FIBERHIT_DEFAULT_STATIC_PCT 100
#endif
fi_tuning default_tuning()
{
    return fi_tuning{FIBERHIT_DEFAULT_REFILL, FIBERHIT_DEFAULT_WAVES_PER_SIMD, FIBERHIT_DEFAULT_ROOT_IN_LDS,
                     FIBERHIT_DEFAULT_CHUNK, FIBERHIT_DEFAULT_STATIC_PCT};
}

// Autotune results, kept for the process: keyed by device and the size class
// of a batch (log2 of its total pairs and of its problem count). A batch
// launched without an explicit tuning uses the entry of its class if one
// exists.
std::mutex g_tune_mutex;
std::map<uint64_t, fi_tuning> g_tune_cache;

uint64_t tune_key(int device, int64_t total, int n_scenes)
{
    int lt = 0, ls = 0;
    while ((int64_t)1 << (lt + 1) <= total && lt < 62) ++lt;
    while ((1 << (ls + 1)) <= n_scenes && ls < 30) ++ls;
    return ((uint64_t)device << 16) | ((uint64_t)lt << 8) | (uint64_t)ls;
}

fi_tuning tuned_or_default(int64_t total, int n_scenes)
{
    int dev = 0;
    if (current_device(dev) != FI_OK) return default_tuning();
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it = g_tune_cache.find(tune_key(dev, total, n_scenes));
    return it == g_tune_cache.end() ? default_tuning() : it->second;
}

void remember_tuning(int64_t total, int n_scenes, const fi_tuning &t)
{
    int dev = 0;
    if (current_device(dev) != FI_OK) return;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[tune_key(dev, total, n_scenes)] = t;
}

int64_t total_pairs(const fi_scene *sc, int32_t n)
{
    int64_t t = 0;
    for (int k = 0; k < n; ++k) t += sc[k].n_pairs > 0 ? sc[k].n_pairs : 0;
    return t;
}

int check_tuning(const fi_tuning &t)
{
    if (t.refill < 1 || t.refill > kWave || t.waves_per_simd < -1 || t.waves_per_simd > 16 ||
        (t.root_in_lds != 0 && t.root_in_lds != 1) || t.chunk < 1 || t.chunk > (1 << 16) ||
        t.static_pct < 0 || t.static_pct > 100)
        return FI_ERR_RANGE;
    return FI_OK;
}

unsigned grid_for(const DeviceInfo &d, int mode, bool batched, const fi_tuning &t, int64_t n_pairs)
{
    const int64_t needed = (n_pairs + kWave - 1) / kWave;
    if (t.waves_per_simd < 0) return (unsigned)needed;       // one wave per 64 pairs: plain grid
    int per_cu = d.resident[mode][batched ? 1 : 0][t.root_in_lds];
    if (t.waves_per_simd > 0 && 4 * t.waves_per_simd < per_cu) per_cu = 4 * t.waves_per_simd;
    const int64_t resident = (int64_t)per_cu * d.cus;
    return (unsigned)(needed < resident ? needed : resident);
}

Sched sched_for(const fi_tuning &t, unsigned grid, int64_t total)
{
    Sched sc;
    // static share: static_pct % of an even split, in whole lane batches
    const int64_t even = grid ? total / grid : 0;
    sc.static_per_wave = (even * t.static_pct / 100) / kWave * kWave;
    // one wave per lane batch: each wave owns exactly its batch, no queue
    if (t.waves_per_simd < 0) sc.static_per_wave = kWave;
    sc.chunk = t.chunk;
    sc.refill = t.refill;
    return sc;
}

int launch_traverse(const DeviceInfo &d, int mode, bool batched, const fi_tuning &t, const Args &a0,
                    const Args *scenes, const int64_t *offsets, int n_scenes, int64_t total,
                    uint32_t *queue, hipStream_t s)
{
    const unsigned grid = grid_for(d, mode, batched, t, total);
    if (grid == 0) return FI_OK;
    // queue[0] ends below total + (grid + 1) * chunk (one claim past the end per
    // wave); keep that within 32 bits
    if (t.waves_per_simd >= 0 && total + ((int64_t)grid + 1) * t.chunk >= ((int64_t)1 << 32))
        return FI_ERR_RANGE;
    hipLaunchKernelGGL(kTraverse[mode][batched ? 1 : 0][t.root_in_lds], dim3(grid), dim3(kWave), 0, s,
                       a0, scenes, offsets, n_scenes, total, queue, sched_for(t, grid, total));
    return FI_OK;
}

int launch(int mode, const Args &a, double *t64, double *u64, void *stream)
{
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    const int st = device_info(d);
    if (st != FI_OK) return st;
    uint32_t *slot = d->slots + 2 * (g_next_slot.fetch_add(1u) % kSlots);
    hipStream_t s = (hipStream_t)stream;
    const int lst = launch_traverse(*d, mode, false, default_tuning(), a, nullptr, nullptr, 1, a.n_pairs, slot, s);
    if (lst != FI_OK) return lst;
    if (t64) {
        const unsigned g2 = (unsigned)((a.n_pairs + 255) / 256);
        hipLaunchKernelGGL(k_refine, dim3(g2), dim3(256), 0, s, a, t64, u64);
    }
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Batched problems
// ---------------------------------------------------------------------------

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t table_bytes(int n) { return align256((size_t)n * sizeof(Args)) + align256((size_t)(n + 1) * sizeof(int64_t)); }

int scenes_to_table(const fi_scene *sc, int32_t n, Args *tab, int64_t *off)
{
    off[0] = 0;
    for (int k = 0; k < n; ++k) {
        const fi_scene &x = sc[k];
        const int st = check_common(x.rays, x.ray_stride, x.n_rays, x.fibers, x.fiber_stride, x.n_fibers,
                                    x.pair_ray, x.pair_fiber, x.depth, x.n_pairs, 0u, x.t_out, x.u_out, x.hit_out);
        if (st != FI_OK) return st;
        tab[k] = Args{x.rays, x.ray_stride, x.n_rays, x.fibers, x.fiber_stride, x.n_fibers,
                      x.pair_ray, x.pair_fiber, x.pair_depth, x.depth, x.n_pairs,
                      x.t_out, x.u_out, x.hit_out, nullptr};
        off[k + 1] = off[k] + x.n_pairs;
    }
    if (off[n] > (int64_t)0x7fffffff - 64) return FI_ERR_RANGE;
    return FI_OK;
}

// Layout of a batched workspace: scene table, pair offsets, queue.
struct BatchLayout {
    Args *scenes;
    int64_t *offsets;
    uint32_t *queue;
};

BatchLayout layout_of(void *ws, int n)
{
    char *p = (char *)ws;
    BatchLayout L;
    L.scenes = (Args *)p;
    L.offsets = (int64_t *)(p + align256((size_t)n * sizeof(Args)));
    L.queue = (uint32_t *)(p + table_bytes(n));
    return L;
}

int batched_enqueue(const fi_scene *scenes, int32_t n_scenes, const fi_tuning &t, void *workspace,
                    size_t workspace_bytes, hipStream_t s)
{
    DeviceInfo *d = nullptr;
    int st = device_info(d);
    if (st != FI_OK) return st;
    const size_t tb = table_bytes(n_scenes);
    if (!workspace || workspace_bytes < tb + 256) return FI_ERR_WORKSPACE;
    if (tb > kStageBytes) return FI_ERR_RANGE;
    std::lock_guard<std::mutex> lock(d->stage_mutex);
    const int k = d->stage_next;
    if (!d->stage[k]) {
        if (hipHostMalloc(&d->stage[k], kStageBytes, hipHostMallocDefault) != hipSuccess) return FI_ERR_HIP;
        if (hipEventCreateWithFlags(&d->stage_done[k], hipEventDisableTiming) != hipSuccess) return FI_ERR_HIP;
    } else if (hipEventSynchronize(d->stage_done[k]) != hipSuccess) {
        return FI_ERR_HIP;
    }
    char *host = (char *)d->stage[k];
    st = scenes_to_table(scenes, n_scenes, (Args *)host, (int64_t *)(host + align256((size_t)n_scenes * sizeof(Args))));
    if (st != FI_OK) return st;
    const int64_t total = ((int64_t *)(host + align256((size_t)n_scenes * sizeof(Args))))[n_scenes];
    const BatchLayout L = layout_of(workspace, n_scenes);
    if (hipMemcpyAsync(workspace, host, tb, hipMemcpyHostToDevice, s) != hipSuccess) return FI_ERR_HIP;
    if (hipEventRecord(d->stage_done[k], s) != hipSuccess) return FI_ERR_HIP;
    d->stage_next = (k + 1) % kStageSlots;
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, L.queue);
    if (total > 0) {
        const int lst = launch_traverse(*d, kPlain, true, t, Args{}, L.scenes, L.offsets, n_scenes, total, L.queue, s);
        if (lst != FI_OK) return lst;
    }
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

}  // namespace

struct fi_batch_plan {
    int device;
    void *mem;                 // device copy of the scene table, offsets and queue
    int n_scenes;
    int64_t total;
    fi_tuning tuning;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {
int fi_version(void) { return (0 << 16) | (3 << 8) | 0; }

const char *fi_strerror(int status)
{
    switch (status) {
    case FI_OK: return "ok";
    case FI_ERR_NULL: return "a required pointer is NULL";
    case FI_ERR_RANGE: return "a count, stride, depth or flag is out of range";
    case FI_ERR_HIP: return "the HIP runtime reported an error";
    case FI_ERR_WORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
    }
}

int fiber_intersect_pairs(const float *rays, int64_t ray_stride, int64_t n_rays,
                          const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                          const int32_t *pair_ray, const int32_t *pair_fiber,
                          const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                          uint32_t flags,
                          float *t_out, float *u_out, uint8_t *hit_out,
                          double *t64_out, double *u64_out,
                          void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    const bool refine = (flags & FI_FP64_REFINE) != 0u;
    if (refine && (!t64_out || !u64_out)) return FI_ERR_NULL;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, nullptr};
    return launch(refine ? kConservative : kPlain, a, refine ? t64_out : nullptr,
                  refine ? u64_out : nullptr, stream);
}

int fiber_intersect_counts(const float *rays, int64_t ray_stride, int64_t n_rays,
                           const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                           const int32_t *pair_ray, const int32_t *pair_fiber,
                           const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                           uint32_t flags,
                           float *t_out, float *u_out, uint8_t *hit_out,
                           int32_t *counts_out, void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    if (!counts_out) return FI_ERR_NULL;
    if (flags != 0u) return FI_ERR_RANGE;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, counts_out};
    return launch(kCount, a, nullptr, nullptr, stream);
}


size_t fiber_batched_workspace_bytes(int32_t n_scenes)
{
    if (n_scenes < 0) return 0;
    return table_bytes(n_scenes) + 256;
}

int fiber_intersect_batched(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, void *workspace, size_t workspace_bytes, void *stream)
{
    if (n_scenes < 0 || flags != 0u) return FI_ERR_RANGE;
    if (n_scenes == 0) return FI_OK;
    if (!scenes) return FI_ERR_NULL;
    const fi_tuning t = tuning ? *tuning : tuned_or_default(total_pairs(scenes, n_scenes), n_scenes);
    if (check_tuning(t) != FI_OK) return FI_ERR_RANGE;
    (void)hipGetLastError();
    return batched_enqueue(scenes, n_scenes, t, workspace, workspace_bytes, (hipStream_t)stream);
}

int fiber_batch_plan_create(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, fi_batch_plan **plan_out)
{
    if (!plan_out) return FI_ERR_NULL;
    *plan_out = nullptr;
    if (n_scenes <= 0 || flags != 0u) return FI_ERR_RANGE;
    if (!scenes) return FI_ERR_NULL;
    const fi_tuning t = tuning ? *tuning : tuned_or_default(total_pairs(scenes, n_scenes), n_scenes);
    if (check_tuning(t) != FI_OK) return FI_ERR_RANGE;
    (void)hipGetLastError();
    DeviceInfo *d = nullptr;
    int st = device_info(d);
    if (st != FI_OK) return st;
    const size_t tb = table_bytes(n_scenes);
    char *host = (char *)malloc(tb);
    if (!host) return FI_ERR_RANGE;
    st = scenes_to_table(scenes, n_scenes, (Args *)host, (int64_t *)(host + align256((size_t)n_scenes * sizeof(Args))));
    if (st != FI_OK) { free(host); return st; }
    fi_batch_plan *p = new fi_batch_plan();
    p->n_scenes = n_scenes;
    p->total = ((int64_t *)(host + align256((size_t)n_scenes * sizeof(Args))))[n_scenes];
    p->tuning = t;
    current_device(p->device);
    hipStream_t cs = nullptr;
    bool ok = hipMalloc(&p->mem, tb + 256) == hipSuccess &&
              hipMemcpy(p->mem, host, tb, hipMemcpyHostToDevice) == hipSuccess &&
              hipStreamCreate(&cs) == hipSuccess;
    free(host);
    if (ok) {
        const BatchLayout L = layout_of(p->mem, n_scenes);
        ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, cs, L.queue);
            int lst = FI_OK;
            if (p->total > 0)
                lst = launch_traverse(*d, kPlain, true, t, Args{}, L.scenes, L.offsets, n_scenes, p->total,
                                      L.queue, cs);
            ok = hipStreamEndCapture(cs, &p->graph) == hipSuccess && lst == FI_OK &&
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
    if (n_scenes <= 0 || flags != 0u || repeats < 1) return FI_ERR_RANGE;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FI_ERR_HIP;
    const int refills[] = {16, 32, 48};
    const int occ[] = {3, 4, 0};
    const int chunks[] = {64, 256};
    const int statics[] = {50, 80, 100};
    float best_t = INFINITY;
    fi_tuning bt = default_tuning();
    int st = FI_OK;
    for (int lds = 0; lds < 2 && st == FI_OK; ++lds)
        for (int oi = 0; oi < 3 && st == FI_OK; ++oi)
          for (int ci = 0; ci < 2 && st == FI_OK; ++ci)
            for (int si = 0; si < 3 && st == FI_OK; ++si)
              for (int ri = 0; ri < 3 && st == FI_OK; ++ri) {
                const fi_tuning t{refills[ri], occ[oi], lds, chunks[ci], statics[si]};
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
    remember_tuning(total_pairs(scenes, n_scenes), n_scenes, bt);
    return FI_OK;
}

}  // extern "C"
