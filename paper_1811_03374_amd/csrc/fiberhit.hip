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

#include "fiberhit.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kRootSize = 1u << 23;      // parametric domain [0, 1) in units of 2^-23
constexpr int kMaxTrips = 1 << 16;            // hang guard; real pairs need < 200 trips
constexpr float kParallelG = 1e-30f;          // axis treated as parallel to the ray below this

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

// Orthonormal basis (u, v) completing the unit w: Duff et al. 2017, the
// revision of Frisvad's construction cited in Section 3.3.
__device__ __forceinline__ void make_onb(double wx, double wy, double wz,
                                         double u[3], double v[3])
{
    const double s = copysign(1.0, wz);
    const double a = -1.0 / (s + wz);
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
    const double il = 1.0 / sqrt(n2);
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
    if (n0z > 0.0f)      l = fmaxf(l, c0 / n0z);
    else if (n0z < 0.0f) h = fminf(h, c0 / n0z);
    else if (c0 > 0.0f)  { l = INFINITY; h = -INFINITY; }
    const float ex = c.p.x + c.d.x, ey = c.p.y + c.d.y, ez = c.p.z + c.d.z;
    const float c1 = dot3(ex, ey, ez, n1x, n1y, n1z);
    if (n1z > 0.0f)      h = fminf(h, c1 / n1z);
    else if (n1z < 0.0f) l = fmaxf(l, c1 / n1z);
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
    const float g = fmaf(a.x, a.x, a.y * a.y);
    if (g < kParallelG) {
        if (fmaf(o.x, o.x, o.y * o.y) < r * r) { te = -INFINITY; tx = INFINITY; return true; }
        return false;
    }
    const float dd = fmaf(a.x, o.y, -(a.y * o.x));
    const float h = rcp(g);
    const float e = fmaf(-(dd * dd), h, r * r);
    if (!(e >= 0.0f)) return false;
    const float tc = fmaf(-a.z, fmaf(a.x, o.x, a.y * o.y) * h, o.z);
    const float s = vsqrt(e * fmaf(a.z, a.z, g) * h);
    te = tc - s;
    tx = tc + s;
    return true;
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
// One pair
// ---------------------------------------------------------------------------

struct Args {
    const float *rays; int64_t ray_stride; int64_t n_rays;
    const float *fibers; int64_t fiber_stride; int64_t n_fibers;
    const int32_t *pair_ray; const int32_t *pair_fiber; const uint8_t *pair_depth;
    int32_t depth; int64_t n_pairs;
    float *t_out; float *u_out; uint8_t *hit_out;
    int32_t *counts;
};

struct Result { float t, u; bool hit; int32_t tests, splits, backtracks, level; };

template <bool COUNT>
__device__ __forceinline__ Result trace_pair(const Args &a, int64_t i)
{
    Result res{INFINITY, __builtin_nanf(""), false, 0, 0, 0, -1};
    const int64_t ri = a.pair_ray ? (int64_t)a.pair_ray[i] : i;
    const int64_t fi = a.pair_fiber ? (int64_t)a.pair_fiber[i] : i;
    const int depth = a.pair_depth ? (int)a.pair_depth[i] : a.depth;
    if (ri < 0 || ri >= a.n_rays || fi < 0 || fi >= a.n_fibers || depth > FI_MAX_DEPTH) return res;

    const float *R = a.rays + ri;
    const float tmax = R[6 * a.ray_stride];
    Node root;
    if (!(tmax == tmax) || !root_in_ray_frame(R, a.ray_stride, a.fibers + fi, a.fiber_stride, root))
        return res;

    Node c = root;
    float lo, hi;
    cap_interval(c, tmax, lo, hi);
    uint32_t bits = 0, size = kRootSize, start = 0;
    const uint32_t min_size = kRootSize >> depth;
    bool found = false;
    float t = INFINITY;

    for (int trip = 0; trip < kMaxTrips; ++trip) {
        if (COUNT) res.tests++;
        float te, tx;
        const float rad = conservative_radius(c);
        const bool vis = unit_ray_cylinder(c.p, c.d, rad, te, tx) && fmaxf(te, lo) <= fminf(tx, hi);
        if (vis) {
            if (size <= min_size) { t = fmaxf(te, lo); found = true; break; }
            // Section 3.2: split plane through the centre, normal to the split tangent
            V4 dp, tc;
            split_terms(c, dp, tc);
            float nx = tc.x, ny = tc.y, nz = tc.z;
            if (zero3(nx, ny, nz)) { nx = c.d.x; ny = c.d.y; nz = c.d.z; }
            const float cs = dot3(c.p.x + dp.x, c.p.y + dp.y, c.p.z + dp.z, nx, ny, nz);
            bool right, both;
            if (nz != 0.0f) {
                const float tp = cs / nz;
                right = (tp > te) != (nz > 0.0f);
                both = te < tp && tp < tx;
                if (tp > te) hi = fminf(hi, tp);
                else         lo = fmaxf(lo, tp);
            } else {
                right = cs < 0.0f;      // the whole ray lies on the side of sign(-cs)
                both = cs == 0.0f;
            }
            take_child(c, dp, tc, right);
            size >>= 1;
            if (both) bits ^= size;
            if (right) start ^= size;
            if (COUNT) res.splits++;
        } else {
            if (bits == 0) break;
            // Section 3.3: jump to the deepest level with a pending sibling
            size = bits & (0u - bits);
            start ^= size;
            bits ^= size;
            start &= ~(size - 1u);
            c = root;
            for (uint32_t s = kRootSize >> 1; s >= size; s >>= 1) {
                V4 dp, tc;
                split_terms(c, dp, tc);
                take_child(c, dp, tc, (start & s) != 0u);
            }
            cap_interval(c, tmax, lo, hi);
            if (COUNT) res.backtracks++;
        }
    }

    if (found && t < tmax) {
        const float cc = dot3(c.d.x, c.d.y, c.d.z, c.d.x, c.d.y, c.d.z);
        float ul = 0.0f;
        if (cc > 0.0f) {
            ul = dot3(-c.p.x, -c.p.y, t - c.p.z, c.d.x, c.d.y, c.d.z) / cc;
            ul = fminf(1.0f, fmaxf(0.0f, ul));
        }
        const float u0 = (float)start * 0x1p-23f;
        const float du = (float)size * 0x1p-23f;
        res.t = t;
        res.u = fmaf(ul, du, u0);
        res.hit = true;
        if (COUNT) res.level = 23 - (31 - __builtin_clz(size));
    }
    return res;
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void k_pairs(Args a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n_pairs) return;
    const Result r = trace_pair<COUNT>(a, i);
    a.t_out[i] = r.t;
    a.u_out[i] = r.u;
    a.hit_out[i] = r.hit ? 1 : 0;
    if (COUNT) {
        int32_t *cn = a.counts + 4 * i;
        cn[0] = r.tests;
        cn[1] = r.splits;
        cn[2] = r.backtracks;
        cn[3] = r.level;
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
    if (flags != 0u) return FI_ERR_RANGE;
    if (n_pairs == 0) return FI_OK;
    if (!rays || !fibers || !t_out || !u_out || !hit_out) return FI_ERR_NULL;
    if (ray_stride < n_rays || fiber_stride < n_fibers) return FI_ERR_RANGE;
    if (!pair_ray && n_pairs > n_rays) return FI_ERR_RANGE;
    if (!pair_fiber && n_pairs > n_fibers) return FI_ERR_RANGE;
    if ((n_pairs + kBlock - 1) / kBlock > (int64_t)0x7fffffff) return FI_ERR_RANGE;
    return FI_OK;
}

}  // namespace

extern "C" {

int fi_version(void) { return (0 << 16) | (1 << 8) | 0; }

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

static int launch(bool count, const Args &a, void *stream)
{
    (void)hipGetLastError();
    const unsigned grid = (unsigned)((a.n_pairs + kBlock - 1) / kBlock);
    if (count)
        hipLaunchKernelGGL(k_pairs<true>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_pairs<false>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

int fiber_intersect_pairs(const float *rays, int64_t ray_stride, int64_t n_rays,
                          const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                          const int32_t *pair_ray, const int32_t *pair_fiber,
                          const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                          uint32_t flags,
                          float *t_out, float *u_out, uint8_t *hit_out,
                          void *stream)
{
    const int st = check_common(rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
                                pair_ray, pair_fiber, depth, n_pairs, flags, t_out, u_out, hit_out);
    if (st != FI_OK || n_pairs == 0) return st;
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, nullptr};
    return launch(false, a, stream);
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
    Args a{rays, ray_stride, n_rays, fibers, fiber_stride, n_fibers,
           pair_ray, pair_fiber, pair_depth, depth, n_pairs, t_out, u_out, hit_out, counts_out};
    return launch(true, a, stream);
}

}  // extern "C"
