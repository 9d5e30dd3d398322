// Fiber validation and pre-subdivision (Section 3.4) for gfx950.
//
// The paper's method needs curves whose recursive halves are separated by
// their split planes (the five inequalities of Section 3.4, proved in
// Appendix B.2) and whose swept solid does not reach across a cap plane
// (Section 3.4, the thick-fiber configuration of Fig. "EvilConfiguration").
// Curves that fail must be split beforehand. These kernels run before the
// per-pair test: one lane per fiber, all arithmetic in FP64 (a pass over
// the fiber table, far from any hot loop).
//
// Cap-plane excess (reading R17): the disc at u (centre C(u), radius r(u),
// normal C'(u)) reaches furthest along a cap normal n at C(u) + r(u) m(u),
// m the unit component of n normal to C'(u) (Gram-Schmidt), i.e. r(u) sin
// of the angle between C'(u) and n beyond its centre. The excess over the
// start plane is r sin - <C(u) - p0, n0>, over the end plane r sin -
// <p3 - C(u), n1>; n0, n1 are the cap normals (the end tangents, or the
// next control-polygon edge, then the chord, where a tangent is negligible).
// A fiber is thick at an end when its largest excess exceeds 1e-9 of its
// extent (|p3 - p0| plus the largest radius value). The largest excess is
// searched on 105 parameters -- 63 evenly spaced, 20 packed geometrically
// towards each end (u = 2^-j and 1 - 2^-j, j = 7, 9, .., 45, where the excess
// shrinks with the distance to the end) and the two ends -- followed by a
// golden-section search in the bracket of the best sample.
//
// Pre-subdivision: a fiber is halved by de Casteljau's construction at
// u = 1/2 (4-D, radius included), depth first and left half first, until a
// piece is valid or max_level halvings deep. Each node is rebuilt from the
// fiber by replaying the halvings along its path (at most max_level of
// them), so a lane keeps no stack; the halving is exact in FP64 for the
// levels allowed here, so every piece is the exact sub-curve rounded once to
// float32.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

#include "fiberhit.h"

namespace {

constexpr int kMaxSplitLevel = 10;

struct Q16 {
    double v[16];                       // p0..p3, each x, y, z, r
};

__device__ __forceinline__ void load_fiber(const float *F, int64_t fs, int64_t i, Q16 &q)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) q.v[k] = (double)F[k * fs + i];
}

__device__ __forceinline__ double d3(double ax, double ay, double az, double bx, double by, double bz)
{
    return ax * bx + ay * by + az * bz;
}

// the five inequalities of Section 3.4: bit k set when inequality k fails
__device__ __forceinline__ int constraint_bits(const Q16 &q)
{
    const double *p = q.v;
    auto dd = [&](int a, int b, int c, int e) {        // <p_a - p_b, p_c - p_e>
        return d3(p[4 * a] - p[4 * b], p[4 * a + 1] - p[4 * b + 1], p[4 * a + 2] - p[4 * b + 2],
                  p[4 * c] - p[4 * e], p[4 * c + 1] - p[4 * e + 1], p[4 * c + 2] - p[4 * e + 2]);
    };
    int m = 0;
    if (!(dd(2, 0, 1, 0) >= 0.0)) m |= 1;
    if (!(dd(3, 1, 1, 0) >= 0.0)) m |= 2;
    if (!(dd(3, 1, 3, 2) >= 0.0)) m |= 4;
    if (!(dd(2, 0, 3, 2) >= 0.0)) m |= 8;
    if (!(dd(2, 0, 3, 1) >= 0.0)) m |= 16;
    return m;
}

// unit cap normal at the start (end = false) or end
__device__ __forceinline__ void cap_normal(const Q16 &q, bool end, double n[3])
{
    const double *p = q.v;
    const double ax = p[12] - p[0], ay = p[13] - p[1], az = p[14] - p[2];
    const double lim = 0x1p-40 * d3(ax, ay, az, ax, ay, az);
    // first non-negligible of (p1 - p0, p2 - p0, p3 - p0) / (p3 - p2, p3 - p1, p3 - p0)
    const int a0 = end ? 3 : 1, b0 = end ? 2 : 0;
    const int a1 = end ? 3 : 2, b1 = end ? 1 : 0;
    double x = p[4 * a0] - p[4 * b0], y = p[4 * a0 + 1] - p[4 * b0 + 1], z = p[4 * a0 + 2] - p[4 * b0 + 2];
    if (d3(x, y, z, x, y, z) <= lim) {
        x = p[4 * a1] - p[4 * b1]; y = p[4 * a1 + 1] - p[4 * b1 + 1]; z = p[4 * a1 + 2] - p[4 * b1 + 2];
    }
    if (d3(x, y, z, x, y, z) <= lim) { x = ax; y = ay; z = az; }
    const double il = 1.0 / sqrt(d3(x, y, z, x, y, z));
    n[0] = x * il; n[1] = y * il; n[2] = z * il;
}

// excess of the disc at u over a cap plane (-inf where C'(u) vanishes)
__device__ __forceinline__ double disc_excess(const Q16 &q, bool end, const double n[3], double u)
{
    const double *p = q.v;
    const double v = 1.0 - u;
    const double b0 = v * v * v, b1 = 3.0 * u * v * v, b2 = 3.0 * u * u * v, b3 = u * u * u;
    const double e0 = v * v, e1 = 2.0 * u * v, e2 = u * u;
    double C[4], D[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) C[k] = b0 * p[k] + b1 * p[4 + k] + b2 * p[8 + k] + b3 * p[12 + k];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        D[k] = e0 * (p[4 + k] - p[k]) + e1 * (p[8 + k] - p[4 + k]) + e2 * (p[12 + k] - p[8 + k]);
    const double dl2 = d3(D[0], D[1], D[2], D[0], D[1], D[2]);
    if (!(dl2 > 0.0)) return -INFINITY;
    const double cx = D[1] * n[2] - D[2] * n[1], cy = D[2] * n[0] - D[0] * n[2], cz = D[0] * n[1] - D[1] * n[0];
    const double s = sqrt(d3(cx, cy, cz, cx, cy, cz) / dl2);
    const double along = end ? d3(p[12] - C[0], p[13] - C[1], p[14] - C[2], n[0], n[1], n[2])
                             : d3(C[0] - p[0], C[1] - p[1], C[2] - p[2], n[0], n[1], n[2]);
    return C[3] * s - along;
}

constexpr int kSamples = 105;

// the k-th search parameter, increasing in k (see the file comment)
__device__ __forceinline__ double sample_u(int k)
{
    if (k <= 0) return 0.0;
    if (k <= 20) return ldexp(1.0, -45 + 2 * (k - 1));            // 2^-45 .. 2^-7
    if (k <= 83) return (double)(k - 20) / 64.0;                  // 1/64 .. 63/64
    if (k <= 103) return 1.0 - ldexp(1.0, -7 - 2 * (k - 84));      // 1 - 2^-7 .. 1 - 2^-45
    return 1.0;
}

__device__ double largest_excess(const Q16 &q, bool end)
{
    double n[3];
    cap_normal(q, end, n);
    double best = -INFINITY;
    int kb = 0;
    for (int k = 0; k < kSamples; ++k) {
        const double h = disc_excess(q, end, n, sample_u(k));
        if (h > best) { best = h; kb = k; }
    }
    // golden-section search in the bracket of the best sample
    constexpr double g = 0.38196601125010515;
    double a = sample_u(kb - 1), b = sample_u(kb + 1 < kSamples ? kb + 1 : kSamples - 1);
    double x1 = a + g * (b - a), x2 = b - g * (b - a);
    double f1 = disc_excess(q, end, n, x1), f2 = disc_excess(q, end, n, x2);
    for (int it = 0; it < 60; ++it) {
        if (f1 > f2) { b = x2; x2 = x1; f2 = f1; x1 = a + g * (b - a); f1 = disc_excess(q, end, n, x1); }
        else         { a = x1; x1 = x2; f1 = f2; x2 = b - g * (b - a); f2 = disc_excess(q, end, n, x2); }
    }
    return fmax(best, fmax(f1, f2));
}

// validity mask (0: valid): bits 0-4 inequalities, 5 thick at the start,
// 6 thick at the end, 7 non-finite; excesses relative to the extent
__device__ int fiber_mask(const Q16 &q, float *ex0, float *ex1)
{
    for (int k = 0; k < 16; ++k)
        if (!isfinite(q.v[k])) {
            *ex0 = *ex1 = __builtin_nanf("");
            return 1 << 7;
        }
    int m = constraint_bits(q);
    const double *p = q.v;
    double rmax = fmax(fmax(fabs(p[3]), fabs(p[7])), fmax(fabs(p[11]), fabs(p[15])));
    const double ax = p[12] - p[0], ay = p[13] - p[1], az = p[14] - p[2];
    const double X = sqrt(d3(ax, ay, az, ax, ay, az)) + rmax;
    const double e0 = largest_excess(q, false) / X, e1 = largest_excess(q, true) / X;
    if (e0 > 1e-9) m |= 1 << 5;
    if (e1 > 1e-9) m |= 1 << 6;
    *ex0 = (float)e0;
    *ex1 = (float)e1;
    return m;
}

__device__ __forceinline__ void halve(Q16 &q, bool right)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double a = q.v[c], b = q.v[4 + c], d = q.v[8 + c], e = q.v[12 + c];
        const double m01 = (a + b) * 0.5, m12 = (b + d) * 0.5, m23 = (d + e) * 0.5;
        const double m012 = (m01 + m12) * 0.5, m123 = (m12 + m23) * 0.5;
        const double s = (m012 + m123) * 0.5;
        q.v[c] = right ? s : a;
        q.v[4 + c] = right ? m123 : m01;
        q.v[8 + c] = right ? m23 : m012;
        q.v[12 + c] = right ? e : s;
    }
}

// the node (level, index) of fiber i, replayed from the fiber
__device__ __forceinline__ void node_of(const float *F, int64_t fs, int64_t i, int level, uint32_t index, Q16 &q)
{
    load_fiber(F, fs, i, q);
    for (int l = level - 1; l >= 0; --l) halve(q, ((index >> l) & 1u) != 0u);
}

// Does node q become a piece (emitted), and its mask: a node below the
// level limit that fails an inequality is halved whatever its cap-plane
// excesses, so they are only searched where they decide (the inequalities
// hold) or where the piece's mask is wanted (`leaf_mask`).
__device__ __forceinline__ bool piece_decision(const Q16 &q, int level, int max_level, bool leaf_mask, int &m)
{
    for (int k = 0; k < 16; ++k)
        if (!isfinite(q.v[k])) {
            m = 1 << 7;
            return true;
        }
    const int ineq = constraint_bits(q);
    if (level >= max_level && !leaf_mask) {
        m = ineq;
        return true;
    }
    if (level < max_level && ineq != 0) {
        m = ineq;
        return false;
    }
    float e0, e1;
    m = fiber_mask(q, &e0, &e1);
    return m == 0 || level >= max_level;
}

// Depth-first walk over the pieces of fiber i: `emit(level, index, q, mask)`
// for every piece in order; returns their number. LEAF_MASK: the pieces'
// masks are wanted (else a piece at the level limit may carry its
// inequality bits only).
template <bool LEAF_MASK, class Emit>
__device__ int64_t walk_pieces(const float *F, int64_t fs, int64_t i, int max_level, Emit emit)
{
    int level = 0;
    uint32_t index = 0;
    int64_t count = 0;
    for (;;) {
        Q16 q;
        node_of(F, fs, i, level, index, q);
        int m;
        if (piece_decision(q, level, max_level, LEAF_MASK, m)) {
            emit(level, index, q, m, count);
            ++count;
            // next node in depth-first order: climb while this is a right child
            while (level > 0 && (index & 1u)) { index >>= 1; --level; }
            if (level == 0) break;
            index += 1;                 // the right sibling
        } else {
            ++level;                    // the left child
            index <<= 1;
        }
    }
    return count;
}

__global__ __launch_bounds__(256) void k_validate(const float *F, int64_t fs, int64_t n, int32_t *mask,
                                                  float *excess)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    Q16 q;
    load_fiber(F, fs, i, q);
    float e0, e1;
    mask[i] = fiber_mask(q, &e0, &e1);
    if (excess) {
        excess[2 * i] = e0;
        excess[2 * i + 1] = e1;
    }
}

__global__ __launch_bounds__(256) void k_presplit_count(const float *F, int64_t fs, int64_t n, int max_level,
                                                        int64_t *counts)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > n) return;
    if (i == n) {                       // the exclusive scan's total lands at index n
        counts[n] = 0;
        return;
    }
    counts[i] = walk_pieces<false>(F, fs, i, max_level, [](int, uint32_t, const Q16 &, int, int64_t) {});
}

__global__ __launch_bounds__(256) void k_presplit_write(const float *F, int64_t fs, int64_t n, int max_level,
                                                        const int64_t *offsets, int64_t n_pieces, float *P,
                                                        int64_t ps, int32_t *pfiber, float *pu0, float *pu1,
                                                        int32_t *pmask)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t base = offsets[i];
    walk_pieces<true>(F, fs, i, max_level, [&](int level, uint32_t index, const Q16 &q, int m, int64_t k) {
        const int64_t j = base + k;
        if (j < 0 || j >= n_pieces) return;
        for (int c = 0; c < 16; ++c) P[c * ps + j] = (float)q.v[c];
        const float w = ldexpf(1.0f, -level);
        pfiber[j] = (int32_t)i;
        pu0[j] = (float)index * w;
        pu1[j] = (float)(index + 1u) * w;
        pmask[j] = m;
    });
}

size_t scan_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int64_t *)nullptr, (int64_t *)nullptr,
                                         (int)(n + 1)) != hipSuccess)
        return 0;
    return bytes;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int fiber_validate(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t *mask_out,
                   float *excess_out, void *stream)
{
    if (n_fibers < 0 || fiber_stride < n_fibers) return FI_ERR_RANGE;
    if (n_fibers == 0) return FI_OK;
    if (!fibers || !mask_out) return FI_ERR_NULL;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((n_fibers + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       fibers, fiber_stride, n_fibers, mask_out, excess_out);
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

size_t fiber_presplit_workspace_bytes(int64_t n_fibers)
{
    if (n_fibers < 0 || n_fibers > (int64_t)0x7ffffffe) return 0;
    return align256((size_t)(n_fibers + 1) * sizeof(int64_t)) + align256(scan_temp_bytes(n_fibers));
}

int fiber_presplit_count(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t max_level,
                         int64_t *offsets_out, void *workspace, size_t workspace_bytes, void *stream)
{
    if (n_fibers < 0 || fiber_stride < n_fibers || n_fibers > (int64_t)0x7ffffffe) return FI_ERR_RANGE;
    if (max_level < 0 || max_level > kMaxSplitLevel) return FI_ERR_RANGE;
    if (!offsets_out) return FI_ERR_NULL;
    if (n_fibers > 0 && !fibers) return FI_ERR_NULL;
    const size_t need = fiber_presplit_workspace_bytes(n_fibers);
    if (!workspace || ((uintptr_t)workspace & 255u) != 0u || workspace_bytes < need) return FI_ERR_WORKSPACE;
    const hipStream_t s = (hipStream_t)stream;
    int64_t *counts = (int64_t *)workspace;
    void *temp = (char *)workspace + align256((size_t)(n_fibers + 1) * sizeof(int64_t));
    size_t temp_bytes = need - align256((size_t)(n_fibers + 1) * sizeof(int64_t));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_presplit_count, dim3((unsigned)((n_fibers + 1 + 255) / 256)), dim3(256), 0, s, fibers,
                       fiber_stride, n_fibers, max_level, counts);
    if (hipGetLastError() != hipSuccess) return FI_ERR_HIP;
    if (hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, counts, offsets_out, (int)(n_fibers + 1), s) !=
        hipSuccess)
        return FI_ERR_HIP;
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

int fiber_presplit(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t max_level,
                   const int64_t *offsets, int64_t n_pieces, float *pieces_out, int64_t piece_stride,
                   int32_t *piece_fiber, float *piece_u0, float *piece_u1, int32_t *piece_mask, void *stream)
{
    if (n_fibers < 0 || fiber_stride < n_fibers || n_pieces < 0 || piece_stride < n_pieces) return FI_ERR_RANGE;
    if (max_level < 0 || max_level > kMaxSplitLevel) return FI_ERR_RANGE;
    if (n_fibers == 0) return FI_OK;
    if (!fibers || !offsets || !pieces_out || !piece_fiber || !piece_u0 || !piece_u1 || !piece_mask)
        return FI_ERR_NULL;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_presplit_write, dim3((unsigned)((n_fibers + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, fibers, fiber_stride, n_fibers, max_level, offsets, n_pieces,
                       pieces_out, piece_stride, piece_fiber, piece_u0, piece_u1, piece_mask);
    return hipGetLastError() == hipSuccess ? FI_OK : FI_ERR_HIP;
}

}  // extern "C"
