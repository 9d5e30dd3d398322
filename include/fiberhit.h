/*
 * fiberhit -- ray/fiber intersection on AMD MI355X (gfx950), C ABI.
 *
 * The method is Binder & Keller, "Fast, High Precision Ray/Fiber Intersection
 * using Tight, Disjoint Bounding Volumes" (arXiv 1811.03374): a fiber is a
 * cubic Bezier curve whose control points carry a radius (Section 3.3); the
 * test moves it into the frame of the ray (Section 3.3), then subdivides it
 * at the parametric centre down to depth d inside bounding cylinders that are
 * cropped by end-cap and split planes (Sections 3.1-3.3), visiting the half
 * that the ray meets first and stopping at the first leaf hit (Section 3).
 *
 * Every function returns an int status (FI_OK or a negative FI_ERR_*) and
 * throws nothing. All array arguments are caller-owned device pointers (for
 * example the data of torch tensors); the library only reads inputs and writes
 * outputs. Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 * the legacy default stream); results are valid once the stream has
 * synchronised.
 *
 * Every call (and every batch) runs one persistent kernel: each 64-lane wave
 * takes an even share of the pairs, prepares them in rounds of up to 64 (load,
 * FP64 move into the ray frame, root test; pairs decided at the root are
 * written out at once) into a queue in LDS, from which each lane takes its
 * next pair as soon as it is free; a lane keeps its pair's root in registers
 * for the subdivision search. The library allocates nothing while a call
 * runs. The only device memory a call needs beyond its inputs and outputs is
 * a copy of the fibers as 64-byte records for calls that gather fibers
 * through an index, in a workspace the caller sizes with
 * fiber_pairs_workspace_bytes; a batch needs its scene table, in a workspace
 * sized by fiber_batched_workspace_bytes, or inside a plan. Device set-up
 * (unit counts, occupancy, pinned staging of batched scene tables) happens
 * once per device, at fi_init_device or at the first call on that device.
 *
 * Layouts (structure of arrays, 32-bit floats, row-major):
 *   rays   : 7 rows of ray_stride floats  -- ox, oy, oz, dx, dy, dz, tmax.
 *            The direction need not be unit length: the library normalises
 *            it, and t and tmax are distances along the normalised direction.
 *   fibers : 16 rows of fiber_stride floats -- p0x, p0y, p0z, p0r, p1x, ...,
 *            p3r: four control points, each with its radius control value.
 *
 * Per-pair data that make a pair meaningless (a zero, infinite or NaN
 * direction, a NaN tmax, an index outside its array, a per-pair depth above
 * 23) are not errors: that pair is reported as a miss.
 */
#ifndef FIBERHIT_H
#define FIBERHIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FI_OK             0
#define FI_ERR_NULL      (-1)   /* a required pointer is NULL                         */
#define FI_ERR_RANGE     (-2)   /* a count, stride or depth is out of range           */
#define FI_ERR_HIP       (-3)   /* the HIP runtime reported an error at launch        */
#define FI_ERR_WORKSPACE (-4)   /* workspace pointer missing, misaligned or too small */
#define FI_ERR_SCRATCH   (-5)   /* more scratch than the no-allocation entry point holds */
#define FI_ERR_IO        (-6)   /* a tuning table file could not be opened or written  */

/* Flags. */
/* FI_FP64_REFINE: for pairs of depth > 16, run the traversal with every
 * pruning test enlarged by a bound on its FP32 rounding error and, once it
 * reaches a leaf, decide the pair against the swept-disc solid in FP64 (see
 * fiber_intersect_pairs). */
#define FI_FP64_REFINE   (1u << 0)
/* FI_COMPENSATED_PROJ: accepted and always in effect. The move into the ray
 * frame (Section 3.3) runs in FP64 from exact differences of the float32
 * inputs, so every root coordinate is the correctly rounded float32 of its
 * exact value -- at least as accurate as compensated FP32 products. The
 * per-pair work counts (node tests, splits, backtracks, leaf level) that a
 * statistics flag would add are the separate entry point
 * fiber_intersect_counts. */
#define FI_COMPENSATED_PROJ (1u << 1)
/* FI_QUADRATIC: the fiber table holds quadratic Bezier curves (Appendix B.1;
 * 12 rows: p0x, p0y, p0z, p0r, p1x, .., p2r). Each is traversed as its exact
 * cubic elevation (q1 = (p0 + 2 p1) / 3, q2 = (2 p1 + p2) / 3: the same
 * curve and radius function; de Casteljau halving commutes with elevation,
 * so the halves, split planes -- normal to the chord at a quadratic's centre
 * -- and cap planes are the quadratic's), bounded by the quadratic's own
 * conservative radius (the middle control point's distance to the chord
 * plus the largest of the three radius values). Refined pairs search the
 * quadratic's swept solid. Accepted by fiber_intersect_pairs, its
 * no-allocation variant and fiber_intersect_counts (not by batched or
 * candidate-list calls: FI_ERR_RANGE); such calls use no workspace. The
 * quadratic's constraint <p1 - p0, p1 - p2> <= 0 keeps every split
 * separating (Appendix B.1). */
#define FI_QUADRATIC (1u << 2)

/* Largest subdivision depth: one bit per level in 32-bit integers and an
 * integer parametric position below 2^23 (Section 3.3, interval conversion). */
#define FI_MAX_DEPTH 23

/* Library version, (major << 16) | (minor << 8) | patch. */
int fi_version(void);

/* Static English text for a status code. */
const char *fi_strerror(int status);

/* Set-up of the current device: unit counts, the occupancy of every kernel
 * variant and the pinned host buffers that stage batched scene tables.
 * Every entry point does this on its first call on a device; callers that
 * must not allocate during later calls run it once beforehand. FI_OK or
 * FI_ERR_HIP. */
int fi_init_device(void);

/* Bytes of device workspace one fiber_intersect_pairs or
 * fiber_intersect_counts call of n_pairs pairs over a table of n_fibers
 * fibers can use: when gathered is non-zero (pair_fiber given) and
 * n_pairs >= n_fibers, the fibers' 64-byte records (tables up to 1 GiB);
 * otherwise 0. A call with a smaller workspace (or none) reads the fiber rows
 * in place, with the same results. flags is reserved. */
size_t fiber_pairs_workspace_bytes(int64_t n_pairs, int64_t n_fibers, int32_t gathered, uint32_t flags);

/*
 * fiber_intersect_pairs -- nearest hit of each (ray, fiber) pair at depth d.
 *
 * Operation: the per-pair routine of the paper's intersection code
 * (Appendix C, final listing; Sections 3.2 and 3.3), iterated with one bit
 * per subdivision level. For pair i it intersects ray pair_ray[i] with fiber
 * pair_fiber[i] and reports the first leaf cylinder the ray enters at
 * subdivision depth pair_depth[i] (or `depth`): t is the entry into the
 * capped leaf cylinder, u is the curve parameter of the hit point projected
 * onto the leaf chord (Section 3.3, last paragraph), hit is 1 when
 * 0 <= t < tmax. Degenerate tangents: a tangent whose squared length is at
 * most 2^-40 of the squared chord counts as zero (its cap plane falls back
 * to the next control-polygon edge; a zero split tangent is a cusp, where
 * the split plane is normal to the chord), and a node that holds an end of
 * the curve whose extent (largest squared length of chord and end
 * tangents) is at most (2^-20 X)^2 (X the largest ray-frame coordinate of
 * the control points) and at most 2^-16 of the root's extent times
 * 4^-level is a leaf before the depth (a stalled end, where the curve's
 * speed vanishes and further halving resolves only rounding).
 *
 * Arguments:
 *   rays, ray_stride, n_rays       ray table (see layout), ray_stride >= n_rays.
 *   fibers, fiber_stride, n_fibers fiber table (see layout), fiber_stride >= n_fibers.
 *   pair_ray, pair_fiber           int32 index per pair, or NULL for the identity
 *                                  pairing (then n_pairs must not exceed n_rays,
 *                                  respectively n_fibers).
 *   pair_depth                     uint8 depth per pair, or NULL to use `depth`.
 *   depth                          0 .. FI_MAX_DEPTH (checked even when pair_depth
 *                                  is given).
 *   n_pairs                        >= 0; 0 enqueues nothing and returns FI_OK.
 *   flags                          FI_FP64_REFINE, FI_COMPENSATED_PROJ,
 *                                  FI_QUADRATIC (12-row fiber table).
 *   t_out, u_out, hit_out          n_pairs each. On a miss: t = +inf, u = NaN, hit = 0.
 *   t64_out, u64_out               n_pairs doubles each; required with
 *                                  FI_FP64_REFINE, ignored (may be NULL) without.
 *   normal_out                     3 * n_pairs floats (rows x, y, z, each of
 *                                  n_pairs: normal_out[k * n_pairs + i]), or NULL
 *                                  for none: the unit outward normal at each hit
 *                                  in world space (see Normals); NaN on a miss.
 *   workspace, workspace_bytes     caller-owned device memory, 256-byte aligned,
 *                                  for the fiber records of a gathered call
 *                                  (size: fiber_pairs_workspace_bytes), or NULL
 *                                  and 0. It must not be used by another call
 *                                  still in flight; its contents on entry do not
 *                                  matter.
 *   stream                         hipStream_t or NULL.
 *
 * FI_FP64_REFINE: the method's leaf cylinders converge to the solid swept by
 * a disc of radius r(u) centred on C(u) in the plane normal to C'(u), closed by
 * the end discs (Section 3.2: the limit surface maps the intersection to the
 * closest point on the curve). For each pair of depth > 16 the search runs
 * with every pruning test enlarged by a bound on its FP32 rounding, so that
 * no leaf holding part of that solid is pruned; a pair whose search reaches
 * no leaf misses. Once it reaches a leaf, the pair is decided in FP64: the
 * first point of that solid along the ray, t in [0, tmax), over the whole
 * curve (boundary points from Newton's method on <P - C(u), C'(u)> = 0,
 * |P - C(u)| = r(u) started at the FP32 leaf hit, from 64 samples of the
 * disc excess with a bracketed root search at sign changes and a bracketed
 * minimisation at local minima, the end discs, t = 0 for an origin inside).
 * All five outputs then describe that point (hit decided in FP64; hit = 0,
 * t = +inf when there is none). Pairs of depth
 * <= 16 keep the plain method's results; their t64/u64 are the float results
 * widened.
 *
 * Normals (Appendix C, the final computation of an intersection; FP32 in the
 * ray frame, turned back into world space with the ray's frame rebuilt in
 * FP64): a hit that enters its leaf through the cylinder's side (or through
 * an inner split plane) gets the direction from the leaf chord's point at the
 * hit's projection to the hit point; a hit that enters through the curve's
 * start (end) cap plane gets minus the start tangent (the end tangent), with
 * the cap plane's fallbacks where that tangent vanishes. Which plane bounded
 * the entry decides, not a clamped u. A refined pair (depth > 16 under
 * FI_FP64_REFINE) gets the normal of the swept solid at its FP64 hit,
 * computed in FP64: on the side the direction from C(u) to the hit, tilted
 * against the tangent by the taper r'(u) (with the curvature term of the
 * turning disc); at an end disc its outward normal; NaN with the origin
 * inside (t = 0). The normal's rows are written only when normal_out is not
 * NULL; the other results do not depend on it.
 *
 * Errors: FI_ERR_NULL when rays, fibers or an output is NULL with n_pairs > 0
 * (t64_out/u64_out only with FI_FP64_REFINE); FI_ERR_RANGE for negative
 * counts, strides below the counts, a depth outside [0, 23], unknown flags,
 * an identity pairing longer than its ray or fiber table, or
 * n_pairs >= 2^31 - 64;
 * FI_ERR_WORKSPACE when the workspace is not 256-byte aligned; FI_ERR_HIP
 * when the launch fails or the device set-up fails. Nothing is enqueued on an argument error. The call
 * allocates, frees and waits for nothing.
 */
int fiber_intersect_pairs(const float *rays, int64_t ray_stride, int64_t n_rays,
                          const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                          const int32_t *pair_ray, const int32_t *pair_fiber,
                          const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                          uint32_t flags,
                          float *t_out, float *u_out, uint8_t *hit_out,
                          double *t64_out, double *u64_out, float *normal_out,
                          void *workspace, size_t workspace_bytes, void *stream);

/*
 * fiber_intersect_pairs_noalloc -- fiber_intersect_pairs without a workspace,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).
 *
 * Operation and arguments: those of fiber_intersect_pairs, minus the
 * workspace; the results are bit for bit the same. The fiber records of a
 * gathered call (pair_fiber given, n_pairs >= n_fibers) go to a fixed array
 * inside the library's code object (32 MiB, one copy per device, held until
 * the process ends; its address is taken once per device at the device's
 * set-up), which holds the records of up to 524,288 fibers: such a call over
 * a larger fiber table is refused with FI_ERR_SCRATCH before anything is
 * enqueued. Other calls use no scratch.
 *
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (a call writes the records it reads first, so nothing needs
 * clearing): gathered calls that overlap on one device -- on two streams, or
 * from two host threads without ordering -- race and give undefined results.
 *
 * Allocation: none on the call path (no hipMalloc, hipFree or allocating
 * library routine). The device's set-up (fi_init_device, or the first call of
 * any entry point on that device) allocates the pinned staging of batched
 * calls once; callers that must not allocate at all call fi_init_device
 * beforehand.
 *
 * Errors: as fiber_intersect_pairs, without FI_ERR_WORKSPACE; FI_ERR_SCRATCH
 * as above.
 */
int fiber_intersect_pairs_noalloc(const float *rays, int64_t ray_stride, int64_t n_rays,
                                  const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                                  const int32_t *pair_ray, const int32_t *pair_fiber,
                                  const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                                  uint32_t flags,
                                  float *t_out, float *u_out, uint8_t *hit_out,
                                  double *t64_out, double *u64_out, float *normal_out,
                                  void *stream);

/*
 * fiber_intersect_counts -- the traversal of fiber_intersect_pairs with its
 * work counted instead of timed.
 *
 * Operation: the same per-pair search (same arguments and meaning as
 * fiber_intersect_pairs), which in addition writes four int32 per pair to
 * counts_out[4*i .. 4*i+3]: node tests (pruning tests of Section 3.2, one per
 * loop trip), splits (descents), backtracks (Section 3.3, jumps to a pending
 * sibling) and the level of the leaf that was hit (-1 on a miss). These are
 * the units of the algorithmic work model.
 *
 * Errors: as fiber_intersect_pairs; counts_out must not be NULL and
 * FI_FP64_REFINE is not accepted. The workspace is sized as for
 * fiber_intersect_pairs.
 */
int fiber_intersect_counts(const float *rays, int64_t ray_stride, int64_t n_rays,
                           const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                           const int32_t *pair_ray, const int32_t *pair_fiber,
                           const uint8_t *pair_depth, int32_t depth, int64_t n_pairs,
                           uint32_t flags,
                           float *t_out, float *u_out, uint8_t *hit_out,
                           int32_t *counts_out, void *workspace, size_t workspace_bytes,
                           void *stream);

/* ------------------------------------------------------------------------ */
/* Nearest hit over candidate lists                                         */
/* ------------------------------------------------------------------------ */

/* Bytes of device workspace fiber_intersect_candidates can use: the fiber
 * records (64 bytes per fiber, 256-byte aligned) when the lists hold at
 * least as many candidates as the table has fibers, else 0. */
size_t fiber_candidates_workspace_bytes(int64_t n_candidates, int64_t n_fibers, uint32_t flags);

/*
 * fiber_intersect_candidates -- nearest hit of each ray over its candidate
 * list.
 *
 * Operation: the interface a renderer's top-level hierarchy calls (Sec. 1
 * and Sec. 4 place the method below such a hierarchy: the fibers referenced
 * by the leaves a ray reaches are tested one after another, and a hit
 * shortens the ray for the fibers after it). Ray r's candidates are
 * cand_fiber[cand_offsets[r]] .. cand_fiber[cand_offsets[r + 1] - 1]; each is
 * tested with the per-pair routine of fiber_intersect_pairs at depth
 * cand_depth[k] (or `depth`), against the ray's tmax until a hit and against
 * the latest hit's t after it. A hit counts when its t lies below that
 * limit, so of equal hits the first in the list is kept. The outputs
 * describe the kept hit: t, u, hit and the normal as for
 * fiber_intersect_pairs, and fiber_out the index of its fiber (-1 when no
 * candidate is hit). With FI_FP64_REFINE, candidates of depth > 16 are
 * decided in FP64 as there, against the FP64 nearest hit so far.
 *
 * Arguments: the ray and fiber tables as for fiber_intersect_pairs;
 * cand_offsets: n_rays + 1 non-decreasing int64 (CSR), cand_offsets[0] >= 0,
 * cand_offsets[n_rays] <= n_candidates; cand_fiber: n_candidates int32 fiber
 * indices (an index outside the table is a candidate that misses);
 * cand_depth: n_candidates uint8 depths, or NULL to use `depth`;
 * max_candidates: the number of list positions tested -- at least the
 * longest list; a longer list is tested on its first max_candidates entries
 * only; outputs: n_rays entries each (normal_out: three rows of n_rays, or
 * NULL); workspace as for fiber_intersect_pairs (size:
 * fiber_candidates_workspace_bytes), or NULL.
 *
 * Implementation: an initialising kernel writes misses, then one persistent
 * launch per list position k (max_candidates launches in stream order), each
 * testing every ray's k-th candidate against the nearest hit of positions
 * before k and writing only hits.
 *
 * Errors: FI_ERR_NULL (rays, fibers, cand_offsets or an output NULL with
 * n_rays > 0; cand_fiber NULL with n_candidates > 0; t64_out/u64_out under
 * FI_FP64_REFINE), FI_ERR_RANGE (negative counts, strides below the counts,
 * depth outside [0, 23], unknown flags, n_rays >= 2^31 - 64),
 * FI_ERR_WORKSPACE (misaligned), FI_ERR_HIP. Nothing is enqueued on an
 * argument error; the call allocates, frees and waits for nothing.
 */
int fiber_intersect_candidates(const float *rays, int64_t ray_stride, int64_t n_rays,
                               const float *fibers, int64_t fiber_stride, int64_t n_fibers,
                               const int64_t *cand_offsets, const int32_t *cand_fiber,
                               const uint8_t *cand_depth, int32_t depth, int32_t max_candidates,
                               int64_t n_candidates, uint32_t flags,
                               float *t_out, float *u_out, uint8_t *hit_out, int32_t *fiber_out,
                               double *t64_out, double *u64_out, float *normal_out,
                               void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Validation and pre-subdivision of fibers (before the per-pair test)       */
/* ------------------------------------------------------------------------ */

/*
 * fiber_validate -- which fibers the method handles as they are.
 *
 * Operation (Section 3.4): a fiber is valid when the five inequalities
 * <p2-p0, p1-p0>, <p3-p1, p1-p0>, <p3-p1, p3-p2>, <p2-p0, p3-p2>,
 * <p2-p0, p3-p1> >= 0 hold (recursive halves are then separated by their
 * split planes, Appendix B.2) and no disc of its swept solid reaches across
 * the start or end cap plane (Fig. "EvilConfiguration": the disc at u reaches
 * r(u) sin(angle(C'(u), n)) beyond its centre along the cap normal n, by
 * Gram-Schmidt; the fiber is thick at that end when the largest excess over
 * the plane exceeds 1e-9 of its extent |p3 - p0| + max radius). Computed in
 * FP64, the excess searched on 105 parameters (63 even, 20 packed towards
 * each end) and refined by golden section around the best one.
 *
 * Arguments: the fiber table (16 rows of fiber_stride floats, as for
 * fiber_intersect_pairs); mask_out: n_fibers int32, 0 for a valid fiber,
 * else bit k (0..4) for a failed inequality, bit 5 thick at the start, bit 6
 * thick at the end, bit 7 a non-finite control point; excess_out: NULL or
 * 2 * n_fibers floats, the largest start and end excesses relative to the
 * extent. Errors: FI_ERR_RANGE, FI_ERR_NULL, FI_ERR_HIP; allocates nothing.
 */
int fiber_validate(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t *mask_out,
                   float *excess_out, void *stream);

/* Bytes of workspace fiber_presplit_count needs for n_fibers fibers (0 for
 * a negative count or more than 2^31 - 2 fibers). */
size_t fiber_presplit_workspace_bytes(int64_t n_fibers);

/*
 * fiber_presplit_count, fiber_presplit -- split invalid fibers beforehand.
 *
 * Operation (Section 3.4: curves that break the constraints, thick ends,
 * cusps "require subdivision beforehand"): each fiber is halved by de
 * Casteljau's construction at u = 1/2 (Appendix B.2; radius included),
 * depth first and left half first, until a piece is valid in the sense of
 * fiber_validate or max_level halvings deep (0..10; a piece stopped by the
 * limit keeps its nonzero mask). A valid fiber is its own single piece.
 * The halving is exact in FP64 at these levels; pieces are rounded to
 * float32 once.
 *
 * fiber_presplit_count writes offsets_out (n_fibers + 1 int64): fiber i's
 * pieces occupy [offsets_out[i], offsets_out[i + 1]), offsets_out[n_fibers]
 * is the total. It needs a workspace of fiber_presplit_workspace_bytes
 * (256-byte aligned). The caller reads the total, sizes the piece table and
 * calls fiber_presplit with the same fibers, max_level and those offsets: it
 * writes the pieces (a fiber table of 16 rows of piece_stride floats,
 * piece_stride >= n_pieces), and per piece its fiber, its parameter interval
 * [piece_u0, piece_u1) on that fiber (a hit at piece parameter v lies at
 * u0 + v (u1 - u0) on the fiber) and its validity mask.
 *
 * Errors: FI_ERR_RANGE (counts, strides, max_level), FI_ERR_NULL,
 * FI_ERR_WORKSPACE, FI_ERR_HIP. Neither call allocates.
 */
int fiber_presplit_count(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t max_level,
                         int64_t *offsets_out, void *workspace, size_t workspace_bytes, void *stream);
int fiber_presplit(const float *fibers, int64_t fiber_stride, int64_t n_fibers, int32_t max_level,
                   const int64_t *offsets, int64_t n_pieces, float *pieces_out, int64_t piece_stride,
                   int32_t *piece_fiber, float *piece_u0, float *piece_u1, int32_t *piece_mask, void *stream);

/* ------------------------------------------------------------------------ */
/* Many independent problems in one launch                                  */
/* ------------------------------------------------------------------------ */

/* One problem: the arguments of one fiber_intersect_pairs call (the flags
 * are the batch's). All pointers are device pointers owned by the caller;
 * t64_out and u64_out are read only when the batch runs with
 * FI_FP64_REFINE; normal_out may be NULL (no normals for that problem). */
typedef struct fi_scene {
    const float *rays;   int64_t ray_stride;   int64_t n_rays;
    const float *fibers; int64_t fiber_stride; int64_t n_fibers;
    const int32_t *pair_ray; const int32_t *pair_fiber; const uint8_t *pair_depth;
    int32_t depth;       int64_t n_pairs;
    float *t_out; float *u_out; uint8_t *hit_out;
    double *t64_out; double *u64_out;
    float *normal_out;
} fi_scene;

/* Launch tuning of the batched kernel (not part of the method):
 *   refill          free lanes take queued pairs once at least this many
 *                   (1..64) are free (default 1);
 *   waves_per_simd  waves of the grid per SIMD (0..16; 0 = as many as fit,
 *                   which is 4 for the batched kernel; fewer leave slots
 *                   free, more are started by the dispatcher as resident
 *                   waves end, each wave with an equal share of the pairs);
 *   stack           layout of the traversal stack (Section 3.3 keeps only the
 *                   bit string): 0 (default) caches the parent of the latest
 *                   split that left a sibling pending in LDS, so the usual
 *                   backtrack rebuilds that sibling with one split; 1 keeps
 *                   no cache, and every backtrack replays the split rules
 *                   from the root.
 * Results never depend on the tuning. */
typedef struct fi_tuning {
    int32_t refill;
    int32_t waves_per_simd;
    int32_t stack;
} fi_tuning;

/* Bytes of device workspace fiber_intersect_batched needs for n_scenes
 * problems of total_pairs pairs in all (0 for negative arguments): the scene
 * table and the pair offsets (about 140 bytes per scene); it does not grow
 * with total_pairs. */
size_t fiber_batched_workspace_bytes(int32_t n_scenes, int64_t total_pairs);

/*
 * fiber_intersect_batched -- all pairs of n_scenes independent problems in
 * one persistent launch.
 *
 * Operation: for every scene k, exactly what fiber_intersect_pairs computes
 * for scenes[k] (same per-pair routine; results are bitwise identical to a
 * separate call per scene). Pairs of all scenes are numbered consecutively
 * and one persistent launch covers them all (each wave an even share), so
 * small scenes do not leave the GPU idle.
 *
 * Arguments: scenes is a host array of n_scenes descriptors (the library
 * copies it before returning); tuning may be NULL (the autotuned entry of
 * this batch's size class if fiber_batch_autotune ran, else defaults);
 * flags: FI_FP64_REFINE (every scene then needs t64_out and u64_out; the
 * per-pair meaning is that of fiber_intersect_pairs with that flag) and/or
 * FI_COMPENSATED_PROJ;
 * workspace is caller-owned device memory, 256-byte aligned, of at least
 * fiber_batched_workspace_bytes(n_scenes, total pairs) bytes, which must not
 * be used by another call that is still in flight. The call allocates
 * nothing; it waits (rarely) for the upload of the scene table four batched
 * calls earlier to leave its pinned staging buffer.
 *
 * Errors: FI_ERR_NULL (scenes NULL or a NULL pointer inside a scene, t64_out
 * or u64_out included under FI_FP64_REFINE),
 * FI_ERR_RANGE (bad counts, strides, depths, tuning, flags, more than 2^31-64
 * pairs in total or a scene table over 1 MiB), FI_ERR_WORKSPACE, FI_ERR_HIP.
 */
int fiber_intersect_batched(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Plans: the scene table is uploaded once into device memory the plan owns,
 * and the launch (one kernel) is captured into a HIP
 * graph that fiber_batch_plan_launch replays on any stream. Scenes, tuning
 * and flags mean what they mean for fiber_intersect_batched. Creating and
 * destroying a plan allocates and frees device memory; launching does not.
 * One plan must not be launched on two streams at once. The scenes' device
 * buffers must outlive the plan.
 */
typedef struct fi_batch_plan fi_batch_plan;

int fiber_batch_plan_create(const fi_scene *scenes, int32_t n_scenes, const fi_tuning *tuning,
                            uint32_t flags, fi_batch_plan **plan_out);
int fiber_batch_plan_launch(fi_batch_plan *plan, void *stream);
int fiber_batch_plan_tuning(const fi_batch_plan *plan, fi_tuning *tuning_out);
int fiber_batch_plan_destroy(fi_batch_plan *plan);

/*
 * fiber_batch_autotune -- time fiber_intersect_batched on these scenes over a
 * grid of tunings (refill 32, 48 or 56, with FI_FP64_REFINE 4, 8 or 16;
 * waves per SIMD as many as fit, 8 or 16; stack 0 or 1), each `repeats`
 * times after one warm-up, and return the fastest
 * in *best (and its time in *best_ms if not NULL). Overwrites the scenes'
 * outputs. Blocks the host until the timing runs finish. The result is also
 * remembered in the process's tuning table, keyed by the current device's
 * architecture name (e.g. "gfx950"), the refinement flag and the batch's
 * class: floor(log2) of its total pairs, floor(log2) of its problem count
 * and the bucket of its largest scene depth field (0: <= 9, 1: <= 16,
 * 2: deeper). Later batched calls and plans of that class that pass
 * tuning = NULL use it.
 */
int fiber_batch_autotune(const fi_scene *scenes, int32_t n_scenes, uint32_t flags, void *workspace,
                         size_t workspace_bytes, void *stream, int32_t repeats,
                         fi_tuning *best, float *best_ms);

/*
 * The tuning table across processes (host only; no GPU needed).
 *
 * fiber_tuning_save -- write every entry of the process's tuning table to the
 * text file at path (created or replaced): the line "fiberhit-tuning 1", then
 * one line per entry, "arch refine log2_pairs log2_scenes depth_bucket refill
 * waves_per_simd stack". FI_ERR_NULL, FI_ERR_IO.
 *
 * fiber_tuning_load -- merge the entries of such a file into the table
 * (entries of the same key are replaced). A file with a bad header, a
 * malformed line or a value out of range merges nothing: FI_ERR_RANGE.
 * FI_ERR_NULL, FI_ERR_IO (cannot open).
 *
 * fiber_tuning_lookup -- the table's entry for a batch of n_scenes problems
 * (>= 1) with total_pairs pairs (>= 0) and largest depth max_depth (0..23)
 * under flags (FI_FP64_REFINE selects the refined entries) on architecture
 * arch: FI_OK and *out, or FI_ERR_RANGE when there is none (or an argument
 * is out of range). FI_ERR_NULL.
 *
 * fiber_tuning_clear -- empty the table. FI_OK.
 */
int fiber_tuning_save(const char *path);
int fiber_tuning_load(const char *path);
int fiber_tuning_lookup(const char *arch, uint32_t flags, int64_t total_pairs, int32_t n_scenes,
                        int32_t max_depth, fi_tuning *out);
int fiber_tuning_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* FIBERHIT_H */
