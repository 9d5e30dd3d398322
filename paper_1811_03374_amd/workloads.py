"""Seeded synthetic ray/fiber workloads.

This module only draws inputs. It holds none of the intersection arithmetic:
no ray frame, no bounding volume, no subdivision. Curve points and tangents
are evaluated here solely to aim rays at fibers.

Layout (structure of arrays, float32, C-contiguous):

* ``rays``   shape (7, n_rays):   rows ox, oy, oz, dx, dy, dz, tmax
* ``fibers`` shape (16, n_fibers): rows p0x, p0y, p0z, p0r, p1x, ..., p3r
  (four cubic Bezier control points; the fourth component of each is the
  radius control value, so the radius is a cubic Bezier too, Section 3.3).
* ``pair_ray`` / ``pair_fiber``: int32 index per pair, or None for the
  identity pairing (pair i uses ray i and fiber i).

Everything is drawn in float64 from ``numpy.random.default_rng`` (PCG64) and
rounded to float32 before any consumer sees it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 1811033740

# Row indices of the SoA layouts.
RAY_ROWS = 7
FIBER_ROWS = 16


@dataclass
class Workload:
    name: str
    rays: np.ndarray                       # (7, n_rays) float32
    fibers: np.ndarray                     # (16, n_fibers) float32
    pair_ray: Optional[np.ndarray] = None  # (n,) int32 or None
    pair_fiber: Optional[np.ndarray] = None
    depth: int = 9
    pair_depth: Optional[np.ndarray] = None  # (n,) uint8 or None
    meta: dict = field(default_factory=dict)

    @property
    def n_pairs(self) -> int:
        if self.pair_ray is not None:
            return int(self.pair_ray.shape[0])
        if self.pair_fiber is not None:
            return int(self.pair_fiber.shape[0])
        return int(min(self.rays.shape[1], self.fibers.shape[1]))

    def with_depth(self, depth: int) -> "Workload":
        return Workload(self.name, self.rays, self.fibers, self.pair_ray,
                        self.pair_fiber, int(depth), None, dict(self.meta))

    def subset(self, idx: np.ndarray) -> "Workload":
        """Pairs ``idx`` of this workload as a self-contained workload."""
        idx = np.asarray(idx, dtype=np.int64)
        ri = self.pair_ray[idx] if self.pair_ray is not None else idx
        fi = self.pair_fiber[idx] if self.pair_fiber is not None else idx
        pd = self.pair_depth[idx] if self.pair_depth is not None else None
        meta = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (self.n_pairs,) else v)
                for k, v in self.meta.items()}
        return Workload(self.name + "[subset]",
                        np.ascontiguousarray(self.rays[:, ri]),
                        np.ascontiguousarray(self.fibers[:, fi]),
                        None, None, self.depth, pd, meta)


# ---------------------------------------------------------------------------
# small sampling helpers (input drawing only)
# ---------------------------------------------------------------------------

def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n directions uniform on the unit sphere, shape (n, 3), float64."""
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def bernstein_point(P: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Point of the cubic Bezier with control points P (n, 4, k) at u (n,)."""
    v = 1.0 - u
    b = np.stack([v ** 3, 3 * u * v * v, 3 * u * u * v, u ** 3], axis=1)
    return np.einsum("nj,njk->nk", b, P)


def bernstein_tangent(P: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Derivative of the cubic Bezier (n, 4, k) at u, shape (n, k)."""
    v = 1.0 - u
    b = np.stack([v * v, 2 * u * v, u * u], axis=1)
    diffs = P[:, 1:, :] - P[:, :-1, :]
    return 3.0 * np.einsum("nj,njk->nk", b, diffs)


def pack_fibers(P: np.ndarray) -> np.ndarray:
    """(n, 4, 4) control points (xyz + radius) -> (16, n) float32 SoA."""
    n = P.shape[0]
    return np.ascontiguousarray(P.reshape(n, 16).T.astype(np.float32))


def unpack_fibers(F: np.ndarray) -> np.ndarray:
    """(16, n) SoA -> (n, 4, 4) float64 control points."""
    return np.ascontiguousarray(F.T.astype(np.float64)).reshape(-1, 4, 4)


def pack_rays(O: np.ndarray, D: np.ndarray, tmax: np.ndarray) -> np.ndarray:
    n = O.shape[0]
    R = np.empty((RAY_ROWS, n), dtype=np.float32)
    R[0:3] = O.T
    R[3:6] = D.T
    R[6] = tmax
    return R


def linear_taper(ra: np.ndarray, rb: np.ndarray) -> np.ndarray:
    """Bezier radius coefficients r_k = ra + (k/3)(rb - ra): r(u) is exactly linear."""
    k = np.arange(4) / 3.0
    return ra[:, None] + k[None, :] * (rb - ra)[:, None]


def _aim_rays(rng, P32: np.ndarray, dist: float, offset_sigma_scale: float):
    """Rays from distance ``dist`` around each fiber's control-point centroid,
    aimed at C(u0) displaced sideways by N(0, (scale*r(u0))^2) along the
    direction perpendicular to both the view vector and the curve tangent
    (about half of the rays hit a locally straight tube)."""
    n = P32.shape[0]
    u0 = rng.uniform(0.0, 1.0, n)
    C = bernstein_point(P32, u0)            # (n, 4): xyz + radius
    T = bernstein_tangent(P32, u0)[:, :3]
    centroid = P32[:, :, :3].mean(axis=1)
    O = centroid + dist * unit_vectors(rng, n)
    view = C[:, :3] - O
    side = np.cross(view, T)
    norm = np.linalg.norm(side, axis=1, keepdims=True)
    bad = norm[:, 0] < 1e-300
    side[bad] = unit_vectors(rng, int(bad.sum()))
    side /= np.maximum(np.linalg.norm(side, axis=1, keepdims=True), 1e-300)
    off = rng.standard_normal(n) * offset_sigma_scale * C[:, 3]
    target = C[:, :3] + off[:, None] * side
    O32 = O.astype(np.float32).astype(np.float64)
    D = target - O32
    return O32, D, u0, off / np.maximum(C[:, 3], 1e-300)


# ---------------------------------------------------------------------------
# Workload 1: plain method, CPU-sized (4,096 rays, 64 fibers, depth 4)
# ---------------------------------------------------------------------------

def plain_unit_cube(n_rays: int = 4096, n_fibers: int = 64, depth: int = 4,
                    seed: int = SEED_BASE + 1) -> Workload:
    """64 fibers with control points uniform in the unit cube and radius linear
    from 0.02 to 0.005; ray i uses fiber i mod 64; origins uniform on the
    sphere of radius 3 about the cube centre; each ray aims at
    C(u0) + N(0, 0.02^2 I) with u0 ~ U[0, 1]; tmax = 100."""
    rng = np.random.default_rng(seed)
    P = np.empty((n_fibers, 4, 4))
    P[:, :, :3] = rng.uniform(0.0, 1.0, (n_fibers, 4, 3))
    P[:, :, 3] = np.array([0.02, 0.015, 0.01, 0.005])[None, :]
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)

    pair_fiber = (np.arange(n_rays) % n_fibers).astype(np.int32)
    Pp = P32[pair_fiber]
    u0 = rng.uniform(0.0, 1.0, n_rays)
    C = bernstein_point(Pp, u0)
    O = np.array([0.5, 0.5, 0.5]) + 3.0 * unit_vectors(rng, n_rays)
    target = C[:, :3] + 0.02 * rng.standard_normal((n_rays, 3))
    O32 = O.astype(np.float32).astype(np.float64)
    D = target - O32
    rays = pack_rays(O32, D, np.full(n_rays, 100.0))
    return Workload("plain_unit_cube_4096x64", rays, fibers,
                    np.arange(n_rays, dtype=np.int32), pair_fiber, depth,
                    meta={"u0": u0})


# ---------------------------------------------------------------------------
# Workload 2: 2^20 ray/segment pairs, half straight, half curved
# ---------------------------------------------------------------------------

def straight_and_curved(n_pairs: int = 1 << 20, depth: int = 9,
                        seed: int = SEED_BASE + 2) -> Workload:
    """Even pairs: straight constant-radius fibers (evenly spaced collinear
    control points, length U[0.05, 0.5], radius U[0.001, 0.01]). Odd pairs:
    curved fibers whose control points are a random walk with step 0.1 and
    whose radius is linear between two values drawn from U[0.001, 0.01].
    Pair i uses ray i and fiber i (identity pairing)."""
    rng = np.random.default_rng(seed)
    n = int(n_pairs)
    P = np.empty((n, 4, 4))
    straight = (np.arange(n) % 2) == 0
    ns = int(straight.sum())
    nc = n - ns
    # straight half
    a = rng.uniform(0.0, 1.0, (ns, 3))
    s = unit_vectors(rng, ns)
    L = rng.uniform(0.05, 0.5, ns)
    k = np.arange(4) / 3.0
    P[straight, :, :3] = a[:, None, :] + (k[None, :, None] * L[:, None, None]) * s[:, None, :]
    r = rng.uniform(0.001, 0.01, ns)
    P[straight, :, 3] = r[:, None]
    # curved half
    p0 = rng.uniform(0.0, 1.0, (nc, 3))
    steps = 0.1 * np.stack([unit_vectors(rng, nc) for _ in range(3)], axis=1)
    walk = np.concatenate([p0[:, None, :], p0[:, None, :] + np.cumsum(steps, axis=1)], axis=1)
    P[~straight, :, :3] = walk
    ra = rng.uniform(0.001, 0.01, nc)
    rb = rng.uniform(0.001, 0.01, nc)
    P[~straight, :, 3] = linear_taper(ra, rb)

    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    O, D, u0, off = _aim_rays(rng, P32, 3.0, 1.4826)
    rays = pack_rays(O, D, np.full(n, 100.0))
    return Workload(f"straight_and_curved_{n}", rays, fibers, None, None, depth,
                    meta={"straight": straight, "u0": u0, "offset_over_r": off})


def exact_straight_fibers(n: int, seed: int = SEED_BASE + 20,
                          cap_fraction: float = 0.25) -> Workload:
    """Straight constant-radius fibers whose four float32 control points are
    exactly collinear and exactly evenly spaced (coordinates on a 2^-12 grid),
    with rays aimed at the side (about half hit) and, for ``cap_fraction`` of
    the rays, along the axis from beyond an end so that they meet an end cap."""
    rng = np.random.default_rng(seed)
    grid = 2.0 ** -12
    p0 = np.round(rng.uniform(0.2, 0.8, (n, 3)) / grid) * grid
    step = np.round(unit_vectors(rng, n) * rng.uniform(0.02, 0.15, (n, 1)) / grid) * grid
    P = np.empty((n, 4, 4))
    for j in range(4):
        P[:, j, :3] = p0 + j * step
    r = rng.uniform(0.005, 0.03, n)
    P[:, :, 3] = r[:, None]
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    O, D, u0, off = _aim_rays(rng, P32, 3.0, 1.4826)
    cap = rng.uniform(0, 1, n) < cap_fraction
    if cap.any():
        A = P32[cap, 0, :3]
        B = P32[cap, 3, :3]
        ax = (B - A) / np.linalg.norm(B - A, axis=1, keepdims=True)
        flip = rng.uniform(0, 1, int(cap.sum())) < 0.5
        start = np.where(flip[:, None], B + 0.7 * ax, A - 0.7 * ax)
        tilt = unit_vectors(rng, int(cap.sum())) * 0.3
        side = tilt - np.sum(tilt * ax, axis=1, keepdims=True) * ax
        rr = P32[cap, 0, 3][:, None]
        Oc = start + side * rr * rng.uniform(0.0, 1.6, (int(cap.sum()), 1)) / 0.3
        Oc32 = Oc.astype(np.float32).astype(np.float64)
        aim = np.where(flip[:, None], A, B)
        Dc = aim + side * rr / 0.3 * rng.uniform(-1.0, 1.0, (int(cap.sum()), 1)) - Oc32
        O[cap] = Oc32
        D[cap] = Dc
    rays = pack_rays(O, D, np.full(n, 100.0))
    return Workload(f"exact_straight_{n}", rays, fibers, None, None, 9,
                    meta={"cap_ray": cap})


def gentle_valid_curves(n: int, seed: int = SEED_BASE + 21,
                        bend: float = 0.08, rmax: float = 0.02) -> Workload:
    """Mildly bent, tapered fibers (control points on a line of length ~0.6
    plus perturbations of size ``bend``), redrawn until they satisfy the five
    cubic constraints of Section 3.4, with rays aimed as for the curved half
    of ``straight_and_curved``."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < n:
        m = 2 * n
        a = rng.uniform(0.2, 0.8, (m, 3))
        s = unit_vectors(rng, m)
        k = np.arange(4) / 3.0
        P = np.empty((m, 4, 4))
        P[:, :, :3] = a[:, None, :] + 0.6 * k[None, :, None] * s[:, None, :]
        P[:, 1:3, :3] += bend * rng.standard_normal((m, 2, 3))
        ra = rng.uniform(0.3, 1.0, m) * rmax
        rb = rng.uniform(0.3, 1.0, m) * rmax
        P[:, :, 3] = linear_taper(ra, rb)
        q = P[:, :, :3]
        ok = np.ones(m, bool)
        for (i, j, k_, l) in ((2, 0, 1, 0), (3, 1, 1, 0), (3, 1, 3, 2), (2, 0, 3, 2), (2, 0, 3, 1)):
            ok &= np.sum((q[:, i] - q[:, j]) * (q[:, k_] - q[:, l]), axis=1) >= 0
        out.append(P[ok])
    P = np.concatenate(out)[:n]
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    O, D, u0, off = _aim_rays(rng, P32, 3.0, 1.4826)
    rays = pack_rays(O, D, np.full(n, 100.0))
    return Workload(f"gentle_valid_{n}", rays, fibers, None, None, 22,
                    meta={"u0": u0, "offset_over_r": off})


# ---------------------------------------------------------------------------
# Workload 3: hair-like precision stress
# ---------------------------------------------------------------------------

def _rotate_towards(v, axis_vec, angle):
    """Rotate unit vectors v by ``angle`` about the unit axes ``axis_vec``."""
    c, s = np.cos(angle)[:, None], np.sin(angle)[:, None]
    return v * c + np.cross(axis_vec, v) * s + axis_vec * np.sum(axis_vec * v, axis=1, keepdims=True) * (1 - c)


def hair_strands(n_strands: int = 100_000, seed: int = SEED_BASE + 3, offset: float = 1000.0,
                 r_root: float = 1e-4, r_tip: float = 2e-5, segments: int = 8):
    """Control points (n_strands * segments, 4, 4) float64 of hair strands:
    knots K_0..K_8 with chord 1/8 (strand length ~1), roots uniform on
    [0,1]^2 x {0}, growth direction a smooth random walk turning at most 20
    degrees per knot; Catmull-Rom tangents (one-sided at the ends) turned into
    C1 cubic Bezier segments; radius linear along the strand from r_root to
    r_tip; every coordinate offset by ``offset`` before rounding to float32."""
    rng = np.random.default_rng(seed)
    n = int(n_strands)
    K = np.empty((n, segments + 1, 3))
    K[:, 0, :2] = rng.uniform(0, 1, (n, 2))
    K[:, 0, 2] = 0.0
    d = unit_vectors(rng, n)
    d[:, 2] = np.abs(d[:, 2]) + 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    step = 1.0 / segments
    for k in range(1, segments + 1):
        K[:, k] = K[:, k - 1] + step * d
        axis = unit_vectors(rng, n)
        axis -= np.sum(axis * d, axis=1, keepdims=True) * d
        axis /= np.linalg.norm(axis, axis=1, keepdims=True)
        d = _rotate_towards(d, axis, np.radians(rng.uniform(0, 20, n)))
    T = np.empty_like(K)
    T[:, 1:-1] = 0.5 * (K[:, 2:] - K[:, :-2])
    T[:, 0] = K[:, 1] - K[:, 0]
    T[:, -1] = K[:, -1] - K[:, -2]
    P = np.empty((n, segments, 4, 4))
    P[:, :, 0, :3] = K[:, :-1]
    P[:, :, 1, :3] = K[:, :-1] + T[:, :-1] / 3
    P[:, :, 2, :3] = K[:, 1:] - T[:, 1:] / 3
    P[:, :, 3, :3] = K[:, 1:]
    s0 = np.arange(segments) / segments
    r0 = r_root + (r_tip - r_root) * s0
    r1 = r_root + (r_tip - r_root) * (s0 + 1.0 / segments)
    P[:, :, :, 3] = (r0[:, None] + (np.arange(4) / 3.0)[None, :] * (r1 - r0)[:, None])[None]
    P[:, :, :, :3] += offset
    return P.reshape(n * segments, 4, 4)


def hair_precision(n_rays: int = 1 << 24, n_strands: int = 100_000, depth: int = 9,
                   seed: int = SEED_BASE + 3, grazing_fraction: float = 0.1,
                   rho: float = 0.25, chunk: int = 1 << 21, graze_width: float = 1e-3,
                   targets: Optional[np.ndarray] = None, strands: Optional[np.ndarray] = None) -> Workload:
    """Rays aimed at uniformly chosen hair segments and parameters u0, from
    C(u0) + rho * s (s uniform on the sphere, rho = 0.25): 90 % regular rays
    displaced sideways by N(0, (1.4826 r)^2), 10 % grazing rays displaced by
    (1 + delta) r with delta ~ U[-w, w] (w = graze_width, 1e-3 by default),
    both along the direction
    normal to the view vector and the tangent. The origin is rounded to
    float32 first, then D = target - O is formed in float64 and rounded.
    Pairs are (ray i, its target segment) through pair_fiber. ``targets``
    (and ``strands``, the float32-exact control points of the table) aim the
    rays at given segments instead of uniformly chosen ones."""
    if strands is None:
        P = hair_strands(n_strands, seed)
        fibers = pack_fibers(P)
        P32 = unpack_fibers(fibers)
    else:
        P32 = strands
        fibers = pack_fibers(P32)
    rng = np.random.default_rng(seed + 7)
    n = int(n_rays)
    seg = rng.integers(0, P32.shape[0], n).astype(np.int32) if targets is None else targets
    rays = np.empty((RAY_ROWS, n), np.float32)
    graze = np.zeros(n, bool)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        m = b - a
        Pp = P32[seg[a:b]]
        u0 = rng.uniform(0, 1, m)
        C = bernstein_point(Pp, u0)
        Tg = bernstein_tangent(Pp, u0)[:, :3]
        O = C[:, :3] + rho * unit_vectors(rng, m)
        O32 = O.astype(np.float32).astype(np.float64)
        view = C[:, :3] - O32
        side = np.cross(view, Tg)
        side /= np.maximum(np.linalg.norm(side, axis=1, keepdims=True), 1e-300)
        g = rng.uniform(0, 1, m) < grazing_fraction
        off = rng.standard_normal(m) * 1.4826
        sign = np.where(rng.uniform(0, 1, m) < 0.5, -1.0, 1.0)
        off = np.where(g, sign * (1.0 + rng.uniform(-graze_width, graze_width, m)), off) * C[:, 3]
        target = C[:, :3] + off[:, None] * side
        D = target - O32
        rays[0:3, a:b] = O32.T
        rays[3:6, a:b] = D.T
        rays[6, a:b] = 100.0
        graze[a:b] = g
    return Workload(f"hair_{n}", rays, fibers, None, seg, depth, meta={"grazing": graze})


def hair_candidates(n_rays: int = 1 << 20, n_strands: int = 100_000, depth: int = 22,
                    seed: int = SEED_BASE + 6, chunk: int = 1 << 20) -> Workload:
    """Candidate lists of a hierarchy leaf per ray over the hair table of
    ``hair_strands``: each ray is aimed as in ``hair_precision`` (90 %
    regular, 10 % grazing) at segment j of strand a; its candidates are
    segments j-1 .. j+1 of strand a and of 1 to 4 other strands whose roots
    lie in the same or a neighbouring cell of a 64 x 64 grid over the root
    square (strands that cross the same region), 6 to 15 segments in all, in
    random order (a leaf's order is not sorted by distance). Offsets (CSR,
    int64) and candidate fibers (int32) are in ``meta`` as ``cand_off`` and
    ``cand_fiber``; ``meta["target"]`` is the aimed segment."""
    segments = 8
    P = hair_strands(n_strands, SEED_BASE + 3)
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    rng = np.random.default_rng(seed)
    n = int(n_rays)
    n_str = P32.shape[0] // segments
    roots = P32[::segments, 0, :2] - 1000.0
    g = 64
    cell = np.clip((roots * g).astype(np.int64), 0, g - 1)
    cid = cell[:, 0] * g + cell[:, 1]
    order = np.argsort(cid, kind="stable")
    start = np.searchsorted(cid[order], np.arange(g * g + 1))
    strand = rng.integers(0, n_str, n)
    j = rng.integers(0, segments, n)
    target = (strand * segments + j).astype(np.int32)
    n_other = rng.integers(1, 5, n)
    # strands: the aimed one, then up to 4 from the same or a neighbouring
    # root cell (a cell may be empty: that strand is dropped)
    st = np.empty((n, 5), np.int64)
    have = np.zeros((n, 5), bool)
    st[:, 0] = strand
    have[:, 0] = True
    cx, cy = cell[strand, 0], cell[strand, 1]
    for k in range(1, 5):
        ox = np.clip(cx + rng.integers(-1, 2, n), 0, g - 1)
        oy = np.clip(cy + rng.integers(-1, 2, n), 0, g - 1)
        c = ox * g + oy
        size = start[c + 1] - start[c]
        pick = start[c] + (rng.random(n) * np.maximum(size, 1)).astype(np.int64)
        st[:, k] = order[np.minimum(pick, len(order) - 1)]
        have[:, k] = (k <= n_other) & (size > 0)
    # segments j - 1 .. j + 1 of each strand, inside the strand
    jj = j[:, None, None] + np.array([-1, 0, 1])[None, None, :]
    segs = (st[:, :, None] * segments + jj).reshape(n, 15)
    mask = (have[:, :, None] & (jj >= 0) & (jj < segments)).reshape(n, 15)
    # each list in random order
    keys = np.where(mask, rng.random((n, 15)), 2.0)
    perm = np.argsort(keys, axis=1)
    segs = np.take_along_axis(segs, perm, axis=1)
    counts = mask.sum(axis=1).astype(np.int64)
    keep = np.arange(15)[None, :] < counts[:, None]
    off = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    cand = segs[keep].astype(np.int32)
    aim = hair_precision(n, n_strands, depth, seed=seed + 1, chunk=chunk, targets=target, strands=P32)
    return Workload(f"hair_candidates_{n}", aim.rays, fibers, None, None, depth,
                    meta={"cand_off": off, "cand_fiber": cand, "target": target,
                          "grazing": aim.meta["grazing"]})


def elevate_quadratic(P3: np.ndarray) -> np.ndarray:
    """(n, 3, 4) quadratic control points -> (n, 4, 4) exact cubic elevation
    (float64): the same curve and radius function."""
    P3 = np.asarray(P3, np.float64)
    out = np.empty((P3.shape[0], 4, 4))
    out[:, 0] = P3[:, 0]
    out[:, 1] = (P3[:, 0] + 2.0 * P3[:, 1]) / 3.0
    out[:, 2] = (2.0 * P3[:, 1] + P3[:, 2]) / 3.0
    out[:, 3] = P3[:, 2]
    return out


def pack_quadratics(P3: np.ndarray) -> np.ndarray:
    """(n, 3, 4) -> (12, n) float32 table (rows p0x, p0y, p0z, p0r, .., p2r)."""
    return np.ascontiguousarray(np.asarray(P3).reshape(-1, 12).T.astype(np.float32))


def unpack_quadratics(table: np.ndarray) -> np.ndarray:
    return np.asarray(table, np.float64).T.reshape(-1, 3, 4)


def quadratic_fibers(n: int, seed: int = SEED_BASE + 8, straight_fraction: float = 0.25) -> Workload:
    """Quadratic Bezier fibers (Appendix B.1): chord of length 0.2..0.8 in a
    random direction from a point of the unit cube, the middle control point
    at the chord's centre displaced sideways by up to 0.45 of the chord (a
    quarter of the fibers straight: the middle point exactly at the centre,
    on a 2^-12 grid), radius tapering linearly between 0.002 and 0.02; rays
    aimed as in ``straight_and_curved`` (about half hit)."""
    rng = np.random.default_rng(seed)
    grid = 2.0 ** -12
    p0 = np.round(rng.uniform(0.1, 0.9, (n, 3)) / grid) * grid
    ch = np.round(unit_vectors(rng, n) * rng.uniform(0.2, 0.8, (n, 1)) / (2 * grid)) * (2 * grid)
    side = unit_vectors(rng, n)
    side -= np.sum(side * ch, axis=1, keepdims=True) * ch / np.sum(ch * ch, axis=1, keepdims=True)
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    bend = rng.uniform(0.0, 0.45, n) * np.linalg.norm(ch, axis=1)
    straight = rng.uniform(0, 1, n) < straight_fraction
    bend[straight] = 0.0
    P = np.empty((n, 3, 4))
    P[:, 0, :3] = p0
    P[:, 1, :3] = p0 + 0.5 * ch + bend[:, None] * side
    P[:, 2, :3] = p0 + ch
    ra = rng.uniform(0.002, 0.02, n)
    rb = rng.uniform(0.002, 0.02, n)
    P[:, :, 3] = ra[:, None] + np.array([0.0, 0.5, 1.0])[None, :] * (rb - ra)[:, None]
    fibers = pack_quadratics(P)
    P32 = unpack_quadratics(fibers)
    O, D, u0, off = _aim_rays(rng, elevate_quadratic(P32), 3.0, 1.4826)
    rays = pack_rays(O, D, np.full(n, 100.0))
    return Workload(f"quadratic_{n}", rays, fibers, None, None, 9,
                    meta={"straight": straight, "u0": u0, "offset_over_r": off})


# ---------------------------------------------------------------------------
# Workload 4: batched uneven scenes with per-segment adaptive depth
# ---------------------------------------------------------------------------

def adaptive_depth(P: np.ndarray, samples: int = 65, chunk: int = 1 << 14) -> np.ndarray:
    """d = clamp(ceil(log2(kappa * len / r)), 2, 22) per curve: kappa is the
    largest curvature |C' x C''| / |C'|^3 over ``samples`` parameters, len the
    length of the polyline through those samples, r the smallest radius
    coefficient (kappa = 0 gives depth 2). Evaluated in float32."""
    u = np.linspace(0, 1, samples, dtype=np.float32)[None, :]
    out = np.empty(P.shape[0], np.uint8)
    for s0 in range(0, P.shape[0], chunk):
        Q = P[s0:s0 + chunk, :, :3].astype(np.float32)
        a1 = 3 * (Q[:, 1] - Q[:, 0])
        a2 = 3 * (Q[:, 2] - 2 * Q[:, 1] + Q[:, 0])
        a3 = Q[:, 3] - 3 * Q[:, 2] + 3 * Q[:, 1] - Q[:, 0]
        X, T, S = [], [], []
        for c in range(3):
            A0, A1, A2, A3 = (Q[:, 0, c][:, None], a1[:, c][:, None], a2[:, c][:, None], a3[:, c][:, None])
            X.append(A0 + u * (A1 + u * (A2 + u * A3)))
            T.append(A1 + u * (2 * A2 + 3 * u * A3))
            S.append(2 * A2 + 6 * u * A3)
        seg = np.sqrt(sum(np.diff(x, axis=1) ** 2 for x in X))
        length = seg.sum(axis=1)
        cx = T[1] * S[2] - T[2] * S[1]
        cy = T[2] * S[0] - T[0] * S[2]
        cz = T[0] * S[1] - T[1] * S[0]
        num = np.sqrt(cx * cx + cy * cy + cz * cz)
        t2 = T[0] * T[0] + T[1] * T[1] + T[2] * T[2]
        den = t2 * np.sqrt(t2)
        kappa = np.max(np.where(den > 0, num / np.maximum(den, 1e-30), 0.0), axis=1).astype(np.float64)
        r = np.maximum(P[s0:s0 + chunk, :, 3].min(axis=1), 1e-30)
        with np.errstate(divide="ignore"):
            d = np.ceil(np.log2(np.maximum(kappa * length / r, 1e-300)))
        d = np.where(kappa > 0, d, 2)
        out[s0:s0 + chunk] = np.clip(d, 2, 22)
    return out


def curved_scene(n_pairs: int, seed: int) -> Workload:
    """One scene: curved random-walk fibers (step 0.1, linear taper in
    [0.001, 0.01]) with rays aimed as in ``straight_and_curved``, identity
    pairing, per-pair adaptive depth."""
    rng = np.random.default_rng(seed)
    n = int(n_pairs)
    P = np.empty((n, 4, 4))
    p0 = rng.uniform(0.0, 1.0, (n, 3))
    steps = 0.1 * np.stack([unit_vectors(rng, n) for _ in range(3)], axis=1)
    P[:, :, :3] = np.concatenate([p0[:, None, :], p0[:, None, :] + np.cumsum(steps, axis=1)], axis=1)
    P[:, :, 3] = linear_taper(rng.uniform(0.001, 0.01, n), rng.uniform(0.001, 0.01, n))
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    O, D, u0, off = _aim_rays(rng, P32, 3.0, 1.4826)
    rays = pack_rays(O, D, np.full(n, 100.0))
    return Workload(f"scene_{seed}", rays, fibers, None, None, 22, adaptive_depth(P32))


def batched_scenes(n_scenes: int = 256, seed: int = SEED_BASE + 4,
                   lo_log2: float = 10.0, hi_log2: float = 18.0):
    """``n_scenes`` independent scenes with round(2^U(10, 18)) pairs each
    (seed + 1000 s for scene s)."""
    rng = np.random.default_rng(seed)
    counts = np.round(2.0 ** rng.uniform(lo_log2, hi_log2, n_scenes)).astype(np.int64)
    return [curved_scene(int(c), seed + 1000 * s) for s, c in enumerate(counts)]


# ---------------------------------------------------------------------------
# Workload 5: degenerate geometry
# ---------------------------------------------------------------------------

def _random_rotations(rng, n):
    """n uniformly random rotation matrices (n, 3, 3)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], axis=1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], axis=1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], axis=1),
    ], axis=1)


def degenerate_geometry(n_pairs: int = 1 << 22, seed: int = SEED_BASE + 5,
                        depth_lo: int = 16, depth_hi: int = 22) -> Workload:
    """Four families of equal size: (0) cusps, p1 and p2 mirrored so that
    C'(1/2) = 0; (1) evenly spaced collinear points jittered by 1e-6 N(0, I);
    (2) zero-length end tangents (p1 = p0 and/or p2 = p3) on random walks;
    (3) radius ratios up to 1000:1. Half of the rays run along the chord (from
    one unit before an end, offset sideways by U[0, 1.5 r_max], so many enter
    through an end cap); the other half cross it perpendicularly. A quarter of
    all rays use an exactly axis-aligned chord (no rotation) with an exactly
    axis-aligned direction, so that plane normals and axes meet the ray frame
    with exact zeros. Depth is uniform in [depth_lo, depth_hi] per pair."""
    rng = np.random.default_rng(seed)
    n = int(n_pairs)
    fam = np.arange(n) % 4
    P = np.empty((n, 4, 4))
    # family 0: cusp in the xy-plane, chord along x
    L = rng.uniform(0.1, 1.0, n)
    h = rng.uniform(0.05, 0.5, n) * L
    z = np.zeros(n)
    cusp = np.stack([np.stack([z, z, z], 1), np.stack([L, h, z], 1), np.stack([z, h, z], 1),
                     np.stack([L, z, z], 1)], axis=1)
    # family 1: near-collinear along x
    k = np.arange(4)[None, :, None] / 3.0
    col = k * np.stack([L, z, z], 1)[:, None, :] + 1e-6 * rng.standard_normal((n, 4, 3))
    # family 2: random walk with zero end tangents, chord re-aligned to x
    steps = 0.1 * rng.standard_normal((n, 3, 3)) / np.sqrt(3)
    walk = np.concatenate([np.zeros((n, 1, 3)), np.cumsum(steps, axis=1)], axis=1)
    which = rng.integers(0, 3, n)
    zt = walk.copy()
    zt[which != 1, 1] = zt[which != 1, 0]
    zt[which != 0, 2] = zt[which != 0, 3]
    # family 3: gentle curve with a steep taper
    gent = k * np.stack([L, z, z], 1)[:, None, :]
    gent[:, 1:3, 1] += rng.uniform(-0.1, 0.1, (n, 2)) * L[:, None]
    shapes = np.where((fam == 0)[:, None, None], cusp,
             np.where((fam == 1)[:, None, None], col,
             np.where((fam == 2)[:, None, None], zt, gent)))
    # radii
    rmax = rng.uniform(0.001, 0.05, n)
    rho = np.exp(rng.uniform(0, np.log(1000.0), n))
    r_lin = linear_taper(rmax, rmax / rho)
    r_flat = np.repeat(rng.uniform(0.001, 0.02, n)[:, None], 4, axis=1)
    radii = np.where((fam == 3)[:, None], r_lin, r_flat)
    # placement: a quarter of the pairs keep the exact axis-aligned chord
    exact = (np.arange(n) // 4) % 4 == 0
    Rm = _random_rotations(rng, n)
    Rm[exact] = np.eye(3)
    shift = np.where(exact[:, None], np.round(rng.uniform(0, 1, (n, 3)) * 64) / 64,
                     rng.uniform(0, 1, (n, 3)))
    P[:, :, :3] = np.einsum("nij,nkj->nki", Rm, shapes) + shift[:, None, :]
    P[:, :, 3] = radii
    fibers = pack_fibers(P)
    P32 = unpack_fibers(fibers)
    # rays
    parallel = rng.uniform(0, 1, n) < 0.5
    chord = P32[:, 3, :3] - P32[:, 0, :3]
    clen = np.linalg.norm(chord, axis=1)
    chat = chord / np.maximum(clen, 1e-300)[:, None]
    flip = rng.uniform(0, 1, n) < 0.5
    side = unit_vectors(rng, n)
    side -= np.sum(side * chat, axis=1, keepdims=True) * chat
    side /= np.maximum(np.linalg.norm(side, axis=1, keepdims=True), 1e-300)
    rmx = P32[:, :, 3].max(axis=1)
    # parallel: from one unit before an end, along +/- chord
    start = np.where(flip[:, None], P32[:, 3, :3] + chat, P32[:, 0, :3] - chat)
    O_par = start + side * (rng.uniform(0, 1.5, n) * rmx)[:, None]
    D_par = np.where(flip[:, None], -chat, chat)
    # perpendicular: aimed at C(u0) from 3 units away along a direction normal to the chord
    u0 = rng.uniform(0, 1, n)
    C = bernstein_point(P32, u0)
    perp = np.cross(chat, side)
    off = rng.standard_normal(n) * 1.4826 * C[:, 3]
    target = C[:, :3] + off[:, None] * side
    O_perp = target + 3.0 * perp
    D_perp = -perp
    # exact axis-aligned cases: chord along x, direction exactly +-z or +-x
    ex_par = exact & parallel
    ex_perp = exact & ~parallel
    D_par[ex_par] = np.where(flip[ex_par, None], [-1.0, 0.0, 0.0], [1.0, 0.0, 0.0])
    D_perp[ex_perp] = [0.0, 0.0, -1.0]
    O_perp[ex_perp] = np.stack([target[ex_perp, 0], target[ex_perp, 1], target[ex_perp, 2] + 3.0], axis=1)
    O = np.where(parallel[:, None], O_par, O_perp)
    D = np.where(parallel[:, None], D_par, D_perp)
    O32 = O.astype(np.float32).astype(np.float64)
    D = np.where(exact[:, None], D, D + (O - O32) * 0)   # directions are exact unit axes where exact
    rays = pack_rays(O32, D, np.full(n, 100.0))
    pd = rng.integers(depth_lo, depth_hi + 1, n).astype(np.uint8)
    return Workload(f"degenerate_{n}", rays, fibers, None, None, depth_hi, pd,
                    meta={"family": fam, "parallel": parallel, "exact_axes": exact})
