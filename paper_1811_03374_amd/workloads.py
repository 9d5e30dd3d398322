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
