"""Pins of the exact swept-disc oracle (CPU only)."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W
from test_oracle_pins import (bezier, bezier_d, brute_force, capped_cylinder,
                              unpack_rays)


def test_straight_fibers_equal_capped_cylinder_all_kinds():
    w = W.exact_straight_fibers(1500)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    r = P[:, 0, 3]
    t_cf, u_cf, h_cf = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r, tmax)
    _, _, h_lo = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r * (1 - 1e-7), tmax)
    _, _, h_hi = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r * (1 + 1e-7), tmax)
    stable = h_lo == h_hi
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers)
    assert np.array_equal(h.astype(bool)[stable], h_cf[stable])
    assert {1, 2, 3} <= set(np.unique(kind[h.astype(bool)]))
    b = stable & h_cf & h.astype(bool)
    assert np.max(np.abs(t[b] - t_cf[b]) / t_cf[b]) < 1e-11
    assert np.abs(u[b] - u_cf[b]).max() < 1e-10


def test_exact_not_later_than_sampled_discs():
    w = W.gentle_valid_curves(400)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t_bf, u_bf, h_bf = brute_force(P, O, D, tmax)
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers)
    assert np.array_equal(h.astype(bool), h_bf)
    b = h.astype(bool)
    rel = (t[b] - t_bf[b]) / t_bf[b]
    assert rel.max() <= 1e-12 and rel.min() > -1e-7
    assert np.abs(u[b] - u_bf[b]).max() < 1e-4


def test_side_hits_are_on_the_circle_in_the_normal_plane():
    w = W.gentle_valid_curves(400, seed=7)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers)
    sel = kind == 1
    assert sel.sum() > 100
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    X = O[sel] + t[sel, None] * Dn[sel]
    C = bezier(P[sel], u[sel, None])[:, 0]
    T = bezier_d(P[sel], u[sel, None])[:, 0, :3]
    dist = np.linalg.norm(X - C[:, :3], axis=1)
    assert np.abs(dist - C[:, 3]).max() < 1e-12
    assert np.abs(np.sum((X - C[:, :3]) * T, axis=1)).max() < 1e-12
    # cap hits: on the end disc
    for kk, ue in ((2, 0.0), (3, 1.0)):
        s = kind == kk
        if s.any():
            Xc = O[s] + t[s, None] * Dn[s]
            Cc = bezier(P[s], np.full((s.sum(), 1), ue))[:, 0]
            assert np.all(np.linalg.norm(Xc - Cc[:, :3], axis=1) <= Cc[:, 3] * (1 + 1e-12))


def _mp_exact(ray, fib, dps=50):
    """First entry from an independent route: the ray frame in 50-digit
    arithmetic, F in the power basis, mpmath.polyroots, caps checked directly."""
    mpmath.mp.dps = dps
    O = [mpmath.mpf(float(x)) for x in ray[:3]]
    Dv = [mpmath.mpf(float(x)) for x in ray[3:6]]
    L = mpmath.sqrt(sum(x * x for x in Dv))
    w = [x / L for x in Dv]
    # any orthonormal completion: Gram-Schmidt against the least aligned axis
    k = int(np.argmin([abs(float(x)) for x in w]))
    e = [mpmath.mpf(0)] * 3
    e[k] = mpmath.mpf(1)
    dot = sum(a * b for a, b in zip(e, w))
    uvec = [a - dot * b for a, b in zip(e, w)]
    un = mpmath.sqrt(sum(x * x for x in uvec))
    uvec = [x / un for x in uvec]
    vvec = [w[1] * uvec[2] - w[2] * uvec[1], w[2] * uvec[0] - w[0] * uvec[2],
            w[0] * uvec[1] - w[1] * uvec[0]]
    q = []
    for j in range(4):
        p = [mpmath.mpf(float(fib[4 * j + c])) - O[c] for c in range(3)]
        q.append([sum(a * b for a, b in zip(p, uvec)), sum(a * b for a, b in zip(p, vvec)),
                  sum(a * b for a, b in zip(p, w)), mpmath.mpf(float(fib[4 * j + 3]))])
    # power-basis coefficients (highest first) of each channel
    def power(c):
        a0, a1, a2, a3 = c
        return [-a0 + 3 * a1 - 3 * a2 + a3, 3 * a0 - 6 * a1 + 3 * a2, -3 * a0 + 3 * a1, a0]
    Cp = [power([q[j][c] for j in range(4)]) for c in range(4)]
    Dp = [mpmath.polyval if False else None for _ in range(3)]
    def deriv(p):
        n = len(p) - 1
        return [p[i] * (n - i) for i in range(n)]
    Dp = [deriv(Cp[c]) for c in range(3)]
    def mul(a, b):
        r = [mpmath.mpf(0)] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                r[i + j] += x * y
        return r
    def add(a, b, s=1):
        n = max(len(a), len(b))
        a = [mpmath.mpf(0)] * (n - len(a)) + a
        b = [mpmath.mpf(0)] * (n - len(b)) + b
        return [x + s * y for x, y in zip(a, b)]
    Dz2 = mul(Dp[2], Dp[2])
    xy = add(mul(Cp[0], Dp[0]), mul(Cp[1], Dp[1]))
    F = add(add(mul(Dz2, add(mul(Cp[0], Cp[0]), mul(Cp[1], Cp[1]))), mul(xy, xy)),
            mul(mul(Cp[3], Cp[3]), Dz2), -1)
    while abs(F[0]) == 0:
        F = F[1:]
    roots = mpmath.polyroots(F, maxsteps=400, extraprec=200)
    best = (math.inf, None)
    def cand(uu):
        C = [mpmath.polyval(Cp[c], uu) for c in range(4)]
        Dd = [mpmath.polyval(Dp[c], uu) for c in range(3)]
        if Dd[2] == 0:
            return None
        return (C[0] * Dd[0] + C[1] * Dd[1] + C[2] * Dd[2]) / Dd[2], C, Dd
    for rt in roots:
        if abs(mpmath.im(rt)) > mpmath.mpf(10) ** -25:
            continue
        uu = mpmath.re(rt)
        if uu < 0 or uu > 1:
            continue
        c = cand(uu)
        if c and 0 <= c[0] < ray[6] and c[0] < best[0]:
            best = (c[0], uu)
    for ue in (mpmath.mpf(0), mpmath.mpf(1)):
        c = cand(ue)
        if c is None:
            continue
        t, C, Dd = c
        rad2 = C[0] ** 2 + C[1] ** 2 + (t - C[2]) ** 2
        if rad2 <= C[3] ** 2 and 0 <= t < ray[6] and t < best[0]:
            best = (t, ue)
    return best


def test_exact_matches_50_digit_polynomial_roots():
    w = W.gentle_valid_curves(40, seed=3)
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers)
    for i in range(40):
        tb, ub = _mp_exact(w.rays[:, i].astype(float), w.fibers[:, i].astype(float))
        if not h[i]:
            assert tb == math.inf
            continue
        assert abs(float(tb) - t[i]) <= 1e-13 * t[i]
        assert abs(float(ub) - u[i]) <= 1e-11


def test_depth_method_converges_to_exact():
    w = W.gentle_valid_curves(300, seed=11)
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers)
    prev = None
    for d in (6, 10, 14, 18, 22):
        td, ud, hd = oracle.intersect_depth(w.rays, w.fibers, d)
        b = hd.astype(bool) & h.astype(bool)
        err = np.median(np.abs(td[b] - t[b]))
        if prev is not None:
            assert err < prev / 6            # about 2x per level on tapered fibers
        prev = err
    assert prev < 5e-9


def test_exact_degenerate():
    fib = np.array([0, 0, 0, .1, 1, 0, 0, .1, 2, 0, 0, .1, 3, 0, 0, .1], float)
    kind, t, u = oracle.single_exact(np.array([-2.0, 0.05, 0, 1, 0, 0, 100]), fib)
    assert kind == 2 and abs(t - 2.0) < 1e-14 and u == 0.0
    kind, t, u = oracle.single_exact(np.array([1.3, 0.0, -4, 0, 0, 1, 100]), fib)
    assert kind == 1 and abs(t - 3.9) < 1e-12 and abs(u - 1.3 / 3) < 1e-12
    kind, t, u = oracle.single_exact(np.array([1.3, 0.0, 0.05, 0, 0, 1, 100]), fib)
    assert kind == 4 and t == 0.0            # origin inside the fiber
    kind, t, u = oracle.single_exact(np.array([1.3, 0.5, -4, 0, 0, 1, 100]), fib)
    assert kind == 0
    kind, t, u = oracle.single_exact(np.array([0, 0, -5, 0, 0, 0, 100]), fib)
    assert kind == 0


@pytest.mark.parametrize("ends", ["start", "both"])
def test_zero_end_tangent_straight_fiber_is_the_capped_cylinder(ends):
    """p1 = p0 (and p2 = p3): the straight fiber's parametrisation stalls at
    the end, C'(0) = 0, but the swept solid is still the capped cylinder. Its
    end disc is normal to the limit of C'(u) as u -> 0 (p2 - p0); without it
    the rays that enter through that cap would be missed. The depth-d method
    gives the same solid (its zero-tangent caps fall back to the same edge)."""
    w = W.exact_straight_fibers(1500, seed=W.SEED_BASE + 23, cap_fraction=0.5)
    P = W.unpack_fibers(w.fibers).copy()
    P[:, 1, :3] = P[:, 0, :3]
    if ends == "both":
        P[:, 2, :3] = P[:, 3, :3]
    fibers = W.pack_fibers(P)
    assert np.array_equal(W.unpack_fibers(fibers), P)      # exact in float32
    O, D, tmax = unpack_rays(w.rays)
    r = P[:, 0, 3]
    A, B = P[:, 0, :3], P[:, 3, :3]
    t_cf, u_cf, h_cf = capped_cylinder(O, D, A, B, r, tmax)
    _, _, h_lo = capped_cylinder(O, D, A, B, r * (1 - 1e-7), tmax)
    _, _, h_hi = capped_cylinder(O, D, A, B, r * (1 + 1e-7), tmax)
    stable = h_lo == h_hi
    t, u, h, kind = oracle.intersect_exact(w.rays, fibers)
    h = h.astype(bool)
    assert np.array_equal(h[stable], h_cf[stable])
    assert (kind == 2).sum() > 50 and (kind == 3).sum() > 50
    b = stable & h_cf & h
    assert np.max(np.abs(t[b] - t_cf[b]) / t_cf[b]) < 1e-11
    # cap hits report the end parameter; side hits a parameter whose point
    # lies at the closed form's axial position
    cap = b & ((kind == 2) | (kind == 3))
    assert np.all(u[cap] == np.where(kind[cap] == 2, 0.0, 1.0))
    side = b & (kind == 1)
    Cu = bezier(P[side][:, :, :3], u[side][:, None])[:, 0]
    axial = np.sum((Cu - A[side]) * (B[side] - A[side]), axis=1) / np.sum((B[side] - A[side]) ** 2, axis=1)
    assert np.abs(axial - u_cf[side]).max() < 1e-9
    for d in (4, 22):
        td, ud, hd = oracle.intersect_depth(w.rays, fibers, d)
        hd = hd.astype(bool)
        assert np.array_equal(hd[stable], h_cf[stable]), d
        bd = stable & h_cf & hd
        assert np.max(np.abs(td[bd] - t_cf[bd]) / t_cf[bd]) < 1e-11, d


@pytest.mark.parametrize("zero_tangents", [False, True])
def test_edge_on_rays_equal_capped_cylinder(zero_tangents):
    """Rays within 1e-10..1e-7 rad of perpendicular to straight constant-
    radius fibers: every disc plane is nearly parallel to the ray, and the
    entry and exit of the disc the ray crosses are two roots of the side
    polynomial about 1e-9 apart. The oracle must still give the analytic
    capped-cylinder entry (side hits, relative t 1e-12), with evenly spaced
    control points and with p1 = p0, p2 = p3 (a stalled parametrisation)."""
    rng = np.random.default_rng(61 + zero_tangents)
    n = 300
    a = rng.uniform(0, 1, (n, 3))
    ax = rng.standard_normal((n, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    L = rng.uniform(0.05, 0.5, n)
    r = rng.uniform(0.001, 0.01, n)
    # a unit vector normal to the axis, tilted towards it by a tiny angle
    perp = np.cross(ax, rng.standard_normal((n, 3)))
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    tilt = 10.0 ** rng.uniform(-10, -7, n)
    Dn = perp * np.cos(tilt)[:, None] + ax * np.sin(tilt)[:, None]
    s = rng.uniform(0.1, 0.9, n)              # where along the fiber the ray passes
    off = rng.uniform(-0.9, 0.9, n) * r       # and how far from the axis
    side = np.cross(Dn, ax)
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    target = a + (s * L)[:, None] * ax + off[:, None] * side
    O = target - 2.0 * Dn
    P = np.empty((n, 4, 4))
    for k in range(4):
        f = (0.0 if k < 2 else 1.0) if zero_tangents else k / 3.0
        P[:, k, :3] = a + (f * L)[:, None] * ax
        P[:, k, 3] = r
    rays = np.concatenate([O, Dn, np.full((n, 1), 10.0)], axis=1).T.copy()
    fibers = P.reshape(n, 16).T.copy()
    t_cf, u_cf, h_cf = capped_cylinder(O, Dn, P[:, 0, :3], P[:, 3, :3], r, np.full(n, 10.0))
    assert h_cf.all()
    t = np.empty(n)
    kind = np.empty(n, int)
    for i in range(n):
        kind[i], t[i], _ = oracle.single_exact(rays[:, i], fibers[:, i])
    assert np.all(kind == 1), np.unique(kind, return_counts=True)
    assert np.max(np.abs(t - t_cf) / t_cf) < 1e-12


def _near_collinear_perpendicular(n, seed=11):
    """Near-collinear fibers along x (control points at thirds, jittered by
    1e-6 N(0, I)) and rays exactly along -z through the fiber: the disc plane
    of one u nearly contains each ray, so the side polynomial's two roots
    about that u (the ray entering and leaving the disc) lie about 1e-11
    apart."""
    rng = np.random.default_rng(seed)
    L = rng.uniform(0.1, 1.0, n)
    k = np.arange(4)[None, :, None] / 3.0
    P = np.zeros((n, 4, 4))
    P[:, :, :3] = k * np.stack([L, 0 * L, 0 * L], 1)[:, None, :] + 1e-6 * rng.standard_normal((n, 4, 3))
    P[:, :, :3] += np.round(rng.uniform(0, 1, (n, 3)) * 64)[:, None, :] / 64
    r = rng.uniform(0.001, 0.02, n)
    P[:, :, 3] = r[:, None]
    F = W.pack_fibers(P)
    P = W.unpack_fibers(F)
    s = rng.uniform(0.05, 0.95, n)
    A, B = P[:, 0, :3], P[:, 3, :3]
    X = A + s[:, None] * (B - A)
    O = X + np.stack([0 * L, rng.uniform(-1.2, 1.2, n) * r, 0 * L + 3.0], 1)
    R = W.pack_rays(O, np.tile([0.0, 0.0, -1.0], (n, 1)), np.full(n, 100.0))
    return R, F, P, r


def test_discs_nearly_containing_the_ray():
    """Where one disc plane nearly contains the ray, the entry and exit of
    that disc are roots of the side polynomial closer together than its
    coefficients' rounding resolves. The oracle must find the entry: every
    hit of the chord's capped cylinder (outside a 1e-4 r band) is a hit,
    within the 1e-6 jitter's effect (relative t 1e-4); pairs that an
    isolation of the side polynomial alone got wrong (the exit taken, no
    hit, or a hit where the ray passes outside the disc) and a sample of the
    rest equal a 50-digit solution to 1e-12."""
    n = 20000
    R, F, P, r = _near_collinear_perpendicular(n)
    O, D = R[0:3].T.astype(float), R[3:6].T.astype(float)
    tmax = np.full(n, 100.0)
    t, u, h, kind = oracle.intersect_exact(R, F)
    with np.errstate(invalid="ignore"):
        tc, uc, hc = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r, tmax)
        # the jitter moves the surface by up to about 5e-6 from the chord's cylinder
        _, _, hl = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r * (1 - 1e-4) - 5e-6, tmax)
        _, _, hh = capped_cylinder(O, D, P[:, 0, :3], P[:, 3, :3], r * (1 + 1e-4) + 5e-6, tmax)
    stable = (hl == hh)
    assert stable.sum() > 0.9 * n and hc[stable].mean() > 0.7
    assert np.array_equal(h[stable].astype(bool), hc[stable])
    both = stable & hc & h.astype(bool)
    assert np.max(np.abs(t[both] - tc[both]) / tc[both]) < 1e-4
    rng = np.random.default_rng(5)
    check = [6579, 6875, 8067, 10714, 18743] + list(rng.choice(np.nonzero(both)[0], 6, replace=False))
    for i in check:
        tb, ub = _mp_exact(R[:, i].astype(float), F[:, i].astype(float), dps=60)
        assert hc[i] and math.isfinite(float(tb)), i
        assert abs(float(tb) - t[i]) <= 1e-12 * float(tb), (i, float(tb), t[i])
    for i in (3022, 16054):
        tb, ub = _mp_exact(R[:, i].astype(float), F[:, i].astype(float), dps=60)
        assert not hc[i] and tb == math.inf and not h[i], i


def test_edge_on_rays_past_stalled_ends_miss():
    """Rays within 1e-10..1e-7 rad of perpendicular to straight fibers with
    p1 = p0 and p2 = p3, passing 2-30 % of the length beyond an end (within
    the radius of the axis line): the capped cylinder is missed, and so must
    the solid be. At a stalled end C' vanishes with both factors of the side
    polynomial, which is no boundary point (no disc plane); taking it had
    given hits here."""
    rng = np.random.default_rng(62)
    n = 400
    a = rng.uniform(0, 1, (n, 3))
    ax = rng.standard_normal((n, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    L = rng.uniform(0.05, 0.5, n)
    r = rng.uniform(0.001, 0.01, n)
    perp = np.cross(ax, rng.standard_normal((n, 3)))
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    tilt = 10.0 ** rng.uniform(-10, -7, n)
    Dn = perp * np.cos(tilt)[:, None] + ax * np.sin(tilt)[:, None]
    s = np.where(rng.uniform(0, 1, n) < 0.5, rng.uniform(1.02, 1.3, n), rng.uniform(-0.3, -0.02, n))
    off = rng.uniform(-0.9, 0.9, n) * r
    side = np.cross(Dn, ax)
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    O = a + (s * L)[:, None] * ax + off[:, None] * side - 2.0 * Dn
    P = np.empty((n, 4, 4))
    for k in range(4):
        P[:, k, :3] = a + ((0.0 if k < 2 else 1.0) * L)[:, None] * ax
        P[:, k, 3] = r
    rays = np.concatenate([O, Dn, np.full((n, 1), 10.0)], axis=1).T.copy()
    fibers = P.reshape(n, 16).T.copy()
    _, _, h_cf = capped_cylinder(O, Dn, P[:, 0, :3], P[:, 3, :3], r, np.full(n, 10.0))
    assert not h_cf.any()
    kinds = [oracle.single_exact(rays[:, i], fibers[:, i])[0] for i in range(n)]
    assert all(k == 0 for k in kinds), np.unique(kinds, return_counts=True)
