"""Pins of the oracles' surface normals (CPU only).

The depth oracle's normal follows the paper's final computation of an
intersection (Appendix C, the listing that computes the normal and u): the
direction from the leaf chord's point at the hit's projection to the hit
point, or a cap's outward normal when the entry is through the curve's start
or end cap plane. The exact oracle's normal is the normal of the swept-disc
solid itself. Both are checked against closed forms (capped cylinder,
truncated cone), against the gradient of the solid's implicit function
(finite differences), and against properties every entry has.
"""
import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W
from test_oracle_pins import bezier, bezier_d, capped_cylinder, unpack_rays


def bezier_dd(P, u):
    a2 = 3 * (P[:, 2] - 2 * P[:, 1] + P[:, 0])
    a3 = P[:, 3] - 3 * P[:, 2] + 3 * P[:, 1] - P[:, 0]
    u = u[..., None]
    return 2 * a2[:, None] + 6 * u * a3[:, None]


def unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def angle(a, b):
    c = np.sum(unit(a) * unit(b), axis=-1)
    s = np.linalg.norm(np.cross(unit(a), unit(b)), axis=-1)
    return np.arctan2(s, c)


def straight_axis_frame(P, X):
    """Axis coordinate s of points X along the chord of straight fibers P, the
    unit axis a, its length L and the unit radial direction of X."""
    A = P[:, 0, :3]
    B = P[:, 3, :3]
    L = np.linalg.norm(B - A, axis=1)
    a = (B - A) / L[:, None]
    s = np.sum((X - A) * a, axis=1)
    radial = X - A - s[:, None] * a
    return s, a, L, radial


def cone_fibers(n, seed):
    """Straight fibers (exactly collinear control points) with a linear taper
    from ra to rb, rays as for the straight pins. The radius coefficients lie
    on a 2^-14 grid (rb - ra a multiple of 3 steps), so float32 holds r(u)
    exactly linear."""
    w = W.exact_straight_fibers(n, seed=seed)
    P = W.unpack_fibers(w.fibers)
    rng = np.random.default_rng(seed + 7)
    g = 2.0 ** -14
    ra = rng.integers(120, 600, n) * g
    step = rng.integers(-35, 36, n) * g
    rb = np.maximum(ra + 3 * step, ra - 3 * np.floor((ra - 80 * g) / (3 * g)) * g)
    P[:, :, 3] = W.linear_taper(ra, rb)
    w.fibers = W.pack_fibers(P)
    return w


# ---------------------------------------------------------------------------
# straight constant radius: the capped cylinder's normal, at every depth
# ---------------------------------------------------------------------------

def _cylinder_expected(w):
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    Dn = unit(D)
    r = P[:, 0, 3]
    A, B = P[:, 0, :3], P[:, 3, :3]
    t_cf, _, h_cf = capped_cylinder(O, D, A, B, r, tmax)
    _, _, h_lo = capped_cylinder(O, D, A, B, r * (1 - 1e-7), tmax)
    _, _, h_hi = capped_cylinder(O, D, A, B, r * (1 + 1e-7), tmax)
    X = O + np.where(h_cf, t_cf, 0.0)[:, None] * Dn
    s, a, L, radial = straight_axis_frame(P, X)
    # which surface: the caps lie at s = 0 and s = L, the side at distance r
    at_start = np.abs(s) <= 1e-9 * L
    at_end = np.abs(s - L) <= 1e-9 * L
    on_side = np.abs(np.linalg.norm(radial, axis=1) - r) <= 1e-9 * r
    expect = np.where(at_start[:, None], -a, np.where(at_end[:, None], a, unit(radial + 1e-300)))
    # rims (side and a cap at once) are left out: both normals are right there
    clear = h_cf & (h_lo == h_hi) & (at_start ^ at_end ^ on_side) & ~(on_side & (at_start | at_end))
    return expect, clear, at_start | at_end


@pytest.mark.parametrize("depth", [0, 3, 9, 16, 22])
def test_depth_normals_on_straight_fibers_are_the_capped_cylinders(depth):
    w = W.exact_straight_fibers(1500)
    expect, clear, cap = _cylinder_expected(w)
    t, u, h, nn = oracle.intersect_depth(w.rays, w.fibers, depth, normal=True)
    assert clear.sum() > 400 and (clear & cap).sum() > 50
    assert np.array_equal(h[clear].astype(bool), np.ones(clear.sum(), bool))
    n, alt = nn[:, 0:3], nn[:, 3:6]
    err = np.minimum(angle(n[clear], expect[clear]), angle(alt[clear], expect[clear]))
    assert err.max() < 1e-9, err.max()
    assert np.allclose(np.linalg.norm(n[clear], axis=1), 1.0, atol=1e-14)


def test_exact_normals_on_straight_fibers_are_the_capped_cylinders():
    w = W.exact_straight_fibers(1500)
    expect, clear, cap = _cylinder_expected(w)
    t, u, h, kind, n = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    assert np.array_equal(h[clear].astype(bool), np.ones(clear.sum(), bool))
    assert set(np.unique(kind[clear & cap])) <= {2, 3} and set(np.unique(kind[clear & ~cap])) == {1}
    err = angle(n[clear], expect[clear])
    assert err.max() < 1e-9, err.max()


# ---------------------------------------------------------------------------
# straight linear taper: a truncated cone
# ---------------------------------------------------------------------------

def test_exact_normals_on_cones_tilt_by_the_taper():
    """The side of a truncated cone with radius r(s) = ra + (rb - ra) s / L
    has the outward normal e - (rb - ra)/L a (e the unit radial direction, a
    the axis), before normalisation; the cap discs have -a and a."""
    w = cone_fibers(1500, W.SEED_BASE + 60)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, kind, n = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    hb = h.astype(bool)
    X = O + np.where(hb, t, 0.0)[:, None] * unit(D)
    s, a, L, radial = straight_axis_frame(P, X)
    ra, rb = P[:, 0, 3], P[:, 3, 3]
    slope = (rb - ra) / L
    side = hb & (kind == 1)
    assert side.sum() > 300 and (hb & (kind > 1)).sum() > 50
    # the entry lies on the cone
    assert np.array_equal(P[:, :, 3], W.linear_taper(ra, rb))
    r_at = ra + slope * s
    assert np.abs(np.linalg.norm(radial[side], axis=1) - r_at[side]).max() < 1e-9
    expect = unit(radial) - slope[:, None] * a
    assert angle(n[side], expect[side]).max() < 1e-9
    assert (np.abs(slope[side]) > 0.02).sum() > 100         # tilts well above the bound
    for k, sgn in ((2, -1.0), (3, 1.0)):
        m = hb & (kind == k)
        assert angle(n[m], sgn * a[m]).max() < 1e-12


@pytest.mark.parametrize("depth", [4, 22])
def test_depth_normals_on_cones_are_radial(depth):
    """The depth method's leaves are cylinders about the chord, which is the
    axis here: its side normal is the radial direction at any taper (the
    listing has no taper term), and its caps give -a and a."""
    w = cone_fibers(1500, W.SEED_BASE + 61)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, nn = oracle.intersect_depth(w.rays, w.fibers, depth, normal=True)
    hb = h.astype(bool)
    X = O + np.where(hb, t, 0.0)[:, None] * unit(D)
    s, a, L, radial = straight_axis_frame(P, X)
    at_cap = (np.abs(s) <= 1e-9 * L) | (np.abs(s - L) <= 1e-9 * L)
    rr = np.linalg.norm(radial, axis=1)
    side = hb & ~at_cap & (rr > 1e-6)
    cap = hb & at_cap & (rr < 0.95 * np.minimum(P[:, 0, 3], P[:, 3, 3]))   # off the rims
    assert side.sum() > 300 and cap.sum() > 30
    assert angle(nn[side, 0:3], radial[side]).max() < 1e-9
    expect = np.where((np.abs(s) <= 1e-9 * L)[:, None], -a, a)
    assert angle(nn[cap, 0:3], expect[cap]).max() < 1e-9


# ---------------------------------------------------------------------------
# bent, thick, tapered fibers: the gradient of the solid's implicit function
# ---------------------------------------------------------------------------

def _phi(P, X, u0):
    """Implicit function of the side surface near the points X: with u the
    parameter of the disc plane through X (<X - C(u), C'(u)> = 0, Newton from
    u0), |X - C(u)| - r(u)."""
    u = u0.copy()
    for _ in range(30):
        C = bezier(P, u[:, None])[:, 0]
        d1 = bezier_d(P, u[:, None])[:, 0]
        d2 = bezier_dd(P, u[:, None])[:, 0]
        e = X - C[:, :3]
        g = np.sum(e * d1[:, :3], axis=1)
        dg = -np.sum(d1[:, :3] ** 2, axis=1) + np.sum(e * d2[:, :3], axis=1)
        u = u - g / dg
    C = bezier(P, u[:, None])[:, 0]
    return np.linalg.norm(X - C[:, :3], axis=1) - C[:, 3]


def test_exact_side_normals_are_the_implicit_gradient():
    """Central differences of the implicit function at the entry give the
    surface normal independently of the closed form (which carries the
    taper's tilt and the curvature term of the moving disc)."""
    w = W.gentle_valid_curves(600, seed=W.SEED_BASE + 62, bend=0.12, rmax=0.09)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, kind, n = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    m = (kind == 1) & (u > 1e-3) & (u < 1 - 1e-3)
    assert m.sum() > 150
    Pm, X, um = P[m], O[m] + t[m, None] * unit(D[m]), u[m]
    h_ = 1e-6
    grad = np.empty_like(X)
    for k in range(3):
        dx = np.zeros(3)
        dx[k] = h_
        grad[:, k] = (_phi(Pm, X + dx, um) - _phi(Pm, X - dx, um)) / (2 * h_)
    err = angle(n[m], grad)
    assert err.max() < 1e-6, err.max()
    # the taper's tilt alone (no curvature term) is measurably different here
    C = bezier(Pm, um[:, None])[:, 0]
    d1 = bezier_d(Pm, um[:, None])[:, 0]
    e = unit(X - C[:, :3])
    tilt_only = e - (d1[:, 3] / np.linalg.norm(d1[:, :3], axis=1))[:, None] * unit(d1[:, :3])
    assert angle(tilt_only, grad).max() > 1e-4


# ---------------------------------------------------------------------------
# properties of every entry; the depth method's normals approach the solid's
# ---------------------------------------------------------------------------

def test_normals_face_the_incoming_ray():
    w = W.straight_and_curved(1 << 12)
    O, D, tmax = unpack_rays(w.rays)
    Dn = unit(D)
    t, u, h, nn = oracle.intersect_depth(w.rays, w.fibers, 22, normal=True)
    # entries through a leaf's side or a cap of the curve (an entry through an
    # inner split plane lies inside the leaf cylinder: the listing's radial
    # normal there has no side to face)
    entry = nn[:, 7]
    hb = h.astype(bool) & (t > 0) & (entry <= 2)
    assert hb.sum() > 1000 and (hb & (entry > 0)).sum() > 20
    assert np.sum(nn[hb, 0:3] * Dn[hb], axis=1).max() <= 1e-12
    tx, ux, hx, kind, n = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    m = (kind >= 1) & (kind <= 3)
    assert np.sum(n[m] * Dn[m], axis=1).max() <= 1e-9
    assert np.allclose(np.linalg.norm(n[m], axis=1), 1.0, atol=1e-14)


def test_depth_normals_converge_to_the_solid_at_constant_radius():
    """At a constant radius the solid's normal is the radial direction from
    C(u); the leaf chord approaches the curve like 4^-d, so the depth
    method's normal approaches it as the depth grows."""
    w = W.gentle_valid_curves(800, seed=W.SEED_BASE + 63)
    P = W.unpack_fibers(w.fibers)
    P[:, :, 3] = P[:, :1, 3]
    w.fibers = W.pack_fibers(P)
    tx, ux, hx, kind, nx_ = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    med = []
    for depth in (6, 10, 14):
        t, u, h, nn = oracle.intersect_depth(w.rays, w.fibers, depth, normal=True)
        m = (kind == 1) & h.astype(bool)
        err = angle(nn[m, 0:3], nx_[m])
        med.append(np.median(err))
    assert med[0] > med[1] > med[2]
    assert med[2] < 1e-4, med


def test_depth_cap_entries_match_the_solids_caps():
    """Where the solid is entered through an end disc well inside its rim, the
    depth method at depth 22 enters its first or last leaf through the same
    cap plane (also when that leaf is reached by backtracking) and reports
    that disc's normal. Curves that break the constraints of Section 3.4 are
    left out: the method may crop their solid."""
    w = W.straight_and_curved(1 << 14)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, st, nn = oracle.intersect_depth(w.rays, w.fibers, 22, stats=True, normal=True)
    tx, ux, hx, kind, n = oracle.intersect_exact(w.rays, w.fibers, normal=True)
    X = O + np.where(hx.astype(bool), tx, 0.0)[:, None] * unit(D)
    end = np.where(kind == 3, 3, 0)
    C = P[np.arange(len(P)), end]
    rim = np.linalg.norm(X - C[:, :3], axis=1) / C[:, 3]
    valid = np.array([oracle.cubic_constraints(P[i].reshape(16)) == 31 for i in range(len(P))])
    m = ((kind == 2) | (kind == 3)) & (rim < 0.99) & valid
    assert m.sum() > 60
    assert np.array_equal(nn[m, 7], (kind[m] - 1).astype(float))
    assert angle(nn[m, 0:3], n[m]).max() < 1e-9


@pytest.mark.parametrize("name,n", [("straight_and_curved", 1 << 14), ("degenerate_geometry", 1 << 13)])
def test_depth_hits_on_a_cap_plane_take_its_normal(name, n):
    """A depth-22 hit point that lies in the plane of the curve's start (end)
    cap -- the plane through p0 normal to the start tangent, through p3
    normal to the end tangent, their limits where a tangent vanishes -- was
    entered through that plane and takes its outward normal (or, at the rim
    of a leaf, may take the side's). This holds for any curve, also where the
    leaf is reached by backtracking, and is checked from the hit point alone."""
    w = getattr(W, name)(n)
    P = W.unpack_fibers(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, st, nn = oracle.intersect_depth(w.rays, w.fibers, 22, stats=True, normal=True)
    hb = h.astype(bool) & (t > 0)
    X = O + np.where(hb, t, 0.0)[:, None] * unit(D)
    q = P[:, :, :3]
    chord = q[:, 3] - q[:, 0]
    cc = np.sum(chord * chord, axis=1, keepdims=True)

    def limit(cands):
        out = cands[-1].copy()
        for c in reversed(cands[:-1]):
            ok = np.sum(c * c, axis=1, keepdims=True) > 2.0 ** -40 * cc
            out = np.where(ok, c, out)
        return unit(out)

    n0 = limit([q[:, 1] - q[:, 0], q[:, 2] - q[:, 0], chord])
    n1 = limit([q[:, 3] - q[:, 2], q[:, 3] - q[:, 1], chord])
    scale = np.abs(X).max(axis=1) + np.abs(q).max(axis=(1, 2))
    on0 = hb & (np.abs(np.sum((X - q[:, 0]) * n0, axis=1)) <= 1e-12 * scale)
    on1 = hb & (np.abs(np.sum((X - q[:, 3]) * n1, axis=1)) <= 1e-12 * scale)
    assert (on0 | on1).sum() > 100 and ((on0 | on1) & (st[:, 2] > 0)).sum() >= 4
    for on, expect in ((on0 & ~on1, -n0), (on1 & ~on0, n1)):
        err = np.minimum(angle(nn[on, 0:3], expect[on]), angle(nn[on, 3:6], expect[on]))
        assert err.max() < 1e-9, err.max()
