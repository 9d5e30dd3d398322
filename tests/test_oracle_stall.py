"""Pins of the oracle's stalled end nodes (reading R19; CPU only).

A node that holds an end of the curve is a leaf before the depth once its
extent (largest squared length of chord and end tangents) is at most
(2^-20 X)^2 and at most 2^-16 of the root's extent times 4^-level. The pins
place straight fibers along the x axis with rays along that axis, where the
ray frame, X and every node's extent have closed forms, and check the leaf
level of the first hit against the level derived here by hand:

* zero tangents at both ends: C(u) = p0 + D (3u^2 - 2u^3); the end node
  [0, h] has chord D h^2 (3 - 2h), end tangent 2 D h^2 (1 - h), start tangent
  0, so its extent is |D|^2 h^4 (3 - 2h)^2; the root's is |D|^2;
* a fiber far from the ray origin binds the relative bound, one close to it
  the absolute bound;
* with regular end tangents (p1 = p0 + D/4) the end node's chord is about
  3/4 |D| 2^-level, its extent about 9/16 |D|^2 4^-level, and the relative
  bound never holds: the search runs to the depth;
* cusps (interior stalls) run to the depth as well.
The hit itself stays the capped cylinder's: the end cap plane at t = s.
"""
import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W


def stall_level(L, X):
    """First level at which the start node of a straight fiber of length L
    with zero end tangents, seen with largest ray-frame coordinate X, is
    stalled (None: never)."""
    for lvl in range(0, 24):
        h = 2.0 ** -lvl
        ext, root = L * L * h ** 4 * (3 - 2 * h) ** 2, L * L
        if ext <= 2.0 ** -40 * X * X and ext <= 2.0 ** -16 * h * h * root:
            return lvl
    return None


def axis_scene(L, s, y0, r, tangents="zero", reverse=False):
    """One straight fiber from (0,0,0) to (L,0,0), radius r, and one ray
    along +x from (-s, y0, 0) (reverse: along -x from (L + s, y0, 0))."""
    if tangents == "zero":
        xs = [0.0, 0.0, L, L]
    else:
        xs = [0.0, L / 4, 3 * L / 4, L]          # p1 - p0 = p3 - p2 = D/4
    P = np.zeros((1, 4, 4))
    P[0, :, 0] = xs
    P[0, :, 3] = r
    O = np.array([[L + s if reverse else -s, y0, 0.0]])
    D = np.array([[-1.0 if reverse else 1.0, 0.0, 0.0]])
    return W.pack_rays(O, D, np.array([1e30])), W.pack_fibers(P)


@pytest.mark.parametrize("L,s", [(1.0, 1.0), (1.0, 1024.0), (0.25, 3.0), (2.0, 62.0), (0.5, 0.5)])
@pytest.mark.parametrize("reverse", [False, True])
def test_zero_tangent_end_stalls_at_the_derived_level(L, s, reverse):
    X = L + s
    want = stall_level(L, X)
    assert want is not None and want < 22
    R, F = axis_scene(L, s, 0.25 * 0.01, 0.01, reverse=reverse)
    t, u, h, st = oracle.intersect_depth(R, F, 22, stats=True)
    assert h[0] == 1
    assert t[0] == s                                  # the end cap plane, exactly
    assert u[0] == (1.0 if reverse else 0.0)
    assert st[0, 3] == want, (st[0], want)
    # both bounds matter: far fibers bind the relative one, near ones the absolute one
    rel_only = next(l for l in range(24) if (2.0 ** -l) ** 2 * (3 - 2 * 2.0 ** -l) ** 2 <= 2.0 ** -16)
    if s >= 64 * L:
        assert want == rel_only
    if s <= L:
        assert want > rel_only


@pytest.mark.parametrize("depth", [12, 16, 22])
def test_regular_end_tangents_run_to_the_depth(depth):
    """p1 - p0 = D/4 (a straight fiber traversed at non-uniform but never
    vanishing speed): the relative bound never holds, every hit's leaf is at
    the depth, also far from the ray origin where the absolute bound holds
    from level 10 on."""
    for L, s in ((1.0, 1.0), (1.0, 1024.0), (0.25, 4096.0)):
        for reverse in (False, True):
            R, F = axis_scene(L, s, 0.0025, 0.01, tangents="regular", reverse=reverse)
            t, u, h, st = oracle.intersect_depth(R, F, depth, stats=True)
            assert h[0] == 1 and t[0] == s and st[0, 3] == depth


def test_cusps_and_collinear_curves_run_to_the_depth():
    """Interior stalls are not cut short: on the cusp and near-collinear
    families every hit's leaf is at the depth."""
    w = W.degenerate_geometry(1 << 12)
    fam = np.arange(w.n_pairs) % 4
    for depth in (16, 22):
        t, u, h, st = oracle.intersect_depth(w.rays, w.fibers, depth, stats=True)
        for f in (0, 1, 3):
            m = (fam == f) & h.astype(bool)
            assert m.sum() > 100
            assert np.all(st[m, 3] == depth), (f, np.unique(st[m, 3]))


def test_zero_tangent_family_stalls_only_at_ends():
    """On random-walk curves with zero end tangents some hits end in
    stalled leaves, and each such leaf lies at an end of the parameter
    range: its hit's u is within the leaf's span of 0 or 1."""
    w = W.degenerate_geometry(1 << 12)
    fam = np.arange(w.n_pairs) % 4
    t, u, h, st = oracle.intersect_depth(w.rays, w.fibers, 22, stats=True)
    m = (fam == 2) & h.astype(bool)
    early = m & (st[:, 3] < 22)
    assert early.sum() > 20
    span = 2.0 ** -st[early, 3]
    assert np.all((u[early] <= span) | (u[early] >= 1 - span))
