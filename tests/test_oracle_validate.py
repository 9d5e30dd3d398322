"""Pins of the validation and pre-subdivision oracle (CPU only).

The five inequalities agree with the pinned classifier; the cap-plane excess
is checked against closed forms (straight fibers never cross their caps, a
circular arc crosses them exactly when the tube radius exceeds the arc's
radius, by (r - rho) in the widest disc) and against an independent dense
evaluation; pre-subdivided pieces reproduce the curve over their intervals,
tile [0, 1] in order, and are valid unless the level limit stopped them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W
from test_oracle_pins import bezier, bezier_d


def arc(r, k=0.5522847498):
    """Quarter-circle cubic of radius 1 in the xy plane (p0 = (1, 0), p3 =
    (0, 1)), tube radius r."""
    P = np.array([[1, 0, 0, r], [1, k, 0, r], [k, 1, 0, r], [0, 1, 0, r]], float)
    return P.reshape(16)


def test_constraint_bits_match_the_classifier():
    w = W.straight_and_curved(3000)
    P = W.unpack_fibers(w.fibers)
    for i in range(P.shape[0]):
        q = P[i].reshape(16)
        m, _, _ = oracle.validate(q)
        assert (m & 31) == (~oracle.cubic_constraints(q)) & 31


def test_straight_fibers_never_cross_their_caps():
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = rng.normal(size=3), rng.normal(size=3)
        s = np.sort(rng.uniform(0, 1, 2))
        P = np.array([a, a + s[0] * (b - a), a + s[1] * (b - a), b])
        r = rng.uniform(0.01, 5.0, 4)
        q = np.concatenate([P, r[:, None]], axis=1).reshape(16)
        m, e0, e1 = oracle.validate(q)
        assert (m & 96) == 0 and e0 <= 1e-12 and e1 <= 1e-12


@pytest.mark.parametrize("r", [0.5, 0.9, 0.99, 1.01, 1.1, 1.5])
def test_arc_crosses_its_caps_when_thicker_than_its_radius(r):
    """For a circular arc of radius rho, the disc at angle phi from an end
    lies rho sin(phi) behind that end's cap plane and reaches r sin(phi)
    towards it: the excess is (r - rho) sin(phi), largest in the disc at the
    other end (phi = 90 degrees). The cubic quarter circle has radius 1 to
    within 3e-4."""
    m, e0, e1 = oracle.validate(arc(r))
    ext = math.sqrt(2) + r
    thick = r > 1.0
    assert bool(m & 32) == thick and bool(m & 64) == thick
    if thick:
        assert abs(e0 * ext - (r - 1.0)) <= 3e-4 and abs(e1 * ext - (r - 1.0)) <= 3e-4
    assert (m & 31) == 0


def dense_excess(q, end, n=200001):
    """The cap-plane excess on a dense grid, in numpy (independent code)."""
    P = q.reshape(1, 4, 4)
    u = np.linspace(0, 1, n)[None, :]
    C = bezier(P, u)[0]
    D = bezier_d(P, u)[0][:, :3]
    pts = P[0, :, :3]
    chord = pts[3] - pts[0]
    cands = [pts[3] - pts[2], pts[3] - pts[1], chord] if end else [pts[1] - pts[0], pts[2] - pts[0], chord]
    nv = next((c for c in cands[:2] if c @ c > 2.0 ** -40 * (chord @ chord)), chord)
    nv = nv / np.linalg.norm(nv)
    dl = np.linalg.norm(D, axis=1)
    s = np.linalg.norm(np.cross(D, nv), axis=1) / np.where(dl > 0, dl, 1)
    along = (pts[3] - C[:, :3]) @ nv if end else (C[:, :3] - pts[0]) @ nv
    h = np.where(dl > 0, C[:, 3] * s - along, -np.inf)
    return h.max()


def test_excess_search_against_a_dense_grid():
    rng = np.random.default_rng(7)
    w = W.degenerate_geometry(600)
    P = W.unpack_fibers(w.fibers)
    for i in rng.choice(P.shape[0], 120, replace=False):
        q = P[i].reshape(16)
        ext = np.linalg.norm(q[12:15] - q[0:3]) + np.abs(q[3::4]).max()
        _, e0, e1 = oracle.validate(q)
        for end, e in ((0, e0), (1, e1)):
            g = dense_excess(q, end) / ext
            # the search finds at least the grid's maximum, and no more than
            # the grid misses between its points
            assert e >= g - 1e-12
            assert e <= g + 1e-7


def test_presplit_pieces_reproduce_and_tile_the_curve():
    w = W.degenerate_geometry(400)
    P = W.unpack_fibers(w.fibers)
    n_split = 0
    for i in range(P.shape[0]):
        q = P[i].reshape(16)
        pieces, u0, u1, masks = oracle.presplit(q, 6)
        assert u0[0] == 0.0 and u1[-1] == 1.0 and np.array_equal(u0[1:], u1[:-1])
        levels = np.round(-np.log2(u1 - u0)).astype(int)
        assert np.all(u1 - u0 == 2.0 ** -levels)
        # valid unless the level limit stopped the halving
        assert np.all((masks == 0) | (levels == 6))
        if oracle.validate(q)[0] == 0:
            assert len(pieces) == 1 and np.array_equal(pieces[0], q)
        n_split += len(pieces) > 1
        v = np.linspace(0, 1, 7)
        for k in range(len(pieces)):
            Cp = bezier(pieces[k].reshape(1, 4, 4), v[None, :])[0]
            Cq = bezier(q.reshape(1, 4, 4), (u0[k] + v * (u1[k] - u0[k]))[None, :])[0]
            assert np.allclose(Cp, Cq, rtol=0, atol=1e-12 * (1 + np.abs(Cq).max()))
    assert n_split > 50
