"""Pins of the oracle's quadratic fibers (Appendix B.1; CPU only).

The oracle holds a quadratic as its exact cubic elevation with the
quadratic's own bound. These pins check that against a plainly written
quadratic recursion (three control points, de Casteljau halves, the split
plane normal to the chord, the middle point's distance plus the largest of
three radius values), against the capped cylinder for straight quadratics,
against Thales' circle for the constraint, against the lemma that valid
quadratics split into valid halves, and the exact oracle's quadratic side
hits against the natively evaluated quadratic.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W
from test_oracle_pins import capped_cylinder, unpack_rays


def onb(w):
    s = math.copysign(1.0, w[2])
    a = -1.0 / (s + w[2])
    b = w[0] * w[1] * a
    return (np.array([1.0 + s * w[0] * w[0] * a, s * b, -s * w[0]]),
            np.array([b, s + w[1] * w[1] * a, -w[1]]))


def native_quadratic(ray, P3, depth):
    """The depth-d method on a quadratic written directly (no elevation):
    returns (hit, t, u)."""
    O, D, tmax = ray[0:3], ray[3:6], ray[6]
    w = D / np.linalg.norm(D)
    u_, v_ = onb(w)
    M = np.stack([u_, v_, w])
    q0 = [np.concatenate([M @ (P3[k, :3] - O), [P3[k, 3]]]) for k in range(3)]

    def caps(q):
        ch = q[2][:3] - q[0][:3]
        lim = 2.0 ** -40 * (ch @ ch)
        n0 = q[1][:3] - q[0][:3]
        if n0 @ n0 <= lim:
            n0 = ch
        n1 = q[2][:3] - q[1][:3]
        if n1 @ n1 <= lim:
            n1 = ch
        lo, hi = 0.0, tmax
        for n, e, start in ((n0, q[0][:3], True), (n1, q[2][:3], False)):
            c = e @ n
            if n[2] == 0.0:
                if (start and c > 0) or (not start and c < 0):
                    return math.inf, -math.inf
                continue
            t = c / n[2]
            if (n[2] > 0) == start:
                lo = max(lo, t)
            else:
                hi = min(hi, t)
        return lo, hi

    def visit(q, lo, hi, level, a0, a1):
        a = q[2][:3] - q[0][:3]
        aa = a @ a
        e1 = q[1][:3] - q[0][:3]
        e1 = e1 - (e1 @ a) / aa * a if aa > 0 else e1
        R = math.sqrt(e1 @ e1) + max(q[0][3], q[1][3], q[2][3])
        o = q[0][:3]
        g = a[0] ** 2 + a[1] ** 2
        if g <= 2.0 ** -100 * a[2] ** 2 or g == 0.0:
            if o[0] ** 2 + o[1] ** 2 > R * R:
                return None
            te, tx = -math.inf, math.inf
        else:
            dd = a[0] * o[1] - a[1] * o[0]
            e = R * R - dd * dd / g
            if e < 0:
                return None
            tc = o[2] - a[2] * (a[0] * o[0] + a[1] * o[1]) / g
            s = math.sqrt(e * (a[2] ** 2 + g) / g)
            te, tx = tc - s, tc + s
        enter, leave = max(te, lo), min(tx, hi)
        if enter > leave:
            return None
        if level >= depth:
            ul = 0.0
            if aa > 0:
                ul = min(1.0, max(0.0, (np.array([0, 0, enter]) - o) @ a / aa))
            return enter, a0 + ul * (a1 - a0)
        m01 = (q[0] + q[1]) * 0.5
        m12 = (q[1] + q[2]) * 0.5
        sp = (m01 + m12) * 0.5
        L, Rt = [q[0], m01, sp], [sp, m12, q[2]]
        n = a                                   # the tangent at the centre
        c = sp[:3] @ n
        flo, fhi = lo, hi
        if n[2] != 0.0:
            tp = c / n[2]
            beyond = tp > te
            right = beyond != (n[2] > 0)
            both = beyond and tp < tx
            if beyond:
                fhi = min(fhi, tp)
            else:
                flo = max(flo, tp)
        else:
            right = -c > 0
            both = c == 0
        am = 0.5 * (a0 + a1)
        first, second = (Rt, L) if right else (L, Rt)
        f0, f1 = (am, a1) if right else (a0, am)
        s0, s1 = (a0, am) if right else (am, a1)
        r = visit(first, flo, fhi, level + 1, f0, f1)
        if r is not None or not both:
            return r
        blo, bhi = caps(second)
        return visit(second, blo, bhi, level + 1, s0, s1)

    lo, hi = caps(q0)
    r = visit(q0, lo, hi, 0, 0.0, 1.0)
    if r is None or not r[0] < tmax:
        return False, math.inf, math.nan
    return True, r[0], r[1]


@pytest.mark.parametrize("depth", [0, 2, 5, 9])
def test_oracle_quadratic_equals_native_recursion(depth):
    w = W.quadratic_fibers(400)
    P = W.unpack_quadratics(w.fibers)
    R = w.rays.astype(np.float64)
    t, u, h = oracle.intersect_depth(w.rays, w.fibers, depth, quadratic=True)
    bad = 0
    for i in range(400):
        hn, tn, un = native_quadratic(R[:, i], P[i], depth)
        if bool(h[i]) != hn:
            bad += 1
            continue
        if hn:
            assert abs(t[i] - tn) <= 1e-11 * tn, (i, t[i], tn)
            assert abs(u[i] - un) <= 1e-9, (i, u[i], un)
    assert 0.3 < h.mean() < (0.95 if depth == 0 else 0.8)
    assert bad <= 1


@pytest.mark.parametrize("depth", [0, 4, 9, 16, 22])
def test_straight_quadratic_equals_capped_cylinder(depth):
    w = W.quadratic_fibers(2000, straight_fraction=1.0)
    P = W.unpack_quadratics(w.fibers)
    P[:, :, 3] = P[:, :1, 3]
    f = W.pack_quadratics(P)
    O, D, tmax = unpack_rays(w.rays)
    r = P[:, 0, 3]
    t_cf, u_cf, h_cf = capped_cylinder(O, D, P[:, 0, :3], P[:, 2, :3], r, tmax)
    _, _, h_lo = capped_cylinder(O, D, P[:, 0, :3], P[:, 2, :3], r * (1 - 1e-7), tmax)
    _, _, h_hi = capped_cylinder(O, D, P[:, 0, :3], P[:, 2, :3], r * (1 + 1e-7), tmax)
    stable = h_lo == h_hi
    t, u, h = oracle.intersect_depth(w.rays, f, depth, quadratic=True)
    assert np.array_equal(h[stable].astype(bool), h_cf[stable])
    both = stable & h_cf
    assert np.max(np.abs(t[both] - t_cf[both]) / t_cf[both]) < 1e-11
    assert np.max(np.abs(u[both] - u_cf[both])) < 1e-11 + 4e-15 * 2.0 ** depth


def test_quadratic_constraint_is_thales_circle():
    """<p1 - p0, p1 - p2> <= 0 exactly when p1 lies in the ball with diameter
    p0 p2 (the angle at p1 is at least a right angle)."""
    rng = np.random.default_rng(2)
    for _ in range(2000):
        p0, p2 = rng.normal(size=3), rng.normal(size=3)
        c, rad = 0.5 * (p0 + p2), 0.5 * np.linalg.norm(p2 - p0)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        k = rng.uniform(0.0, 2.0)
        if abs(k - 1.0) < 1e-6:
            continue
        p1 = c + k * rad * d
        q = np.concatenate([np.append(p0, 0.01), np.append(p1, 0.01), np.append(p2, 0.01)])
        assert oracle.quadratic_constraint(q) == (k < 1.0)


def test_valid_quadratics_split_into_valid_halves():
    """Appendix B.1's lemma: the halves of a quadratic meeting the
    constraint meet it again, down to depth 8."""
    rng = np.random.default_rng(4)
    checked = 0
    while checked < 300:
        P = rng.normal(size=(3, 4))
        if not oracle.quadratic_constraint(P.reshape(12)):
            continue
        checked += 1
        stack = [(P, 0)]
        while stack:
            Q, lvl = stack.pop()
            assert oracle.quadratic_constraint(Q.reshape(12)) or \
                abs(np.dot(Q[1, :3] - Q[0, :3], Q[1, :3] - Q[2, :3])) < 1e-12
            if lvl == 8:
                continue
            m01, m12 = (Q[0] + Q[1]) / 2, (Q[1] + Q[2]) / 2
            s = (m01 + m12) / 2
            stack += [(np.array([Q[0], m01, s]), lvl + 1), (np.array([s, m12, Q[2]]), lvl + 1)]


def test_exact_quadratic_side_hits_lie_on_the_quadratic_solid():
    w = W.quadratic_fibers(1500)
    P = W.unpack_quadratics(w.fibers)
    O, D, tmax = unpack_rays(w.rays)
    t, u, h, kind = oracle.intersect_exact(w.rays, w.fibers, quadratic=True)
    m = kind == 1
    assert m.sum() > 300
    X = O[m] + t[m, None] * D[m] / np.linalg.norm(D[m], axis=1, keepdims=True)
    uu = u[m][:, None]
    Pm = P[m]
    C = (1 - uu) ** 2 * Pm[:, 0] + 2 * uu * (1 - uu) * Pm[:, 1] + uu ** 2 * Pm[:, 2]
    Cd = 2 * (1 - uu) * (Pm[:, 1] - Pm[:, 0]) + 2 * uu * (Pm[:, 2] - Pm[:, 1])
    e = X - C[:, :3]
    assert np.abs(np.linalg.norm(e, axis=1) - C[:, 3]).max() < 1e-10
    assert np.abs(np.sum(e * Cd[:, :3], axis=1)).max() / np.linalg.norm(Cd[:, :3], axis=1).min() < 1e-9
