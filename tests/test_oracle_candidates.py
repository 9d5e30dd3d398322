"""Pins of the oracles' nearest hit over candidate lists (CPU only).

The nearest hit of a ray over its candidate list, each candidate tested
against the ray shortened to the latest hit, is checked against the minimum
of the independent per-pair results (the list brute-forced pair by pair,
ties to the first in the list), against lists whose order, duplicates and
truncation have known outcomes, and against scenes whose nearest fiber is
known by construction (translated copies of one fiber along the ray).
"""
import numpy as np
import pytest

import oracle
from paper_1811_03374_amd import workloads as W


def brute_min(t, hit, off):
    """Per ray: index (into the flattened list) of the smallest hit t, the
    first of equal ones; -1 when no candidate hits."""
    n = off.shape[0] - 1
    best = np.full(n, -1, np.int64)
    for r in range(n):
        a, b = off[r], off[r + 1]
        h = np.nonzero(hit[a:b])[0]
        if h.size:
            tt = t[a:b][h]
            best[r] = a + h[np.argmin(tt)]          # argmin keeps the first of equal values
    return best


def copies_scene(n, seed=W.SEED_BASE + 70):
    """Rays of the 2^20 recipe with candidate lists holding their own fiber,
    two copies of it translated along the ray (one nearer, one farther) and
    two fibers of other rays, shuffled: the nearer copy is the nearest hit
    whenever the fiber is hit."""
    w = W.straight_and_curved(n)
    P = W.unpack_fibers(w.fibers)
    O, D = w.rays[0:3].T.astype(np.float64), w.rays[3:6].T.astype(np.float64)
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    near, far = P.copy(), P.copy()
    near[:, :, :3] -= 0.05 * Dn[:, None, :]
    far[:, :, :3] += 0.05 * Dn[:, None, :]
    fibers = np.concatenate([w.fibers, W.pack_fibers(near), W.pack_fibers(far)], axis=1)
    rng = np.random.default_rng(seed)
    lists = []
    for r in range(n):
        c = np.array([r, n + r, 2 * n + r, rng.integers(0, n), rng.integers(0, n)], np.int32)
        rng.shuffle(c)
        lists.append(c)
    off = np.arange(n + 1, dtype=np.int64) * 5
    return w.rays, fibers, off, np.concatenate(lists), n


@pytest.mark.parametrize("scene", ["copies", "hair"])
def test_nearest_equals_min_over_candidates(scene):
    if scene == "copies":
        rays, fibers, off, cand, n = copies_scene(3000)
        depth = 16
    else:
        w = W.hair_candidates(1 << 13)
        rays, fibers, off, cand, n = w.rays, w.fibers, w.meta["cand_off"], w.meta["cand_fiber"], w.rays.shape[1]
        depth = 22
    t, u, h, f = oracle.intersect_nearest(rays, fibers, off, cand, depth)
    pr = np.repeat(np.arange(n), np.diff(off)).astype(np.int32)
    tp, up, hp = oracle.intersect_depth(rays, fibers, depth, pair_ray=pr, pair_fiber=cand)
    best = brute_min(tp, hp.astype(bool), off)
    hit = best >= 0
    assert np.array_equal(h.astype(bool), hit)
    assert np.array_equal(t[hit], tp[best[hit]]) and np.array_equal(u[hit], up[best[hit]])
    assert np.array_equal(f[hit], cand[best[hit]]) and (f[~hit] == -1).all()
    assert np.isinf(t[~hit]).all() and np.isnan(u[~hit]).all()
    nh = np.add.reduceat(hp.astype(np.int64), off[:-1]) if n else np.zeros(0)
    assert (nh >= 2).sum() > (0.3 * n if scene == "copies" else 20)
    if scene == "copies":
        # the nearer copy wins whenever the ray's own fiber is hit alone
        assert (f[hit] >= n).mean() > 0.9


def test_nearest_order_duplicates_and_truncation():
    w = W.straight_and_curved(500)
    n = 500
    fibers = np.concatenate([w.fibers, w.fibers], axis=1)        # fiber n + r duplicates fiber r
    t1, u1, h1 = oracle.intersect_depth(w.rays, w.fibers, 9)
    # [r, r]: the duplicate never beats the first (equal t is not nearer)
    off = np.arange(n + 1, dtype=np.int64) * 2
    cand = np.stack([np.arange(n), np.arange(n)], axis=1).reshape(-1).astype(np.int32)
    t, u, h, f = oracle.intersect_nearest(w.rays, fibers, off, cand, 9)
    assert np.array_equal(t, t1, equal_nan=True) and np.array_equal(h, h1)
    assert np.array_equal(f[h1.astype(bool)], np.arange(n)[h1.astype(bool)])
    # [n + r, r]: identical geometry, the first in the list is kept
    cand2 = np.stack([np.arange(n) + n, np.arange(n)], axis=1).reshape(-1).astype(np.int32)
    _, _, _, f2 = oracle.intersect_nearest(w.rays, fibers, off, cand2, 9)
    assert np.array_equal(f2[h1.astype(bool)], n + np.arange(n)[h1.astype(bool)])
    # truncation: only the first max_cand candidates are tested
    cand3 = np.stack([np.full(n, 10**6 % n), np.arange(n)], axis=1).reshape(-1).astype(np.int32)
    _, _, h3, f3 = oracle.intersect_nearest(w.rays, fibers, off, cand3, 9, max_cand=1)
    t4, _, h4 = oracle.intersect_depth(w.rays, w.fibers, 9, pair_fiber=np.full(n, 10**6 % n, np.int32))
    assert np.array_equal(h3, h4)
    # empty lists and out-of-range fibers are misses
    off0 = np.zeros(n + 1, np.int64)
    t0, u0, h0, f0 = oracle.intersect_nearest(w.rays, fibers, off0, np.zeros(0, np.int32), 9)
    assert not h0.any() and (f0 == -1).all() and np.isinf(t0).all()
    offb = np.arange(n + 1, dtype=np.int64)
    _, _, hb, fb = oracle.intersect_nearest(w.rays, fibers, offb, np.full(n, 2 * n, np.int32), 9)
    assert not hb.any() and (fb == -1).all()


def test_exact_nearest_equals_min_over_candidates():
    rays, fibers, off, cand, n = copies_scene(1500, seed=W.SEED_BASE + 71)
    t, u, h, kind, f = oracle.nearest_exact(rays, fibers, off, cand)
    pr = np.repeat(np.arange(n), np.diff(off)).astype(np.int32)
    tp, up, hp, kp = oracle.intersect_exact(rays, fibers, pair_ray=pr, pair_fiber=cand)
    best = brute_min(tp, hp.astype(bool), off)
    hit = best >= 0
    assert np.array_equal(h.astype(bool), hit)
    assert np.array_equal(t[hit], tp[best[hit]]) and np.array_equal(f[hit], cand[best[hit]])
    assert np.array_equal(kind[hit], kp[best[hit]])
