"""GPU parity of the nearest hit over candidate lists (through the C ABI).

FP32 results are held to the depth oracle's nearest hit (each candidate
tested against the ray shortened to the latest hit) with the per-pair bar;
refined results to the exact oracle's nearest entry. Where two candidates'
hits lie within the bar of each other, either fiber may be the nearest (an
inter-candidate tie); such rays are counted and bounded like per-pair ties.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1811_03374_amd import binding
from paper_1811_03374_amd import workloads as W
from parity import BAND, T_REL_TOL, TIE_RATE, TIE_SCALE, Band, compare
from test_oracle_candidates import copies_scene

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scene(name):
    if name == "copies":
        rays, fibers, off, cand, n = copies_scene(4000)
        return rays, fibers, off, cand, None
    w = W.hair_candidates(1 << 14)
    return w.rays, w.fibers, w.meta["cand_off"], w.meta["cand_fiber"], None


def gpu(rays, fibers, off, cand, depth, **kw):
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    out = binding.intersect_candidates(g(rays), g(fibers), g(off), g(cand), depth, **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def per_pair(rays, fibers, off, cand, depth):
    n = rays.shape[1]
    pr = np.repeat(np.arange(n), np.diff(off)).astype(np.int32)
    return pr, oracle.intersect_depth(rays, fibers, depth, pair_ray=pr, pair_fiber=cand)


@pytest.mark.parametrize("name,depth", [("copies", 9), ("copies", 22), ("hair", 9), ("hair", 22)])
def test_nearest_fp32_against_oracle(name, depth):
    rays, fibers, off, cand, _ = scene(name)
    n = rays.shape[1]
    say(f"[candidates] {name} depth={depth} rays={n} candidates={cand.size}")
    t, u, h, f = gpu(rays, fibers, off, cand, depth)
    t_o, u_o, h_o, f_o, te = oracle.intersect_nearest(rays, fibers, off, cand, depth, t_err=True)
    _, _, hl, _ = oracle.intersect_nearest(rays, fibers, off, cand, depth, radius_scale=1 - BAND)
    _, _, hh, _ = oracle.intersect_nearest(rays, fibers, off, cand, depth, radius_scale=1 + BAND)
    pr, (tp, up, hp) = per_pair(rays, fibers, off, cand, depth)

    def alt(i):
        # tie outcomes of the oracle's winner and of the GPU's candidate
        ts, us, hs = [], [], []
        for fib in {int(f_o[i]), int(f[i])} - {-1}:
            a, b, c = oracle.tie_outcomes(rays[:, i], fibers[:, fib], depth, scale=TIE_SCALE)
            ts += list(a); us += list(b); hs += list(c)
        # the per-pair hits of every candidate (a different nearest candidate)
        for j in range(off[i], off[i + 1]):
            if hp[j]:
                ts.append(tp[j]); us.append(up[j]); hs.append(True)
        return np.array(ts), np.array(us), np.array(hs, bool)

    st = compare(t, u, h, t_o, u_o, h_o, Band(hl != hh, np.zeros(n), te), depth, alt=alt)
    hb, hob = h.astype(bool), h_o.astype(bool)
    other = hb & hob & (f != f_o)
    say(f"[candidates]   {st}")
    say(f"[candidates]   other fiber kept: {other.sum()} (hits {hb.sum()})")
    assert st["ok"], st
    # a different fiber only where its own hit ties the oracle's nearest
    for i in np.nonzero(other)[0]:
        j = off[i] + np.nonzero(cand[off[i]:off[i + 1]] == f[i])[0]
        assert hp[j].any()
        assert np.min(np.abs(tp[j] - t_o[i])) <= max(T_REL_TOL * t_o[i], te[i]) * 2
    assert other.sum() <= 2 + TIE_RATE * n
    assert (f[~hb] == -1).all() and np.isinf(t[~hb]).all()


def test_single_candidate_lists_equal_pairs_bitwise():
    """A list of one candidate is the per-pair call: t, u, hit and the normal
    bit for bit, plain and refined."""
    w = W.straight_and_curved(1 << 13 | 3)
    n = w.rays.shape[1]
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    rays, fibers = g(w.rays), g(w.fibers)
    off = g(np.arange(n + 1, dtype=np.int64))
    cand = g(np.arange(n, dtype=np.int32))
    bits = lambda x: x.contiguous().view(torch.uint8)
    for refine in (False, True):
        a = binding.intersect_pairs(rays, fibers, 22, refine=refine, normal=True)
        b = binding.intersect_candidates(rays, fibers, off, cand, 22, refine=refine, normal=True)
        torch.cuda.synchronize()
        for x, y in zip(a[:3], b[:3]):
            assert torch.equal(bits(x), bits(y))
        if refine:
            assert torch.equal(bits(a[3]), bits(b[4])) and torch.equal(bits(a[4]), bits(b[5]))
        assert torch.equal(bits(a[-1]), bits(b[-1]))
        hb = b[2].bool()
        assert torch.equal(b[3][hb], cand[hb]) and bool((b[3][~hb] == -1).all())


@pytest.mark.parametrize("name", ["copies", "hair"])
def test_nearest_refined_against_exact(name):
    rays, fibers, off, cand, _ = scene(name)
    n = rays.shape[1]
    t, u, h, f, t64, u64 = gpu(rays, fibers, off, cand, 22, refine=True)
    tx, ux, hx, kind, fx = oracle.nearest_exact(rays, fibers, off, cand)
    _, _, hl, _, _ = oracle.nearest_exact(rays, fibers, off, cand, radius_scale=1 - BAND)
    _, _, hh, _, _ = oracle.nearest_exact(rays, fibers, off, cand, radius_scale=1 + BAND)
    # rays whose candidates all meet the constraints of Section 3.4 (the
    # method may crop the solid of others: they are reported only)
    P = W.unpack_fibers(fibers)
    ok = np.array([oracle.cubic_constraints(P[i].reshape(16)) == 31 for i in range(P.shape[0])])
    valid = np.logical_and.reduceat(ok[cand], off[:-1]) if cand.size else np.ones(n, bool)
    valid &= np.diff(off) > 0
    hb, hxb = h.astype(bool), hx.astype(bool)
    say(f"[candidates] refined {name}: rays with an invalid candidate: {(~valid).sum()}, "
        f"flag disagreement there {((hb != hxb) & ~valid & (hl == hh)).sum()}")
    out = (hl == hh) & valid
    flag = (hb != hxb) & out
    both = out & hb & hxb
    rel = np.abs(t64[both] - tx[both]) / tx[both]
    other = both & (f != fx)
    say(f"[candidates] refined {name}: flag_disagree={flag.sum()} of {out.sum()} max_rel_t={rel.max():.2e} "
        f"other_fiber={other.sum()}")
    assert flag.sum() == 0
    assert rel.max() <= 1e-12
    assert other.sum() <= 2 + TIE_RATE * n


def test_truncation_empty_lists_and_bad_indices():
    w = W.straight_and_curved(2000)
    n = 2000
    rays, fibers = w.rays, w.fibers
    # list r: [bad index, r, (r + 1) % n] with every third list empty
    lists = [np.array([] if r % 3 == 0 else [n + 5, r, (r + 1) % n], np.int32) for r in range(n)]
    off = np.zeros(n + 1, np.int64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    cand = np.concatenate(lists)
    t, u, h, f = gpu(rays, fibers, off, cand, 9)
    t_o, u_o, h_o, f_o = oracle.intersect_nearest(rays, fibers, off, cand, 9)
    assert not h[::3].any() and (f[::3] == -1).all()
    agree = (h == h_o) & ((f == f_o) | ~h.astype(bool))
    assert agree.mean() > 0.995
    # max_candidates = 2: the third candidate is never tested
    t2, u2, h2, f2 = gpu(rays, fibers, off, cand, 9, max_candidates=2)
    t2o, _, h2o, f2o = oracle.intersect_nearest(rays, fibers, off, cand, 9, max_cand=2)
    assert ((h2 == h2o) & ((f2 == f2o) | ~h2.astype(bool))).mean() > 0.995
    assert not (f2 == (np.arange(n) + 1) % n).any()
    # all lists empty
    t3, u3, h3, f3 = gpu(rays, fibers, np.zeros(n + 1, np.int64), np.zeros(1, np.int32), 9)
    assert not h3.any() and (f3 == -1).all() and np.isinf(t3).all()
