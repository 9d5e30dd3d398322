"""GPU parity of the FP64 refinement against the exact swept-disc oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1811_03374_amd import binding
from paper_1811_03374_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
T_REL_TOL64 = 1e-12
BAND = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def exact_with_band(w):
    t, u, h, k = oracle.intersect_exact(w.rays, w.fibers, w.pair_ray, w.pair_fiber)
    _, ul, hl, _ = oracle.intersect_exact(w.rays, w.fibers, w.pair_ray, w.pair_fiber,
                                          radius_scale=1 - BAND)
    _, uh, hh, _ = oracle.intersect_exact(w.rays, w.fibers, w.pair_ray, w.pair_fiber,
                                          radius_scale=1 + BAND)
    both = hl.astype(bool) & hh.astype(bool)
    spread = np.where(both, np.abs(np.where(both, ul, 0) - np.where(both, uh, 0)), 0.0)
    return t, u, h.astype(bool), k, hl != hh, spread


def run_refined(w, depth):
    g = lambda a: None if a is None else torch.from_numpy(a).to(DEV)
    out = binding.intersect_pairs(g(w.rays), g(w.fibers), depth, g(w.pair_ray), g(w.pair_fiber),
                                  refine=True)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def validity(w):
    P = W.unpack_fibers(w.fibers)
    if w.pair_fiber is not None:
        P = P[w.pair_fiber]
    return np.array([oracle.cubic_constraints(P[i].reshape(16)) == 31 for i in range(P.shape[0])])


def check_refined(w, depth, label):
    """Refined results against the exact surface. Curves that break the
    constraints of Section 3.4 (the paper splits them beforehand) are
    reported separately and not included in the statistics asserted on."""
    say(f"[refine] {label} depth={depth} n={w.n_pairs}")
    t32, u32, h, t64, u64 = run_refined(w, depth)
    t_x, u_x, h_x, kind, band, spread = exact_with_band(w)
    hg = h.astype(bool)
    valid = validity(w)
    inv = ~band & ~valid
    if inv.any():
        say(f"[refine]   invalid curves: n={inv.sum()} flag_disagree={(hg[inv] != h_x[inv]).mean():.3e}")
    out = ~band & valid
    flag_bad = (hg != h_x) & out
    both = hg & h_x & out
    rel = np.abs(t64[both] - t_x[both]) / t_x[both]
    du = np.abs(u64[both] - u_x[both])
    utol = 1e-9 + spread[both]
    st = {"pairs": int(hg.size), "in_band": int(band.sum()), "flag_bad": int(flag_bad.sum()),
          "hit_rate": float(h_x.mean()), "max_rel_t": float(rel.max()) if rel.size else 0.0,
          "p999_rel_t": float(np.quantile(rel, 0.999)) if rel.size else 0.0,
          "max_du": float(du.max()) if du.size else 0.0, "u_bad": int((du > utol).sum()),
          "cap_hits": int(((kind == 2) | (kind == 3)).sum())}
    say(f"[refine]   {st}")
    bi = np.nonzero(both)[0]
    for j in np.argsort(-rel)[:3] if rel.size else []:
        i = bi[j]
        say(f"[refine]     worst pair {i}: rel_t={rel[j]:.3e} t64={t64[i]!r} t_x={t_x[i]!r} "
            f"u64={u64[i]!r} u_x={u_x[i]!r} kind={kind[i]} t32={t32[i]!r}")
    for i in np.nonzero(flag_bad)[0][:5]:
        say(f"[refine]     flag pair {i}: gpu hit={hg[i]} t64={t64[i]!r} u64={u64[i]!r} | exact "
            f"hit={h_x[i]} t={t_x[i]!r} u={u_x[i]!r} kind={kind[i]}")
    # float outputs are the rounded refined values; misses are encoded as usual
    assert np.all(np.isinf(t64[~hg])) and np.all(np.isnan(u64[~hg]))
    assert np.array_equal(t32[hg], t64[hg].astype(np.float32))
    return st


@pytest.mark.parametrize("depth", [17, 22])
def test_refine_straight_and_curved(depth):
    w = W.straight_and_curved(1 << 14 | 77)
    st = check_refined(w, depth, "straight_and_curved")
    assert st["flag_bad"] == 0 and st["u_bad"] == 0, st
    assert st["max_rel_t"] <= T_REL_TOL64, st


def test_refine_near_tangent_rays():
    # every ray within 1e-6 r of the silhouette: the entry point is ill-
    # conditioned (a residual that passes Newton's test can still move t far
    # beyond rounding), so a refined t must come from a bracketed root. All
    # pairs lie in the flag band; t is checked wherever both sides hit.
    # Bound: FP64 evaluation of C(u) rounds at eps times the control points'
    # spread across the ray (about 0.1 here, against r ~ 5e-5), and at a
    # penetration of delta * r the entry moves by that error over
    # |dphi/du| ~ r sqrt(delta); down to delta ~ 1e-8 this keeps t within
    # about 1e-12 relative. The tail is asserted at 1e-11 (a Newton point
    # accepted on its residual alone was off by up to 5e-10), the bulk at
    # 1e-12. The exact oracle bisects in extended precision.
    w = W.hair_precision(1 << 14, 2000, depth=22, grazing_fraction=1.0, graze_width=1e-6)
    t32, u32, h, t64, u64 = run_refined(w, 22)
    t_x, u_x, h_x, kind = oracle.intersect_exact(w.rays, w.fibers, w.pair_ray, w.pair_fiber)
    both = h.astype(bool) & h_x.astype(bool)
    rel = np.abs(t64[both] - t_x[both]) / t_x[both]
    say(f"[refine] near-tangent n={w.n_pairs} gpu hits={int(h.sum())} exact hits={int(h_x.sum())} "
        f"both={int(both.sum())} max_rel_t={rel.max():.3e} p99.9={np.quantile(rel, 0.999):.3e}")
    assert both.sum() > 1000
    assert np.quantile(rel, 0.999) <= T_REL_TOL64
    assert rel.max() <= 10 * T_REL_TOL64


def test_refine_hair_precision_stress():
    w = W.hair_precision(1 << 16, 20000, depth=22)
    st = check_refined(w, 22, "hair (10% grazing within 1e-3 r)")
    assert st["flag_bad"] == 0 and st["u_bad"] == 0, st
    assert st["max_rel_t"] <= T_REL_TOL64, st


def test_refine_keeps_shallow_pairs_plain():
    """Depth <= 16 is not refined: the refined call gives the plain results bit
    for bit, with t64/u64 the widened floats (pairs of depths 12 and 19 mixed
    in one call)."""
    w = W.straight_and_curved(4096)
    pd = np.where(np.arange(w.n_pairs) % 3 == 0, 19, 12).astype(np.uint8)
    g = lambda a: torch.from_numpy(a).to(DEV)
    t, u, h = [o.cpu().numpy() for o in binding.intersect_pairs(g(w.rays), g(w.fibers), 12,
                                                              pair_depth=g(pd))]
    t2, u2, h2, t64, u64 = [o.cpu().numpy() for o in binding.intersect_pairs(
        g(w.rays), g(w.fibers), 12, pair_depth=g(pd), refine=True)]
    torch.cuda.synchronize()
    shallow = pd == 12
    bits = lambda a: a.view(np.uint32)
    assert np.array_equal(bits(t[shallow]), bits(t2[shallow]))
    assert np.array_equal(bits(u[shallow]), bits(u2[shallow]))
    assert np.array_equal(h[shallow], h2[shallow])
    hit = h2.astype(bool) & shallow
    assert np.array_equal(t64[hit], t2[hit].astype(np.float64))
    assert np.array_equal(u64[hit], u2[hit].astype(np.float64))
