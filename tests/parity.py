"""Comparison of device results with the FP64 oracle (shared by tests, smoke
and the benchmark's self-check).

Bar (per pair, outside the silhouette band):
  * hit flags identical; a pair is in the band when the oracle's flag changes
    between all radius control values scaled by (1 - 1e-4) and (1 + 1e-4);
  * relative t error <= 1e-5 where both report a hit, or within the FP32
    error bound of the oracle's t where that is larger (the entry's bound in
    the oracle's node error model: large only for an ill-conditioned leaf,
    such as one next to a cusp that the ray meets nearly along its axis);
    such pairs are counted as ``t_by_bound``;
  * |u error| <= 1e-5 + s_u + c_u (both sides take u in the same leaf of
    size 2^-d, so u agrees far below the leaf size); s_u is how far the
    oracle's own u moves between the two band
    radii (1 -/+ 1e-4): near a silhouette a ray grazes the surface, the entry
    t stays well defined but its curve parameter slides along the fiber; c_u
    = 2^-20 max(1, t) / |C'(u)| is a position error of 16 float32 ulp at the
    hit mapped through the curve's speed: where the curve stalls (a zero end
    tangent makes |C'(u)| ~ u near the end) u is only that well determined.

A pair whose u lies in the neighbouring leaf (a hit on a leaf boundary, where
the ordering of the two leaves is a tie) meets the bar only through the tie
outcomes below. The number of pairs resolved as ties is bounded too:
``tie_resolved`` <= 2 + 2e-3 * pairs, so a real error cannot hide as a common
tie (the workloads here give at most about 1e-3).

Near ties: the method's result is discontinuous where a pruning or ordering
comparison is an exact tie (for example a ray that enters a leaf cylinder
exactly where it crosses an ancestor's split plane). A pair that misses the
bar above is accepted when the device result meets the same bar against one
of the results the oracle reaches by flipping at most two comparisons whose
sides differ by less than their FP32 error bounds (the oracle derives them
from a bound on the rounding of an FP32 node's coordinates, (2 + 2 level)
2^-24 times the root's extent, times each comparison's sensitivity); such
pairs are counted as ``tie_resolved``, and callers bound that count.
"""
from __future__ import annotations

import numpy as np

import oracle

BAND = 1e-4
T_REL_TOL = 1e-5
TIE_SCALE = 1.0      # multiple of the oracle's FP32 error bounds that makes a tie
TIE_RATE = 2e-3      # bound on the share of pairs that may be resolved as ties


class Band:
    """Silhouette band of the oracle: ``flag`` marks pairs whose hit flag
    changes between the two band radii; ``u_spread`` is how far u moves
    between them where both hit (plus the speed term c_u); ``t_err`` is the
    FP32 error bound of the oracle's t (0 when unknown)."""

    def __init__(self, flag, u_spread, t_err=None):
        self.flag = flag
        self.u_spread = u_spread
        self.t_err = np.zeros(np.shape(flag)) if t_err is None else t_err

    def __getitem__(self, idx):
        return Band(self.flag[idx], self.u_spread[idx], self.t_err[idx])


def speed_term(w, t_o, u_o):
    """c_u = 2^-20 max(1, t) / |C'(u)| at the oracle's hits (0 on misses)."""
    hit = np.isfinite(t_o)
    out = np.zeros(t_o.shape)
    if not hit.any():
        return out
    fi = w.pair_fiber if w.pair_fiber is not None else np.arange(t_o.shape[0])
    P = np.asarray(w.fibers, np.float64).T.reshape(-1, 4, 4)[np.asarray(fi)[hit], :, :3]
    u = u_o[hit][:, None]
    v = 1.0 - u
    d = 3 * (v * v * (P[:, 1] - P[:, 0]) + 2 * u * v * (P[:, 2] - P[:, 1]) + u * u * (P[:, 3] - P[:, 2]))
    sp = np.linalg.norm(d, axis=1)
    out[hit] = 2.0 ** -20 * np.maximum(1.0, np.abs(t_o[hit])) / np.maximum(sp, 1e-300)
    return out


def oracle_with_band(w, depth=None, stats=False):
    d = w.depth if depth is None else depth
    res = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber, w.pair_depth,
                                 stats=stats, t_err=True)
    t_err = res[-1]
    res = res[:-1]
    _, u_lo, h_lo = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber,
                                           w.pair_depth, radius_scale=1 - BAND)
    _, u_hi, h_hi = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber,
                                           w.pair_depth, radius_scale=1 + BAND)
    both = h_lo.astype(bool) & h_hi.astype(bool)
    spread = np.where(both, np.abs(np.where(both, u_lo, 0) - np.where(both, u_hi, 0)), 0.0)
    spread = spread + speed_term(w, res[0], res[1])
    return res, Band(h_lo != h_hi, spread, t_err)


def tie_resolver(w, depth=None):
    """Callable i -> (t, u, hit) arrays of the oracle's tie outcomes for pair i."""
    d0 = w.depth if depth is None else depth

    def alt(i):
        ri = int(w.pair_ray[i]) if w.pair_ray is not None else i
        fi = int(w.pair_fiber[i]) if w.pair_fiber is not None else i
        d = int(w.pair_depth[i]) if w.pair_depth is not None else d0
        return oracle.tie_outcomes(w.rays[:, ri], w.fibers[:, fi], d, scale=TIE_SCALE)
    return alt


def _meets(tg, ug, hg, to, uo, ho, utol, terr=0.0):
    if bool(hg) != bool(ho):
        return False
    if not hg:
        return True
    return abs(tg - to) <= max(T_REL_TOL * abs(to), terr) and abs(ug - uo) <= utol


def compare(t_g, u_g, h_g, t_o, u_o, h_o, band, depth, alt=None):
    """Return a dict of error statistics; ``ok`` tells whether the bar is met.
    ``band`` is a Band (or a bare flag array); ``alt`` (optional) maps a pair
    index to the oracle's tie outcomes."""
    if isinstance(band, Band):
        u_spread = np.asarray(band.u_spread, np.float64)
        t_err = np.asarray(band.t_err, np.float64)
        band = np.asarray(band.flag, bool)
    else:
        band = np.asarray(band, bool)
        u_spread = np.zeros(band.shape)
        t_err = np.zeros(band.shape)
    t_g = np.asarray(t_g, np.float64)
    u_g = np.asarray(u_g, np.float64)
    h_g = np.asarray(h_g).astype(bool)
    h_o = np.asarray(h_o).astype(bool)
    depth = np.broadcast_to(np.asarray(depth), h_g.shape).astype(np.float64)
    out = ~band
    utol_all = 1e-5 + u_spread
    with np.errstate(invalid="ignore"):
        rel_all = np.abs(t_g - t_o) / np.maximum(np.abs(t_o), 1e-30)
        du_all = np.abs(u_g - u_o)
        t_off = np.abs(t_g - t_o) > np.maximum(T_REL_TOL * np.abs(t_o), t_err)
    by_bound = out & h_g & h_o & (rel_all > T_REL_TOL) & ~t_off
    bad = out & ((h_g != h_o) | (h_g & h_o & (t_off | (du_all > utol_all))))
    resolved = np.zeros_like(bad)
    if alt is not None:
        for i in np.nonzero(bad)[0]:
            ta, ua, ha = alt(int(i))
            if any(_meets(t_g[i], u_g[i], h_g[i], ta[k], ua[k], ha[k], utol_all[i], t_err[i])
                   for k in range(len(ta))):
                resolved[i] = True
    ok_pair = ~bad | resolved
    prim = out & ~bad
    both = prim & h_g & h_o
    rel = rel_all[both]
    du = du_all[both]
    miss_ok = bool(np.all(np.isinf(t_g[~h_g])) and np.all(np.isnan(u_g[~h_g])))
    st = {
        "pairs": int(h_g.size),
        "in_band": int(band.sum()),
        "u_widened": int((u_spread > 1e-5).sum()),
        "flag_disagree_outside_band": int(((h_g != h_o) & out & ~resolved).sum()),
        "flag_disagree_rate": float(((h_g != h_o) & out & ~resolved).sum() / max(1, out.sum())),
        "tie_resolved": int(resolved.sum()),
        "t_by_bound": int(by_bound.sum()),
        "unresolved": int((~ok_pair).sum()),
        "hit_rate": float(h_o.mean()) if h_o.size else 0.0,
        "max_rel_t": float(rel.max()) if rel.size else 0.0,
        "p999_rel_t": float(np.quantile(rel, 0.999)) if rel.size else 0.0,
        "max_abs_u": float(du.max()) if du.size else 0.0,
        "miss_outputs_ok": miss_ok,
    }
    st["ok"] = bool(st["unresolved"] == 0 and miss_ok and st["tie_resolved"] <= 2 + TIE_RATE * h_g.size)
    return st
