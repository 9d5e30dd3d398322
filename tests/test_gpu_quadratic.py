"""GPU parity for quadratic fibers (FI_QUADRATIC; through the C ABI).

FP32 results against the depth oracle's quadratic mode with the per-pair bar
(tie outcomes from the oracle's quadratic mode); refined results against the
exact oracle on quadratics that meet the constraint of Appendix B.1.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1811_03374_amd import binding
from paper_1811_03374_amd import workloads as W
from parity import BAND, TIE_SCALE, Band, compare

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def g(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def oracle_band(w, d):
    t, u, h, te = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber, t_err=True,
                                         quadratic=True)
    _, u_lo, h_lo = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber,
                                           radius_scale=1 - BAND, quadratic=True)
    _, u_hi, h_hi = oracle.intersect_depth(w.rays, w.fibers, d, w.pair_ray, w.pair_fiber,
                                           radius_scale=1 + BAND, quadratic=True)
    both = h_lo.astype(bool) & h_hi.astype(bool)
    spread = np.where(both, np.abs(np.where(both, u_lo, 0) - np.where(both, u_hi, 0)), 0.0)
    return (t, u, h), Band(h_lo != h_hi, spread, te)


def resolver(w, d):
    def alt(i):
        ri = int(w.pair_ray[i]) if w.pair_ray is not None else i
        fi = int(w.pair_fiber[i]) if w.pair_fiber is not None else i
        return oracle.tie_outcomes(w.rays[:, ri], w.fibers[:, fi], d, scale=TIE_SCALE, quadratic=True)
    return alt


@pytest.mark.parametrize("depth", [0, 2, 9, 16, 22])
def test_quadratic_fp32_against_oracle(depth):
    w = W.quadratic_fibers(1 << 14 | 77)
    say(f"[quadratic] depth={depth} n={w.n_pairs}")
    t, u, h = (x.cpu().numpy() for x in binding.intersect_pairs(g(w.rays), g(w.fibers), depth, quadratic=True))
    torch.cuda.synchronize()
    (t_o, u_o, h_o), band = oracle_band(w, depth)
    st = compare(t, u, h, t_o, u_o, h_o, band, depth, alt=resolver(w, depth))
    say(f"[quadratic]   {st}")
    assert st["ok"], st


def test_quadratic_gathered_equals_identity_and_counts_run():
    w = W.quadratic_fibers(1 << 12)
    n = w.n_pairs
    rays, fibers = g(w.rays), g(w.fibers)
    perm = np.random.default_rng(1).permutation(n).astype(np.int32)
    a = binding.intersect_pairs(rays, fibers, 22, quadratic=True)
    b = binding.intersect_pairs(rays, fibers, 22, g(np.arange(n, dtype=np.int32)), g(np.arange(n, dtype=np.int32)),
                                quadratic=True)
    c = binding.intersect_pairs(rays, fibers, 22, counts=True, quadratic=True)
    d = binding.intersect_pairs_noalloc(rays, fibers, 22, quadratic=True)
    torch.cuda.synchronize()
    bits = lambda x: x.contiguous().view(torch.uint8)
    for x, y, z, q in zip(a, b, c[:3], d):
        assert torch.equal(bits(x), bits(y)) and torch.equal(bits(x), bits(z)) and torch.equal(bits(x), bits(q))
    assert int(c[3][:, 0].min().item()) >= 1


def test_quadratic_refined_against_exact():
    w = W.quadratic_fibers(1 << 13)
    P = W.unpack_quadratics(w.fibers)
    valid = np.array([oracle.quadratic_constraint(P[i].reshape(12)) for i in range(P.shape[0])])
    t, u, h, t64, u64, n = (x.cpu().numpy() for x in binding.intersect_pairs(
        g(w.rays), g(w.fibers), 22, refine=True, normal=True, quadratic=True))
    torch.cuda.synchronize()
    tx, ux, hx, kind, nx = oracle.intersect_exact(w.rays, w.fibers, normal=True, quadratic=True)
    _, _, hl, _ = oracle.intersect_exact(w.rays, w.fibers, radius_scale=1 - BAND, quadratic=True)
    _, _, hh, _ = oracle.intersect_exact(w.rays, w.fibers, radius_scale=1 + BAND, quadratic=True)
    m = valid & (hl == hh)
    hb, hxb = h.astype(bool), hx.astype(bool)
    both = m & hb & hxb
    rel = np.abs(t64[both] - tx[both]) / tx[both]
    a, b = n.T[both].astype(np.float64), nx[both]
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
    say(f"[quadratic] refined: valid {valid.mean():.3f}, flag disagree {(hb[m] != hxb[m]).sum()} of {m.sum()}, "
        f"max rel t {rel.max():.2e}, max normal angle {ang.max():.2e}")
    assert (hb[m] == hxb[m]).all()
    assert rel.max() <= 1e-12
    assert np.abs(u64[both] - ux[both]).max() <= 1e-9
    assert ang.max() <= 1e-6
