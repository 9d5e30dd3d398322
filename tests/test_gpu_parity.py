"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1811_03374_amd import binding
from paper_1811_03374_amd import workloads as W
from parity import compare, oracle_with_band, tie_resolver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(w, depth=None, counts=False):
    d = w.depth if depth is None else depth
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    pr = None if w.pair_ray is None else torch.from_numpy(w.pair_ray).to(DEV)
    pf = None if w.pair_fiber is None else torch.from_numpy(w.pair_fiber).to(DEV)
    pd = None if w.pair_depth is None else torch.from_numpy(w.pair_depth).to(DEV)
    out = binding.intersect_pairs(rays, fibers, d, pr, pf, pd, counts=counts)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def check(w, depth=None, label=""):
    d = w.depth if depth is None else depth
    say(f"[parity] {label} {w.name} depth={d} n={w.n_pairs}")
    (t_o, u_o, h_o), band = oracle_with_band(w, d)
    t_g, u_g, h_g = run_gpu(w, d)
    dd = w.pair_depth if w.pair_depth is not None else d
    st = compare(t_g, u_g, h_g, t_o, u_o, h_o, band, dd, alt=tie_resolver(w, d))
    say(f"[parity]   {st}")
    return st


def test_plain_unit_cube_depth4():
    st = check(W.plain_unit_cube())
    assert st["ok"], st
    assert 0.35 < st["hit_rate"] < 0.65


@pytest.mark.parametrize("depth", [2, 3, 4, 6, 9, 12, 16, 19, 22])
def test_straight_and_curved_depth_sweep(depth):
    w = W.straight_and_curved(1 << 14 | 77)    # several blocks plus a ragged tail
    st = check(w, depth)
    assert st["ok"], st


@pytest.mark.parametrize("depth", [9, 22])
def test_hair_precision_fp32(depth):
    """The hair workload in FP32 at depths 9 and 22: the full table of
    100,000 strands (800,000 segments offset by 1e3 in every coordinate),
    2^16 rays of which 10 % graze within 1e-3 r of the silhouette, pairs
    gathered through an index, element by element against the depth
    oracle."""
    w = W.hair_precision(1 << 16, 100_000, depth=depth)
    st = check(w, depth, "hair (10% grazing)")
    assert st["ok"], st
    assert 0.4 < st["hit_rate"] < 0.6


def test_depth_extremes():
    w = W.straight_and_curved(3001)
    for d in (0, 1, 23):
        st = check(w, d)
        assert st["ok"], st


def test_node_counts_match_oracle():
    """Integer work: node tests, splits, backtracks and leaf level per pair are
    the oracle's except where a rounding-level tie flips a decision. Ties grow
    common once nodes shrink to the FP32 resolution of their coordinates
    (deep levels), where different paths still end on the same surface point."""
    w = W.straight_and_curved(1 << 13)
    for d, need in ((4, 0.999), (9, 0.998), (16, 0.98), (22, 0.95)):
        _, _, h_o, st_o = oracle.intersect_depth(w.rays, w.fibers, d, stats=True)
        t_g, u_g, h_g, cn = run_gpu(w, d, counts=True)
        same = np.all(cn == st_o, axis=1)
        say(f"[counts] depth={d} identical={same.mean():.5f} "
            f"tests gpu={cn[:, 0].mean():.3f} oracle={st_o[:, 0].mean():.3f}")
        assert same.mean() >= need
        assert abs(cn[:, 0].mean() / st_o[:, 0].mean() - 1) < 0.01
        assert np.array_equal(h_g.astype(bool)[same], h_o.astype(bool)[same])
        assert np.array_equal((cn[:, 3] >= 0), h_g.astype(bool))
        assert np.all(cn[h_g.astype(bool), 3] == d)


def test_per_pair_depth_and_gathered_indices():
    w = W.plain_unit_cube()
    rng = np.random.default_rng(4)
    w.pair_depth = rng.integers(0, 24, w.n_pairs).astype(np.uint8)
    st = check(w, 9, "per-pair depth")
    assert st["ok"], st


def test_strided_tables_and_index_gather():
    w = W.straight_and_curved(5000)
    rng = np.random.default_rng(8)
    n = 7000
    pr = rng.integers(0, 5000, n).astype(np.int32)
    pf = pr.copy()
    # pad the tables: row stride larger than the count
    R = np.zeros((7, 5200), np.float32); R[:, :5000] = w.rays
    F = np.zeros((16, 5300), np.float32); F[:, :5000] = w.fibers
    rays = torch.from_numpy(R).to(DEV)[:, :5000]
    fibers = torch.from_numpy(F).to(DEV)[:, :5000]
    t, u, h = (o.cpu().numpy() for o in binding.intersect_pairs(
        rays, fibers, 9, torch.from_numpy(pr).to(DEV), torch.from_numpy(pf).to(DEV)))
    torch.cuda.synchronize()
    ws = W.Workload("strided", w.rays, w.fibers, pr, pf, 9)
    (t_o, u_o, h_o), band = oracle_with_band(ws, 9)
    st = compare(t, u, h, t_o, u_o, h_o, band, 9, alt=tie_resolver(ws, 9))
    say(f"[strided] {st}")
    assert st["ok"], st


def test_gathered_fiber_records_bitwise():
    """A gathered call with at least as many pairs as fibers reads the fibers
    through 64-byte records copied first; its results equal, bit for bit,
    those of the same pairs materialised as tables and called with identity
    pairing (no records), and agree with the oracle."""
    w = W.straight_and_curved(3000, seed=515)
    rng = np.random.default_rng(9)
    n = 9000
    pr = rng.integers(0, 3000, n).astype(np.int32)
    pf = pr.copy()                                   # rays aim at their own fiber ...
    pf[::3] = rng.integers(0, 3000, n)[::3]          # ... except a third (mostly misses)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    for d in (9, 22):
        t, u, h = (o.cpu().numpy() for o in binding.intersect_pairs(
            rays, fibers, d, torch.from_numpy(pr).to(DEV), torch.from_numpy(pf).to(DEV)))
        R = torch.from_numpy(np.ascontiguousarray(w.rays[:, pr])).to(DEV)
        F = torch.from_numpy(np.ascontiguousarray(w.fibers[:, pf])).to(DEV)
        t2, u2, h2 = (o.cpu().numpy() for o in binding.intersect_pairs(R, F, d))
        torch.cuda.synchronize()
        say(f"[gather] depth={d} pairs={n} hits={h.mean():.3f}")
        assert np.array_equal(_bits(t), _bits(t2))
        assert np.array_equal(_bits(u), _bits(u2))
        assert np.array_equal(h, h2)
        ws = W.Workload("gathered", w.rays, w.fibers, pr, pf, d)
        (t_o, u_o, h_o), band = oracle_with_band(ws, d)
        st = compare(t, u, h, t_o, u_o, h_o, band, np.full(n, d, np.uint8), alt=tie_resolver(ws, d))
        assert st["ok"], st


def test_prepared_calls_on_two_streams():
    """binding.PreparedPairs (checked and marshalled once) launched repeatedly
    on two streams at once gives, bit for bit, the results of intersect_pairs;
    outputs too small for the call are refused before any launch."""
    w = W.straight_and_curved(20_000, seed=616)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    ref = {d: [o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, d)] for d in (9, 22)}
    calls = {d: binding.PreparedPairs(rays, fibers, d) for d in (9, 22)}
    side = {9: torch.cuda.Stream(), 22: torch.cuda.Stream()}
    for d in (9, 22):
        side[d].wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        for d in (22, 9):
            calls[d].launch(side[d])
    torch.cuda.synchronize()
    for d in (9, 22):
        t, u, h = (o.cpu().numpy() for o in (calls[d].t, calls[d].u, calls[d].hit))
        assert np.array_equal(_bits(t), _bits(ref[d][0]))
        assert np.array_equal(_bits(u), _bits(ref[d][1]))
        assert np.array_equal(h, ref[d][2])
    small = (torch.empty(100, device=DEV), torch.empty(20_000, device=DEV),
             torch.empty(20_000, dtype=torch.uint8, device=DEV))
    with pytest.raises(ValueError):
        binding.PreparedPairs(rays, fibers, 9, out=small)
    with pytest.raises(ValueError):
        binding.intersect_pairs(rays, fibers, 9, out=small)


def test_degenerate_pairs_are_misses():
    w = W.straight_and_curved(512)
    R = w.rays.copy()
    R[3:6, 0] = 0.0                         # zero direction
    R[3, 1] = np.nan                         # NaN direction
    R[6, 2] = np.nan                         # NaN tmax
    R[3:6, 3] = np.inf                       # infinite direction
    w2 = W.Workload("degenerate", R, w.fibers, None, None, 9)
    t, u, h = run_gpu(w2)
    assert not h[:4].any() and np.all(np.isinf(t[:4])) and np.all(np.isnan(u[:4]))
    # out-of-range indices and per-pair depth above 23
    pr = np.arange(512, dtype=np.int32); pr[5] = 512; pr[6] = -1
    pf = np.arange(512, dtype=np.int32); pf[7] = 10 ** 6
    pd = np.full(512, 9, np.uint8); pd[8] = 24; pd[9] = 255
    w3 = W.Workload("bad-index", w.rays, w.fibers, pr, pf, 9, pd)
    t, u, h = run_gpu(w3)
    assert not h[5:10].any() and np.all(np.isinf(t[5:10])) and np.all(np.isnan(u[5:10]))
    # every other pair is an ordinary pair, held to the full bar
    keep = np.ones(512, bool); keep[5:10] = False
    ws = w.subset(np.nonzero(keep)[0])
    (t_o, u_o, h_o), band = oracle_with_band(ws, 9)
    st = compare(t[keep], u[keep], h[keep], t_o, u_o, h_o, band, 9, alt=tie_resolver(ws, 9))
    assert st["ok"], st


def test_empty_and_single():
    w = W.straight_and_curved(1)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    t, u, h = binding.intersect_pairs(rays[:, :0], fibers[:, :0], 9)
    torch.cuda.synchronize()
    assert t.numel() == 0
    for seed in range(8):                    # one pair per call, hits and misses
        w = W.straight_and_curved(1, seed=900 + seed)
        t, u, h = run_gpu(w)
        (t_o, u_o, h_o), band = oracle_with_band(w, 9)
        st = compare(t, u, h, t_o, u_o, h_o, band, 9, alt=tie_resolver(w, 9))
        assert st["ok"], (seed, st)


def test_argument_errors_on_device():
    w = W.straight_and_curved(64)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    with pytest.raises(binding.FiberHitError):
        binding.intersect_pairs(rays, fibers, 24)
    with pytest.raises(ValueError):
        binding.intersect_pairs(rays.double(), fibers, 9)


@pytest.mark.parametrize("depth", [9, 22])
def test_full_size_sampled(depth):
    """The 2^20-pair workload in the benchmark's launch configuration, checked
    on a seeded sample of 16384 pairs that the oracle computes one by one."""
    w = W.straight_and_curved(1 << 20, depth)
    say(f"[parity] full size 2^20 depth={depth}")
    t_g, u_g, h_g = run_gpu(w, depth)
    idx = np.sort(np.random.default_rng(depth).choice(w.n_pairs, 16384, replace=False))
    ws = w.subset(idx)
    (t_o, u_o, h_o), band = oracle_with_band(ws, depth)
    st = compare(t_g[idx], u_g[idx], h_g[idx], t_o, u_o, h_o, band, depth,
                 alt=tie_resolver(ws, depth))
    say(f"[parity]   {st}")
    assert st["ok"], st
    # properties that hold for every pair: miss encoding, t within [0, tmax)
    hit = h_g.astype(bool)
    assert np.all(np.isinf(t_g[~hit])) and np.all(np.isnan(u_g[~hit]))
    assert np.all((t_g[hit] >= 0) & (t_g[hit] < w.rays[6][hit]))
    assert np.all((u_g[hit] >= 0) & (u_g[hit] <= 1))
    assert 0.45 < hit.mean() < 0.55


@pytest.mark.parametrize("depth", [9, 22])
def test_hair_full_size_sampled(depth):
    """The hair configuration at its full size (2^24 rays against 800,000
    segments gathered through an index), in the benchmark's launch
    configuration, checked on a seeded sample of 8192 pairs against the depth
    oracle; at depth 22 also the refined call against the exact oracle
    (flags identical outside the 1e-4 r band, relative t <= 1e-12). Every
    pair's miss encoding and t range are checked too."""
    w = W.hair_precision(1 << 24, 100_000, depth=depth)
    say(f"[parity] hair full size 2^24 depth={depth}")
    t_g, u_g, h_g = run_gpu(w, depth)
    idx = np.sort(np.random.default_rng(100 + depth).choice(w.n_pairs, 8192, replace=False))
    ws = w.subset(idx)
    (t_o, u_o, h_o), band = oracle_with_band(ws, depth)
    st = compare(t_g[idx], u_g[idx], h_g[idx], t_o, u_o, h_o, band, depth, alt=tie_resolver(ws, depth))
    say(f"[parity]   {st}")
    assert st["ok"], st
    hit = h_g.astype(bool)
    assert np.all(np.isinf(t_g[~hit])) and np.all(np.isnan(u_g[~hit]))
    tmax = w.rays[6][w.pair_ray[hit]] if w.pair_ray is not None else w.rays[6][hit]
    assert np.all((t_g[hit] >= 0) & (t_g[hit] < tmax))
    if depth != 22:
        return
    g = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    r = binding.intersect_pairs(g(w.rays), g(w.fibers), depth, g(w.pair_ray), g(w.pair_fiber), refine=True)
    torch.cuda.synchronize()
    h64, t64 = r[2].cpu().numpy()[idx].astype(bool), r[3].cpu().numpy()[idx]
    tx, ux, hx, _ = oracle.intersect_exact(ws.rays, ws.fibers, ws.pair_ray, ws.pair_fiber)
    _, _, hl, _ = oracle.intersect_exact(ws.rays, ws.fibers, ws.pair_ray, ws.pair_fiber, radius_scale=1 - 1e-4)
    _, _, hh, _ = oracle.intersect_exact(ws.rays, ws.fibers, ws.pair_ray, ws.pair_fiber, radius_scale=1 + 1e-4)
    m = hl == hh
    both = m & h64 & hx.astype(bool)
    rel = np.abs(t64[both] - tx[both]) / tx[both]
    say(f"[parity]   refined: outside band {m.sum()}, flag disagree {(h64[m] != hx.astype(bool)[m]).sum()}, "
        f"max rel t {rel.max():.2e}")
    assert np.array_equal(h64[m], hx.astype(bool)[m])
    assert rel.max() <= 1e-12


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32 if a.dtype == np.float32 else np.uint8)


def test_results_independent_of_call_size():
    """A call of 2^20 + 4099 pairs (wave shares of uneven length, a ragged
    tail): every pair's result equals that of a separate call on a subset of
    the pairs (bitwise), at the start, across the 2^20 mark and at the end."""
    n = (1 << 20) + 4099
    w = W.straight_and_curved(n, 22)
    say(f"[call size] n={n}")
    t_g, u_g, h_g = run_gpu(w, 22)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    for lo, hi in ((0, 3000), ((1 << 20) - 1500, (1 << 20) + 1500), (n - 3000, n)):
        idx = torch.arange(lo, hi, dtype=torch.int32, device=DEV)
        t, u, h = (o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, 22, idx, idx))
        torch.cuda.synchronize()
        assert np.array_equal(_bits(t), _bits(t_g[lo:hi]))
        assert np.array_equal(_bits(u), _bits(u_g[lo:hi]))
        assert np.array_equal(h, h_g[lo:hi])


def test_concurrent_streams():
    """Calls enqueued alternately on two streams (each with its own workspace,
    which the allocator keeps until its stream has passed the call) give the
    results of the same calls made one after another."""
    ws = [W.straight_and_curved(50_000 + 1000 * k, 9, seed=77 + k) for k in range(6)]
    dev_in = [(torch.from_numpy(w.rays).to(DEV), torch.from_numpy(w.fibers).to(DEV)) for w in ws]
    ref = []
    for (r, f), d in zip(dev_in, (9, 22, 4, 16, 9, 22)):
        ref.append([o.cpu().numpy() for o in binding.intersect_pairs(r, f, d)])
        torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for k, ((r, f), d) in enumerate(zip(dev_in, (9, 22, 4, 16, 9, 22))):
        outs.append(binding.intersect_pairs(r, f, d, stream=streams[k % 2]))
    torch.cuda.synchronize()
    for got, want in zip(outs, ref):
        got = [o.cpu().numpy() for o in got]
        assert np.array_equal(_bits(got[0]), _bits(want[0]))
        assert np.array_equal(_bits(got[1]), _bits(want[1]))
        assert np.array_equal(got[2], want[2])
