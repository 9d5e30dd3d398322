"""Batched launches: bitwise equal to one plain call per problem."""
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


def make_scenes(k=12, seed=5):
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in np.round(2.0 ** rng.uniform(6, 13, k))]
    if k > 3:
        sizes[3] = 0      # an empty problem
    if k > 5:
        sizes[5] = 1      # a single pair
    ws = [W.curved_scene(max(n, 1), 1811033744 + 1000 * s) for s, n in enumerate(sizes)]
    probs = []
    for w, n in zip(ws, sizes):
        g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
        probs.append(binding.Problem(g(w.rays[:, :n]) if n else g(w.rays[:, :0]),
                                     g(w.fibers[:, :n]) if n else g(w.fibers[:, :0]), 22,
                                     None, None, g(w.pair_depth[:n])))
    return ws, sizes, probs


def plain_reference(probs):
    out = []
    for p in probs:
        if p.n == 0:
            out.append((np.zeros(0, np.float32),) * 2 + (np.zeros(0, np.uint8),))
            continue
        t, u, h = binding.intersect_pairs(p.rays, p.fibers, p.depth, pair_depth=p.pair_depth)
        torch.cuda.synchronize()
        out.append((t.cpu().numpy(), u.cpu().numpy(), h.cpu().numpy()))
    return out


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32 if a.dtype == np.float32 else np.uint8)


def assert_same(probs, ref):
    for p, (t, u, h) in zip(probs, ref):
        assert np.array_equal(bits(p.t.cpu().numpy()), bits(t))
        assert np.array_equal(bits(p.u.cpu().numpy()), bits(u))
        assert np.array_equal(p.hit.cpu().numpy(), h)


def clear(probs):
    for p in probs:
        p.t.fill_(-1.0); p.u.fill_(-1.0); p.hit.fill_(7)


def test_batched_equals_plain_bitwise():
    ws, sizes, probs = make_scenes()
    say(f"[batched] {len(probs)} problems, {sum(sizes)} pairs")
    ref = plain_reference(probs)
    clear(probs)
    binding.intersect_batched(probs)
    torch.cuda.synchronize()
    assert_same(probs, ref)


def test_results_do_not_depend_on_tuning():
    ws, sizes, probs = make_scenes(seed=9)
    ref = plain_reference(probs)
    for t in ({"refill": 8, "waves_per_simd": 2}, {"refill": 64, "waves_per_simd": 0},
              {"refill": 1, "waves_per_simd": 1}, {"refill": 32, "waves_per_simd": 16},
              {"refill": 56, "waves_per_simd": 0, "stack": 1}, {"refill": 4, "waves_per_simd": 4, "stack": 1}):
        clear(probs)
        binding.intersect_batched(probs, tuning=t)
        torch.cuda.synchronize()
        assert_same(probs, ref)


def test_graph_plan_replays():
    ws, sizes, probs = make_scenes(seed=13)
    ref = plain_reference(probs)
    plan = binding.BatchPlan(probs)
    for rep in range(3):
        clear(probs)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert_same(probs, ref)
        x = torch.randn(1000, device=DEV).sum().item()     # eager work between replays
    plan.close()


def test_plan_on_a_side_stream():
    """A plan replayed on a stream other than the current one: work enqueued
    on that stream right after the launch (here, copies of every output) sees
    every scene's results, on two replays in a row."""
    ws, sizes, probs = make_scenes(seed=29)
    ref = plain_reference(probs)
    plan = binding.BatchPlan(probs)
    s = torch.cuda.Stream()
    for rep in range(2):
        clear(probs)
        s.wait_stream(torch.cuda.current_stream())
        plan.launch(s)
        with torch.cuda.stream(s):
            copies = [(p.t.clone(), p.u.clone(), p.hit.clone()) for p in probs]
        torch.cuda.synchronize()
        for (t, u, h), (tr, ur, hr) in zip(copies, ref):
            assert np.array_equal(bits(t.cpu().numpy()), bits(tr))
            assert np.array_equal(bits(u.cpu().numpy()), bits(ur))
            assert np.array_equal(h.cpu().numpy(), hr)
    plan.close()


def test_batched_parity_against_oracle():
    ws, sizes, probs = make_scenes(k=6, seed=21)
    binding.intersect_batched(probs)
    torch.cuda.synchronize()
    for w, n, p in zip(ws, sizes, probs):
        if n == 0:
            continue
        ws_ = w.subset(np.arange(n))
        ws_.pair_depth = w.pair_depth[:n]
        (t_o, u_o, h_o), band = oracle_with_band(ws_)
        st = compare(p.t.cpu().numpy(), p.u.cpu().numpy(), p.hit.cpu().numpy(), t_o, u_o, h_o,
                     band, ws_.pair_depth, alt=tie_resolver(ws_))
        assert st["ok"], st


def test_autotune_returns_a_grid_point(tmp_path):
    """The fastest grid point is remembered under the device's architecture
    and the batch's class, used by later calls, and survives a save and a
    load of the table."""
    ws, sizes, probs = make_scenes(seed=17)
    binding.clear_tuning()
    best, ms = binding.autotune(probs, repeats=1)
    say(f"[autotune] {best} {ms:.3f} ms")
    assert best["refill"] in (32, 48, 56) and best["waves_per_simd"] in (0, 8, 16) and best["stack"] in (0, 1)
    assert ms > 0
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    total = sum(int(p.n) for p in probs)
    depth = max(int(p.depth) for p in probs)
    assert binding.lookup_tuning(arch, total, len(probs), depth) == best
    assert binding.BatchPlan(probs).tuning() == best
    path = str(tmp_path / "tuning.txt")
    binding.save_tuning(path)
    binding.clear_tuning()
    binding.load_tuning(path)
    assert binding.lookup_tuning(arch, total, len(probs), depth) == best
    binding.clear_tuning()


def test_batched_argument_errors():
    ws, sizes, probs = make_scenes(k=3)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, workspace=small)
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, tuning={"refill": 0, "waves_per_simd": 0})
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, tuning={"refill": 32, "waves_per_simd": -1})
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, tuning={"refill": 65, "waves_per_simd": 0})
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, tuning={"refill": 32, "waves_per_simd": 17})
    with pytest.raises(binding.FiberHitError):
        binding.intersect_batched(probs, tuning={"refill": 32, "waves_per_simd": 0, "stack": 2})


def test_batched_four_million_pairs():
    """4.3 million pairs in three problems in one launch: wave shares cross
    problem boundaries (one problem has 3 pairs); results stay bitwise equal
    to one call per problem."""
    sizes = [1_500_000, 3, 2_800_000]
    probs = []
    for k, n in enumerate(sizes):
        w = W.straight_and_curved(n, 22, seed=4242 + k)
        g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
        probs.append(binding.Problem(g(w.rays), g(w.fibers), 22 if k != 1 else 9))
    say(f"[batched] {sum(sizes)} pairs in three problems")
    ref = plain_reference(probs)
    clear(probs)
    binding.intersect_batched(probs)
    torch.cuda.synchronize()
    assert_same(probs, ref)


def test_refined_batch_equals_refined_calls():
    """A batch run with FI_FP64_REFINE (per-pair depths 16..22, so some pairs
    stay on the plain rules) gives, bit for bit, the five outputs of one
    refined call per problem -- as a plain batched call and as a plan."""
    rng = np.random.default_rng(31)
    sizes = [700, 0, 1, 2500, 64, 1300]
    probs = []
    for k, n in enumerate(sizes):
        w = W.curved_scene(max(n, 1), 1811033744 + 77 * k)
        pd = rng.integers(16, 23, max(n, 1)).astype(np.uint8)
        g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
        probs.append(binding.Problem(g(w.rays[:, :n]), g(w.fibers[:, :n]), 22, None, None, g(pd[:n]),
                                     refine=True))
    say(f"[batched refine] {len(probs)} problems, {sum(sizes)} pairs")
    ref = []
    for p in probs:
        if p.n == 0:
            ref.append(None)
            continue
        out = binding.intersect_pairs(p.rays, p.fibers, p.depth, pair_depth=p.pair_depth, refine=True)
        torch.cuda.synchronize()
        ref.append([o.cpu().numpy() for o in out])

    def check():
        for p, r in zip(probs, ref):
            if r is None:
                continue
            got = [o.cpu().numpy() for o in (p.t, p.u, p.hit, p.t64, p.u64)]
            for a, b in zip(got, r):
                assert np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))

    for p in probs:
        p.t64.fill_(-1.0); p.u64.fill_(-1.0)
    clear(probs)
    binding.intersect_batched(probs, refine=True)
    torch.cuda.synchronize()
    check()
    plan = binding.BatchPlan(probs, refine=True)
    for rep in range(2):
        clear(probs)
        plan.launch()
        torch.cuda.synchronize()
        check()
    plan.close()
    with pytest.raises(ValueError):
        binding.intersect_batched(make_scenes(k=2)[2], refine=True)


def _curved_scene(args):
    n, seed = args
    return W.curved_scene(n, seed)


def test_batched_full_size_sampled():
    """The uneven batch at its full size: 256 scenes of round(2^U(10, 18))
    pairs (13.1 M in all) with per-segment adaptive depth, in one captured
    plan launch as the benchmark runs it. A seeded sample of 8192 pairs
    across the scenes meets the bar against the depth oracle, and eight
    scenes are bitwise equal to plain calls."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    rng = np.random.default_rng(W.SEED_BASE + 4)
    counts = np.round(2.0 ** rng.uniform(10.0, 18.0, 256)).astype(np.int64)
    jobs = [(int(c), W.SEED_BASE + 4 + 1000 * s) for s, c in enumerate(counts)]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        scenes = list(ex.map(_curved_scene, jobs, chunksize=4))
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    probs = [binding.Problem(g(w.rays), g(w.fibers), 22, None, None, g(w.pair_depth)) for w in scenes]
    say(f"[batched] full size: {len(probs)} scenes, {int(counts.sum())} pairs")
    plan = binding.BatchPlan(probs)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    offs = np.concatenate([[0], np.cumsum(counts)])
    pick = np.sort(np.random.default_rng(9).choice(int(offs[-1]), 8192, replace=False))
    sc = np.searchsorted(offs, pick, side="right") - 1
    t_g = np.empty(len(pick), np.float32)
    u_g = np.empty(len(pick), np.float32)
    h_g = np.empty(len(pick), np.uint8)
    t_o = np.empty(len(pick))
    u_o = np.empty(len(pick))
    h_o = np.empty(len(pick), np.uint8)
    flag = np.empty(len(pick), bool)
    spread = np.empty(len(pick))
    terr = np.empty(len(pick))
    depths = np.empty(len(pick), np.uint8)
    alts = {}
    for s in np.unique(sc):
        sel = np.nonzero(sc == s)[0]
        local = pick[sel] - offs[s]
        ws = scenes[s].subset(local)
        (to, uo, ho), band = oracle_with_band(ws)
        t_g[sel] = probs[s].t.cpu().numpy()[local]
        u_g[sel] = probs[s].u.cpu().numpy()[local]
        h_g[sel] = probs[s].hit.cpu().numpy()[local]
        t_o[sel], u_o[sel], h_o[sel] = to, uo, ho
        flag[sel], spread[sel], terr[sel] = band.flag, band.u_spread, band.t_err
        depths[sel] = ws.pair_depth
        resolver = tie_resolver(ws)
        for k, j in enumerate(sel):
            alts[int(j)] = (resolver, k)
    from parity import Band
    st = compare(t_g, u_g, h_g, t_o, u_o, h_o, Band(flag, spread, terr), depths,
                 alt=lambda i: alts[int(i)][0](alts[int(i)][1]))
    say(f"[batched]   sample: {st}")
    assert st["ok"], st
    for s in np.random.default_rng(3).choice(len(probs), 8, replace=False):
        p = probs[int(s)]
        t, u, h = binding.intersect_pairs(p.rays, p.fibers, 22, pair_depth=p.pair_depth)
        torch.cuda.synchronize()
        assert np.array_equal(bits(p.t.cpu().numpy()), bits(t.cpu().numpy()))
        assert np.array_equal(bits(p.u.cpu().numpy()), bits(u.cpu().numpy()))
        assert np.array_equal(p.hit.cpu().numpy(), h.cpu().numpy())
