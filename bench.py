"""Throughput of the per-pair ray/fiber test on one MI355X.

A step is one pass of the whole per-pair path over the 2^20-pair workload
(half straight constant-radius fibers, half curved random-walk fibers with a
linear taper; one ray per fiber aimed for about 50 % hits), once at depth 9
and once at depth 22. Inputs are resident in device memory before timing.

Prints one JSON line (metric, value in Gpairs/s, roofline of the dominant
launch, the FP64 oracle timed on the host as a CPU baseline).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DEPTHS = (9, 22)
N_PAIRS = 1 << 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # the GPU's throughput still rises over the first few tens of steps
    # (8.85 Gpairs/s after 5 warm-up steps, 9.60 after 50, 9.64 after 200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the 2^20-pair line (no normals, hair and batched blocks)")
    ap.add_argument("--workload", choices=("straight_and_curved", "batched", "hair", "degenerate", "candidates",
                                                    "quadratic"),
                    default="straight_and_curved",
                    help="batched: 256 uneven scenes (~13 M pairs, adaptive depth), one graph launch "
                         "against 256 plain launches; hair: precision stress with error report")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for counter runs: one 256 MiB device copy (calibration), then one launch "
                         "per depth, nothing else")
    ap.add_argument("--refine-probe", action="store_true",
                    help="for counter runs: two FP64-refined depth-22 calls on 2^22 hair pairs, "
                         "nothing else")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1811_03374_amd", "csrc", "fiberhit.hip")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(depth):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        return None
    if tr.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return tr.get("bytes_per_launch", {}).get(str(depth))


def _scene(args):
    from paper_1811_03374_amd import workloads as W
    n, seed = args
    return W.curved_scene(n, seed)


def _timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def batched_block(steps, warmup):
    """256 independent scenes of round(2^U(10, 18)) pairs with per-segment
    adaptive depth: autotune, then one captured-graph launch against one
    plain launch per scene, on the same stream. Returns a dict."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    rng = np.random.default_rng(W.SEED_BASE + 4)
    counts = np.round(2.0 ** rng.uniform(10.0, 18.0, 256)).astype(np.int64)
    jobs = [(int(c), W.SEED_BASE + 4 + 1000 * s) for s, c in enumerate(counts)]
    print("batched: generating scenes", file=sys.stderr, flush=True)
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        scenes = list(ex.map(_scene, jobs, chunksize=4))
    print("batched: generated", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(a).to(dev)
    probs = [binding.Problem(g(w.rays), g(w.fibers), 22, None, None, g(w.pair_depth)) for w in scenes]
    total = int(counts.sum())
    best, best_ms = binding.autotune(probs, repeats=2)
    print(f"batched: autotuned {best}", file=sys.stderr, flush=True)
    plan = binding.BatchPlan(probs)
    stream = torch.cuda.current_stream()

    def plain():
        for p in probs:
            binding.intersect_pairs(p.rays, p.fibers, 22, pair_depth=p.pair_depth,
                                    out=(p.t, p.u, p.hit), stream=stream)

    ms_graph = _timed(lambda: plan.launch(stream), steps, warmup, stream)
    ms_plain = _timed(plain, steps, warmup, stream)
    depth_hist = np.bincount(np.concatenate([w.pair_depth for w in scenes]), minlength=23)
    plan.close()
    return {"gpairs_per_s": total / (ms_graph * 1e-3) / 1e9, "graph_launch_ms": ms_graph,
            "plain_launches_ms": ms_plain, "plain_gpairs_per_s": total / (ms_plain * 1e-3) / 1e9,
            "batched_over_plain": ms_plain / ms_graph, "autotuned": best, "autotune_best_ms": best_ms,
            "workload": "256 scenes, round(2^U(10,18)) pairs each, curved random-walk fibers, "
                        "per-segment adaptive depth 2..22",
            "pairs": total, "scenes": 256, "depth_histogram": depth_hist.tolist()}


def bench_batched(args):
    b = batched_block(args.steps, args.warmup)
    line = {
        "metric": "ray-fiber intersections/sec (Gpairs/s), batched uneven scenes",
        "value": b["gpairs_per_s"], "unit": "Gpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["graph_launch_ms"],
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": b["workload"], "pairs": b["pairs"], "scenes": b["scenes"],
                   "depth_histogram": b["depth_histogram"]},
        "graph_launch_ms": b["graph_launch_ms"], "plain_launches_ms": b["plain_launches_ms"],
        "plain_gpairs_per_s": b["plain_gpairs_per_s"], "batched_over_plain": b["batched_over_plain"],
        "autotuned": b["autotuned"], "autotune_best_ms": b["autotune_best_ms"],
    }
    print(json.dumps(line), flush=True)


def refine_probe():
    """Two refined depth-22 calls (the second is the one to read) on the hair
    workload with 2^22 rays: the input of counter runs on the refining
    kernel."""
    import torch
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    w = W.hair_precision(1 << 22, 100_000)
    dev = torch.device("cuda:0")
    rays = torch.from_numpy(w.rays).to(dev)
    fibers = torch.from_numpy(w.fibers).to(dev)
    pf = torch.from_numpy(w.pair_fiber).to(dev)
    for _ in range(2):
        out = binding.intersect_pairs(rays, fibers, 22, pair_fiber=pf, refine=True)
        torch.cuda.synchronize()
    print(json.dumps({"refine_probe": True, "pairs": w.n_pairs,
                      "hit_rate": float(out[2].float().mean().item()),
                      "kernel_source_sha256_16": kernel_source_hash()}))


def hair_block(steps, warmup, cpu=True):
    """The hair configuration in FP32 as one block of the default line: 2^24
    rays against 800,000 segments gathered through an int32 index, at depth
    9 and 22. Per depth: the call time (HIP events around `steps` calls on
    one stream), its roofline from the traversal's counted work, parity on a
    seeded 4,096-pair sample against the depth oracle with the tie
    resolver, and the oracle timed on a 2^14-pair sample."""
    import numpy as np
    import torch
    import oracle
    from paper_1811_03374_amd import binding, workmodel
    from paper_1811_03374_amd import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare, oracle_with_band, tie_resolver

    w = W.hair_precision(1 << 24, 100_000)
    dev = torch.device("cuda:0")
    rays, fibers = torch.from_numpy(w.rays).to(dev), torch.from_numpy(w.fibers).to(dev)
    pf = torch.from_numpy(w.pair_fiber).to(dev)
    n, nf = w.n_pairs, w.fibers.shape[1]
    stream = torch.cuda.current_stream()
    out = {}
    idx = np.sort(np.random.default_rng(11).choice(n, 4096, replace=False))
    ws = w.subset(idx)
    for d in (9, 22):
        _, _, h, cn = binding.intersect_pairs(rays, fibers, d, pair_fiber=pf, counts=True)
        s_ = cn.to(torch.int64).sum(dim=0).cpu().numpy()
        hits = int(h.sum().item())
        fl = workmodel.flops(n, int(s_[0]), int(s_[1]), int(s_[2]), hits)
        by = workmodel.bytes_gathered(n, nf)
        call = binding.PreparedPairs(rays, fibers, d, pair_fiber=pf)
        ms = _timed(lambda: call.launch(stream), steps, warmup, stream)
        t, u, hh = (x.cpu().numpy() for x in call.launch(stream))
        torch.cuda.synchronize()
        (t_o, u_o, h_o), band = oracle_with_band(ws, d)
        st = compare(t[idx], u[idx], hh[idx], t_o, u_o, h_o, band, d, alt=tie_resolver(ws, d))
        tfl = fl / (ms * 1e-3) / 1e12
        out[str(d)] = {"launch_ms_avg": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9,
                       "roofline": {"bound": "alu", "achieved": tfl, "peak": workmodel.PEAK_FP32_TFLOPS,
                                    "unit": "TFLOP/s", "frac": tfl / workmodel.PEAK_FP32_TFLOPS,
                                    "traffic": None, "algorithmic_bytes": by,
                                    "hbm_gbs_algorithmic": by / (ms * 1e-3) / 1e9},
                       "tests_per_pair": int(s_[0]) / n, "hit_rate": hits / n,
                       "parity_sample": {k: st[k] for k in ("ok", "pairs", "flag_disagree_outside_band",
                                                            "max_rel_t", "max_abs_u", "tie_resolved")}}
    cpu_res = None
    if cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        cs = w.subset(np.arange(1 << 21))
        passes, spent = 0, 0.0
        while spent < 3.0 and passes < 100:
            c0 = time.perf_counter()
            for d in (9, 22):
                oracle.intersect_depth(cs.rays, cs.fibers, d, pair_fiber=cs.pair_fiber, nthreads=threads)
            spent += time.perf_counter() - c0
            passes += 1
        cpu_res = {"value": passes * 2 * (1 << 21) / spent / 1e9, "unit": "Gpairs/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"the first 2,097,152 pairs at depths 9 and 22, {passes} times ({spent:.1f} s), "
                             f"FP64 depth-d oracle"}
    return {"workload": "hair: 100k strands x 8 C1 segments (800,000 fibers, +1e3 offset, r 1e-4..2e-5), "
                        "2^24 rays aimed at random segments, 10% grazing within 1e-3 r, fibers gathered "
                        "through an int32 index",
            "pairs": n, "fibers": nf, "bytes_per_pair": 41, "per_depth": out, "cpu_baseline": cpu_res}


def bench_hair(args):
    """Hair-like precision stress: 2^24 rays against 800,000 segments offset
    by 1e3 (10 % grazing within 1e-3 r): throughput of the FP32 search at
    depth 9 and 22 and of the FP64-refined search at 22, and their errors
    against the oracles on a seeded sample of 2^17 pairs."""
    import numpy as np
    import torch
    import oracle
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    print("hair: generating 2^24 rays", file=sys.stderr, flush=True)
    w = W.hair_precision(1 << 24, 100_000)
    print("hair: generated", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    rays, fibers = torch.from_numpy(w.rays).to(dev), torch.from_numpy(w.fibers).to(dev)
    pf = torch.from_numpy(w.pair_fiber).to(dev)
    n = w.n_pairs
    stream = torch.cuda.current_stream()
    res, outs = {}, {}
    for d in (9, 22):
        ms = _timed(lambda: binding.intersect_pairs(rays, fibers, d, pair_fiber=pf, stream=stream),
                    args.steps, args.warmup, stream)
        outs[d] = [o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, d, pair_fiber=pf)]
        res[f"fp32_d{d}"] = {"ms": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9}
    ms = _timed(lambda: binding.intersect_pairs(rays, fibers, 22, pair_fiber=pf, refine=True,
                                                stream=stream), args.steps, args.warmup, stream)
    ref = [o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, 22, pair_fiber=pf, refine=True)]
    res["fp64_refined_d22"] = {"ms": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9}
    print("hair: timed; oracle sample", file=sys.stderr, flush=True)

    idx = np.sort(np.random.default_rng(3).choice(n, 1 << 17, replace=False))
    ws = w.subset(idx)
    P = W.unpack_fibers(ws.fibers)
    valid = np.array([oracle.cubic_constraints(P[i].reshape(16)) == 31 for i in range(P.shape[0])])

    def stats(h, t, u, h_o, t_o, u_o, band):
        h = h.astype(bool)
        h_o = h_o.astype(bool)
        m = ~band & valid
        both = m & h & h_o
        rel = np.abs(t[both] - t_o[both]) / t_o[both]
        return {"pairs": int(m.sum()), "in_band": int(band.sum()),
                "flag_disagree_rate": float((h[m] != h_o[m]).mean()),
                "max_rel_t": float(rel.max()) if rel.size else 0.0,
                "p999_rel_t": float(np.quantile(rel, 0.999)) if rel.size else 0.0,
                "max_abs_u": float(np.abs(u[both] - u_o[both]).max()) if rel.size else 0.0}

    for d in (9, 22):
        t_o, u_o, h_o = oracle.intersect_depth(ws.rays, ws.fibers, d)
        _, _, hl = oracle.intersect_depth(ws.rays, ws.fibers, d, radius_scale=1 - 1e-4)
        _, _, hh = oracle.intersect_depth(ws.rays, ws.fibers, d, radius_scale=1 + 1e-4)
        t, u, h = (a[idx] for a in outs[d])
        res[f"fp32_d{d}"]["vs_depth_oracle"] = stats(h, t, u, h_o, t_o, u_o, hl != hh)
    t_x, u_x, h_x, _ = oracle.intersect_exact(ws.rays, ws.fibers)
    _, _, hl, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 - 1e-4)
    _, _, hh, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 + 1e-4)
    t, u, h = outs[22][0][idx], outs[22][1][idx], outs[22][2][idx]
    res["fp32_d22"]["vs_exact_oracle"] = stats(h, t, u, h_x, t_x, u_x, hl != hh)
    res["fp64_refined_d22"]["vs_exact_oracle"] = stats(ref[2][idx], ref[3][idx], ref[4][idx],
                                                       h_x, t_x, u_x, hl != hh)
    line = {"metric": "ray-fiber intersections/sec (Gpairs/s), hair precision stress",
            "value": res["fp32_d22"]["gpairs_per_s"], "unit": "Gpairs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "f32 (+f64 refinement)",
            "data": "synthetic",
            "config": {"workload": "hair: 100k strands x 8 C1 segments, +1e3 offset, r 1e-4..2e-5, "
                                   "2^24 rays, 10% grazing within 1e-3 r", "pairs": n,
                       "error_sample": int(len(idx)), "valid_in_sample": int(valid.sum())},
            "results": res}
    print(json.dumps(line), flush=True)


def bench_candidates(args):
    """Nearest hit over candidate lists: 2^20 rays over the hair table, each
    with a shuffled list of 6..15 segments of neighbouring strands (about
    10.1M candidates in all), at depth 9 and 22 in FP32 and at 22 with FP64
    refinement; errors against the oracles' nearest hit on a seeded sample of
    4,096 rays."""
    import numpy as np
    import torch
    import oracle
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    w = W.hair_candidates(1 << 20)
    off_np, cand_np = w.meta["cand_off"], w.meta["cand_fiber"]
    dev = torch.device("cuda:0")
    rays, fibers = torch.from_numpy(w.rays).to(dev), torch.from_numpy(w.fibers).to(dev)
    off, cand = torch.from_numpy(off_np).to(dev), torch.from_numpy(cand_np).to(dev)
    n, nc = rays.shape[1], cand.numel()
    mc = int(np.diff(off_np).max())
    stream = torch.cuda.current_stream()
    nb = binding.lib().fiber_candidates_workspace_bytes(nc, fibers.shape[1], 0)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None
    res, outs = {}, {}
    for name, d, ref in (("fp32_d9", 9, False), ("fp32_d22", 22, False), ("fp64_refined_d22", 22, True)):
        def call():
            return binding.intersect_candidates(rays, fibers, off, cand, d, max_candidates=mc, refine=ref,
                                                stream=stream, workspace=ws)
        ms = _timed(call, args.steps, args.warmup, stream)
        outs[name] = [o.cpu().numpy() for o in call()]
        res[name] = {"ms": ms, "grays_per_s": n / (ms * 1e-3) / 1e9,
                     "candidate_tests_per_s_G": nc / (ms * 1e-3) / 1e9,
                     "hit_rate": float(outs[name][2].mean())}
    # errors on a sample of rays (their whole lists)
    idx = np.sort(np.random.default_rng(5).choice(n, 4096, replace=False))
    lists = [cand_np[off_np[i]:off_np[i + 1]] for i in idx]
    so = np.zeros(len(idx) + 1, np.int64)
    np.cumsum([len(x) for x in lists], out=so[1:])
    sc = np.concatenate(lists)
    sr = w.rays[:, idx]
    for name, d in (("fp32_d9", 9), ("fp32_d22", 22)):
        t_o, u_o, h_o, f_o = oracle.intersect_nearest(sr, w.fibers, so, sc, d)
        _, _, hl, _ = oracle.intersect_nearest(sr, w.fibers, so, sc, d, radius_scale=1 - 1e-4)
        _, _, hh, _ = oracle.intersect_nearest(sr, w.fibers, so, sc, d, radius_scale=1 + 1e-4)
        t, u, h, f = (a[idx] for a in outs[name][:4])
        m = hl == hh
        both = m & h.astype(bool) & h_o.astype(bool)
        rel = np.abs(t[both] - t_o[both]) / t_o[both]
        res[name]["vs_depth_oracle"] = {"rays": int(m.sum()),
                                        "flag_disagree": int((h[m] != h_o[m]).sum()),
                                        "fiber_disagree": int((f[both] != f_o[both]).sum()),
                                        "max_rel_t": float(rel.max()) if rel.size else 0.0}
    t_x, u_x, h_x, _, f_x = oracle.nearest_exact(sr, w.fibers, so, sc)
    _, _, hl, _, _ = oracle.nearest_exact(sr, w.fibers, so, sc, radius_scale=1 - 1e-4)
    _, _, hh, _, _ = oracle.nearest_exact(sr, w.fibers, so, sc, radius_scale=1 + 1e-4)
    t64, h, f = outs["fp64_refined_d22"][4][idx], outs["fp64_refined_d22"][2][idx], outs["fp64_refined_d22"][3][idx]
    m = hl == hh
    both = m & h.astype(bool) & h_x.astype(bool)
    rel = np.abs(t64[both] - t_x[both]) / t_x[both]
    res["fp64_refined_d22"]["vs_exact_oracle"] = {"rays": int(m.sum()),
                                                  "flag_disagree": int((h[m] != h_x[m]).sum()),
                                                  "fiber_disagree": int((f[both] != f_x[both]).sum()),
                                                  "max_rel_t": float(rel.max()) if rel.size else 0.0}
    line = {"metric": "nearest hits over candidate lists per second (Grays/s)",
            "value": res["fp32_d22"]["grays_per_s"], "unit": "Grays/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "f32 (+f64 refinement)",
            "data": "synthetic",
            "config": {"workload": "hair candidate lists: 2^20 rays (10% grazing) over 100k strands x 8 "
                                   "segments (+1e3 offset), 6..15 shuffled segments of neighbouring strands "
                                   "per ray", "rays": n, "candidates": nc, "max_candidates": mc,
                       "launch": "one initialising kernel, then one persistent k_fused launch per list "
                                 "position (max_candidates launches)"},
            "results": res}
    print(json.dumps(line), flush=True)


def bench_quadratic(args):
    """Quadratic fibers (Appendix B.1, FI_QUADRATIC): 2^20 pairs of the
    quadratic recipe at depth 9 and 22 in FP32 and at 22 with FP64
    refinement, with the cubic calls on the same curves (their exact
    elevations, as 16-row tables) beside them; errors on a seeded sample of
    4,096 pairs against the depth oracle's quadratic mode, and refined
    against the exact oracle on the quadratics that meet the constraint."""
    import numpy as np
    import torch
    import oracle
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    w = W.quadratic_fibers(1 << 20)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rays, fibers = g(w.rays), g(w.fibers)
    cubic = g(W.pack_fibers(W.elevate_quadratic(W.unpack_quadratics(w.fibers))))
    n = rays.shape[1]
    stream = torch.cuda.current_stream()
    res, outs = {}, {}
    for name, d, ref, tab, quad in (("fp32_d9", 9, False, fibers, True), ("fp32_d22", 22, False, fibers, True),
                                    ("fp64_refined_d22", 22, True, fibers, True),
                                    ("cubic_fp32_d9", 9, False, cubic, False),
                                    ("cubic_fp32_d22", 22, False, cubic, False)):
        def call():
            return binding.intersect_pairs(rays, tab, d, refine=ref, quadratic=quad, stream=stream)
        ms = _timed(call, args.steps, args.warmup, stream)
        outs[name] = [o.cpu().numpy() for o in call()]
        res[name] = {"ms": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9, "hit_rate": float(outs[name][2].mean())}
    idx = np.sort(np.random.default_rng(5).choice(n, 4096, replace=False))
    ws = w.subset(idx)
    for name, d in (("fp32_d9", 9), ("fp32_d22", 22)):
        t_o, u_o, h_o = oracle.intersect_depth(ws.rays, ws.fibers, d, quadratic=True)
        _, _, hl = oracle.intersect_depth(ws.rays, ws.fibers, d, radius_scale=1 - 1e-4, quadratic=True)
        _, _, hh = oracle.intersect_depth(ws.rays, ws.fibers, d, radius_scale=1 + 1e-4, quadratic=True)
        t, u, h = (a[idx] for a in outs[name][:3])
        m = hl == hh
        both = m & h.astype(bool) & h_o.astype(bool)
        rel = np.abs(t[both] - t_o[both]) / t_o[both]
        res[name]["vs_depth_oracle"] = {"pairs": int(m.sum()), "flag_disagree": int((h[m] != h_o[m]).sum()),
                                        "max_rel_t": float(rel.max()) if rel.size else 0.0}
    P = W.unpack_quadratics(ws.fibers)
    valid = np.array([oracle.quadratic_constraint(P[i].reshape(12)) for i in range(P.shape[0])])
    t_x, _, h_x, _ = oracle.intersect_exact(ws.rays, ws.fibers, quadratic=True)
    _, _, hl, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 - 1e-4, quadratic=True)
    _, _, hh, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 + 1e-4, quadratic=True)
    h, t64 = outs["fp64_refined_d22"][2][idx], outs["fp64_refined_d22"][3][idx]
    m = valid & (hl == hh)
    both = m & h.astype(bool) & h_x.astype(bool)
    rel = np.abs(t64[both] - t_x[both]) / t_x[both]
    res["fp64_refined_d22"]["vs_exact_oracle"] = {"valid_pairs": int(m.sum()),
                                                  "flag_disagree": int((h[m] != h_x[m]).sum()),
                                                  "max_rel_t": float(rel.max()) if rel.size else 0.0}
    line = {"metric": "ray-fiber intersections/sec (Gpairs/s), quadratic fibers",
            "value": res["fp32_d22"]["gpairs_per_s"], "unit": "Gpairs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "f32 (+f64 refinement)",
            "data": "synthetic",
            "config": {"workload": "quadratic Bezier fibers: 2^20 pairs, chords 0.2..0.8, middle point "
                                   "displaced up to 0.45 chord (a quarter straight), radius 0.002..0.02, "
                                   "about half hit", "pairs": n},
            "results": res}
    print(json.dumps(line), flush=True)


def bench_degenerate(args):
    """Degenerate-geometry batch: 2^22 pairs in four families (cusps,
    near-collinear points, zero end tangents, steep tapers), per-pair depth
    16..22, FP32 and with FP64 refinement. Errors per family on a seeded
    sample of 2^15 pairs: FP32 against the depth oracle at each pair's depth,
    refined against the exact oracle, both outside the 1e-4 r band; curves
    that break the constraints of Section 3.4 (which the paper splits
    beforehand) are counted apart."""
    import numpy as np
    import torch
    import oracle
    from paper_1811_03374_amd import binding
    from paper_1811_03374_amd import workloads as W

    w = W.degenerate_geometry(1 << 22)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rays, fibers, pd = g(w.rays), g(w.fibers), g(w.pair_depth)
    n = w.n_pairs
    stream = torch.cuda.current_stream()
    res = {}
    ms = _timed(lambda: binding.intersect_pairs(rays, fibers, 22, pair_depth=pd, stream=stream),
                args.steps, args.warmup, stream)
    plain = [o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, 22, pair_depth=pd)]
    res["fp32"] = {"ms": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9}
    ms = _timed(lambda: binding.intersect_pairs(rays, fibers, 22, pair_depth=pd, refine=True, stream=stream),
                args.steps, args.warmup, stream)
    ref = [o.cpu().numpy() for o in binding.intersect_pairs(rays, fibers, 22, pair_depth=pd, refine=True)]
    res["fp64_refined"] = {"ms": ms, "gpairs_per_s": n / (ms * 1e-3) / 1e9}
    print("degenerate: timed; oracle sample", file=sys.stderr, flush=True)

    idx = np.sort(np.random.default_rng(5).choice(n, 1 << 15, replace=False))
    ws = w.subset(idx)
    P = W.unpack_fibers(ws.fibers)
    valid = np.array([oracle.cubic_constraints(P[i].reshape(16)) == 31 for i in range(P.shape[0])])
    fam = w.meta["family"][idx]
    t_d, u_d, h_d = oracle.intersect_depth(ws.rays, ws.fibers, pair_depth=ws.pair_depth)
    _, _, hl = oracle.intersect_depth(ws.rays, ws.fibers, pair_depth=ws.pair_depth, radius_scale=1 - 1e-4)
    _, _, hh = oracle.intersect_depth(ws.rays, ws.fibers, pair_depth=ws.pair_depth, radius_scale=1 + 1e-4)
    band_d = hl != hh
    t_x, u_x, h_x, _ = oracle.intersect_exact(ws.rays, ws.fibers)
    _, _, hl, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 - 1e-4)
    _, _, hh, _ = oracle.intersect_exact(ws.rays, ws.fibers, radius_scale=1 + 1e-4)
    band_x = hl != hh
    refined = ws.pair_depth > 16

    def stats(h, t, m, h_o, t_o):
        h, h_o = h.astype(bool), h_o.astype(bool)
        both = m & h & h_o
        rel = np.abs(t[both] - t_o[both]) / np.maximum(np.abs(t_o[both]), 1e-300)   # t = 0: origin inside
        return {"pairs": int(m.sum()), "flag_disagree_rate": float((h[m] != h_o[m]).mean()) if m.any() else 0.0,
                "max_rel_t": float(rel.max()) if rel.size else 0.0,
                "p999_rel_t": float(np.quantile(rel, 0.999)) if rel.size else 0.0}

    names = ("cusp", "near-collinear", "zero tangent", "steep taper")
    for key, (h, t), (h_o, t_o), band, extra in (
            ("fp32", (plain[2][idx], plain[0][idx]), (h_d, t_d), band_d, np.ones(len(idx), bool)),
            ("fp64_refined", (ref[2][idx], ref[3][idx]), (h_x, t_x), band_x, refined)):
        per = {}
        for f, name in enumerate(names):
            for val in (True, False):
                m = (fam == f) & (valid == val) & ~band & extra
                if m.any():
                    per[f"{name}{'' if val else ' (breaks Sec. 3.4 constraints)'}"] = stats(h, t, m, h_o, t_o)
        res[key]["vs_oracle"] = per
    # validation and pre-subdivision of the 2^22-fiber table (Section 3.4)
    mask = binding.validate(fibers)
    ms_v = _timed(lambda: binding.validate(fibers, stream=stream), 5, 1, stream)
    nb = binding.lib().fiber_presplit_workspace_bytes(fibers.shape[1])
    wsp = torch.empty(nb, dtype=torch.uint8, device=dev)
    off = torch.empty(fibers.shape[1] + 1, dtype=torch.int64, device=dev)
    import ctypes as C
    count = lambda: binding.lib().fiber_presplit_count(fibers.data_ptr(), fibers.stride(0), fibers.shape[1], 6,
                                                       off.data_ptr(), C.c_void_p(wsp.data_ptr()), wsp.numel(),
                                                       stream.cuda_stream)
    ms_c = _timed(count, 3, 1, stream)
    t0 = time.perf_counter()
    pieces, pf, u0, u1, mk, off2 = binding.presplit(fibers, 6)
    torch.cuda.synchronize()
    ms_split = (time.perf_counter() - t0) * 1e3
    mask = mask.cpu().numpy()
    fam_all = w.meta["family"]
    npc = np.diff(off2.cpu().numpy())
    mkn = mk.cpu().numpy()
    still = np.logical_or.reduceat(mkn != 0, off2.cpu().numpy()[:-1])
    res["presplit"] = {
        "validate_ms": ms_v, "count_ms": ms_c, "count_and_write_wall_ms": ms_split,
        "fibers": int(fibers.shape[1]), "pieces": int(pieces.shape[1]),
        "per_family": {name: {"valid": float((mask[fam_all == f] == 0).mean()),
                              "mean_pieces": float(npc[fam_all == f].mean()),
                              "still_invalid_at_level_6": float(still[fam_all == f].mean())}
                       for f, name in enumerate(names)}}
    line = {"metric": "ray-fiber intersections/sec (Gpairs/s), degenerate geometry",
            "value": res["fp32"]["gpairs_per_s"], "unit": "Gpairs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "f32 (+f64 refinement)",
            "data": "synthetic",
            "config": {"workload": "degenerate: cusps, near-collinear (jitter 1e-6), zero end tangents, "
                                   "radius ratios to 1000:1; rays along and across the chord; depth 16..22",
                       "pairs": n, "error_sample": int(len(idx)),
                       "refined_sample": "pairs of depth > 16 (shallower pairs keep the FP32 result)"},
            "results": res}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the per-pair test has no cross-GPU step, and "
              "this benchmark runs on a single GPU only (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.refine_probe:
        refine_probe()
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "hair":
        bench_hair(args)
        return
    if args.workload == "degenerate":
        bench_degenerate(args)
        return
    if args.workload == "quadratic":
        bench_quadratic(args)
        return
    if args.workload == "candidates":
        bench_candidates(args)
        return

    import numpy as np
    import torch
    from paper_1811_03374_amd import binding, workmodel
    from paper_1811_03374_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.traffic_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)      # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    w = W.straight_and_curved(N_PAIRS, DEPTHS[0])
    rays = torch.from_numpy(w.rays).to(dev)
    fibers = torch.from_numpy(w.fibers).to(dev)
    n = w.n_pairs
    outs = {d: (torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.uint8, device=dev)) for d in DEPTHS}
    if args.traffic_probe:
        for d in DEPTHS:
            binding.intersect_pairs(rays, fibers, d, out=outs[d])
            torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "kernel_source_sha256_16": kernel_source_hash()}))
        return

    # algorithmic work of each launch (untimed counting pass; same traversal)
    work = {}
    for d in DEPTHS:
        _, _, h, cn = binding.intersect_pairs(rays, fibers, d, counts=True)
        s = cn.to(torch.int64).sum(dim=0).cpu().numpy()
        hits = int(h.sum().item())
        work[d] = {"tests": int(s[0]), "splits": int(s[1]), "backtracks": int(s[2]), "hits": hits,
                   "flops": workmodel.flops(n, int(s[0]), int(s[1]), int(s[2]), hits),
                   "bytes": workmodel.bytes_streamed(n)}
    torch.cuda.synchronize()

    parity = None
    if not args.no_check:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import compare, oracle_with_band, tie_resolver
        idx = np.sort(np.random.default_rng(0).choice(n, 4096, replace=False))
        ws = w.subset(idx)
        parity = {}
        for d in DEPTHS:
            t, u, h = binding.intersect_pairs(rays, fibers, d, out=outs[d])
            torch.cuda.synchronize()
            (t_o, u_o, h_o), band = oracle_with_band(ws, d)
            st = compare(t.cpu().numpy()[idx], u.cpu().numpy()[idx], h.cpu().numpy()[idx],
                         t_o, u_o, h_o, band, d, alt=tie_resolver(ws, d))
            parity[str(d)] = {k: st[k] for k in ("ok", "flag_disagree_outside_band", "max_rel_t",
                                                 "max_abs_u", "tie_resolved")}

    stream = torch.cuda.current_stream()
    # A step's calls (one per depth) are independent: each depth has a
    # stream of its own, on which its calls run in order, the longer one
    # (depth 22) issued first, so that one call's waves fill the SIMDs the
    # other's finishing waves leave empty. The streams fork from the main
    # stream before the steps and join it after them. Per-call figures (per
    # depth, roofline) come from the same calls made one after another on
    # one stream, each between HIP events.
    side = {d: torch.cuda.Stream() for d in DEPTHS}
    order = sorted(DEPTHS, reverse=True)
    # each call checked and marshalled once (binding.PreparedPairs): the
    # timed loop then only enqueues, and the host keeps ahead of the GPU
    call = {d: binding.PreparedPairs(rays, fibers, d, out=outs[d]) for d in DEPTHS}

    def fork():
        for d in order:
            side[d].wait_stream(stream)

    def join():
        for d in order:
            stream.wait_stream(side[d])

    def step():
        for d in order:
            call[d].launch(side[d])

    def isolated_step(ev=None):
        for j, d in enumerate(DEPTHS):
            if ev is not None:
                ev[j][0].record(stream)
            call[d].launch(stream)
            if ev is not None:
                ev[j][1].record(stream)

    fork()
    for _ in range(args.warmup):
        step()
    join()
    for _ in range(args.warmup):
        isolated_step()
    torch.cuda.synchronize()

    # timed region: exactly K steps, device idle on both sides
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fork()
    for k in range(args.steps):
        step()
    join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = len(DEPTHS) * n / (ms_per_step * 1e-3) / 1e9

    # per-call timing: the same K steps with the calls one after another
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in DEPTHS] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        isolated_step(ev[k])
    torch.cuda.synchronize()
    sequential_ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    launch_ms = {d: [ev[k][j][0].elapsed_time(ev[k][j][1]) for k in range(args.steps)]
                 for j, d in enumerate(DEPTHS)}

    # the same calls writing the normal at each hit as well (not part of the
    # step: the cost of the extra output)
    normals = None
    if not args.no_extras:
        ncall = {d: binding.PreparedPairs(rays, fibers, d, normal=True) for d in DEPTHS}
        for _ in range(5):
            for d in DEPTHS:
                ncall[d].launch(stream)
        nev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
                for _ in DEPTHS] for _ in range(args.steps)]
        for k in range(args.steps):
            for j, d in enumerate(DEPTHS):
                nev[k][j][0].record(stream)
                ncall[d].launch(stream)
                nev[k][j][1].record(stream)
        torch.cuda.synchronize()
        nms = {d: statistics.mean(nev[k][j][0].elapsed_time(nev[k][j][1]) for k in range(args.steps))
               for j, d in enumerate(DEPTHS)}
        normals = {str(d): {"launch_ms_avg": nms[d], "gpairs_per_s": n / (nms[d] * 1e-3) / 1e9} for d in DEPTHS}

    per_depth = {}
    roof = {}
    for d in DEPTHS:
        avg = statistics.mean(launch_ms[d])
        tflops = work[d]["flops"] / (avg * 1e-3) / 1e12
        gbs = work[d]["bytes"] / (avg * 1e-3) / 1e9
        per_depth[str(d)] = {
            "gpairs_per_s": n / (avg * 1e-3) / 1e9,
            "launch_ms_avg": avg,
            "launch_ms_median": statistics.median(launch_ms[d]),
            "algorithmic_tflops": tflops,
            "frac_fp32_peak": tflops / workmodel.PEAK_FP32_TFLOPS,
            "hbm_gbs_algorithmic": gbs,
            "frac_hbm_peak": gbs / workmodel.PEAK_HBM_GBS,
            "tests_per_pair": work[d]["tests"] / n,
            "splits_per_pair": work[d]["splits"] / n,
            "backtracks_per_pair": work[d]["backtracks"] / n,
            "hit_rate": work[d]["hits"] / n,
            "flops_per_launch": work[d]["flops"],
        }
        roof[d] = {"bound": "alu", "achieved": tflops, "peak": workmodel.PEAK_FP32_TFLOPS,
                   "unit": "TFLOP/s", "frac": tflops / workmodel.PEAK_FP32_TFLOPS,
                   "traffic": measured_traffic(d), "kernel": "k_fused (one call)", "depth": d,
                   "algorithmic_bytes": work[d]["bytes"],
                   # the same against the peak without packed FP32 (not used here)
                   "frac_unpacked": tflops / workmodel.PEAK_FP32_UNPACKED_TFLOPS}
    dominant = max(DEPTHS, key=lambda d: statistics.mean(launch_ms[d]))
    step_flops = sum(work[d]["flops"] for d in DEPTHS)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        # passes over the whole workload until about 10 s of CPU time have run
        passes, spent = 0, 0.0
        while spent < 10.0 and passes < 1000:
            c0 = time.perf_counter()
            for d in DEPTHS:
                oracle.intersect_depth(w.rays, w.fibers, d, nthreads=threads)
            spent += time.perf_counter() - c0
            passes += 1
        cpu = {"value": passes * len(DEPTHS) * n / spent / 1e9, "unit": "Gpairs/s", "cores": threads,
               "kind": "oracle",
               "sample": f"the whole workload ({n} pairs at depths {list(DEPTHS)}) {passes} times "
                         f"({spent:.1f} s), FP64 depth-d oracle, OpenMP over pairs"}
        # one core on the first 2^16 pairs, and the host CPU's model
        sub = w.subset(np.arange(1 << 16))
        c0 = time.perf_counter()
        for d in DEPTHS:
            oracle.intersect_depth(sub.rays, sub.fibers, d, pair_ray=sub.pair_ray, pair_fiber=sub.pair_fiber,
                                   nthreads=1)
        one = time.perf_counter() - c0
        cpu["single_core"] = {"value": len(DEPTHS) * (1 << 16) / one / 1e9, "unit": "Gpairs/s",
                              "sample": f"the first 65,536 pairs at depths {list(DEPTHS)} ({one:.2f} s), one thread"}
        cpu["cpu_model"] = cpu_model()

    line = {
        "metric": "ray-fiber intersections/sec (Gpairs/s) at depth 9 and 22",
        "value": value, "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "straight_and_curved 2^20 pairs (half straight constant-radius, "
                               "half curved random-walk, ~50% hits)",
                   "pairs": n, "depths": list(DEPTHS), "pairing": "identity",
                   "launch": "per call: k_fused (persistent 64-lane waves, each draining an even share of "
                             "the pairs: FP64 frame and root test in the lane refill, then the FP32 "
                             "subdivision search); a step's two calls on two streams",
                   "sequential_ms_per_step": sequential_ms_per_step,
                   "sequential_gpairs_per_s": len(DEPTHS) * n / (sequential_ms_per_step * 1e-3) / 1e9},
        "per_depth": per_depth,
        "roofline": roof[dominant],
        "step_roofline": {
            "bound": "alu", "unit": "TFLOP/s", "peak": workmodel.PEAK_FP32_TFLOPS,
            "achieved": step_flops / (ms_per_step * 1e-3) / 1e12,
            "frac": step_flops / (ms_per_step * 1e-3) / 1e12 / workmodel.PEAK_FP32_TFLOPS,
            "what": "both calls' algorithmic flops over the step time (calls overlapped on two streams)"},
        "cpu_baseline": cpu,
        "parity": parity,
        "with_normals": normals,
    }
    if not args.no_extras:
        # the other configurations: hair (gathered fibers) and batched scenes
        print("bench: hair block", file=sys.stderr, flush=True)
        line["hair"] = hair_block(args.steps, min(args.warmup, 10), cpu=not args.no_cpu_baseline)
        print("bench: batched block", file=sys.stderr, flush=True)
        line["batched"] = batched_block(min(args.steps, 20), min(args.warmup, 5))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
