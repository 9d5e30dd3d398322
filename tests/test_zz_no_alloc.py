"""fiber_intersect_pairs_noalloc (root slots in the library's fixed
per-device array) against fiber_intersect_pairs (root slots in a caller
workspace): bit-for-bit equal results on two calls in a row, the second with
a smaller input, plain and refined, with no change of the device's free
memory across the calls."""
import numpy as np
import pytest
import torch

from paper_1811_03374_amd import binding
from paper_1811_03374_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def _same(got, want):
    for g, w in zip(got, want):
        assert np.array_equal(_bits(g.cpu().numpy()), _bits(w.cpu().numpy()))


@pytest.mark.parametrize("refine", [False, True])
def test_noalloc_equals_workspace_entry_point(refine):
    binding.lib().fi_init_device()
    sizes = (300_000, 70_001)                  # second call smaller than the first
    w = W.straight_and_curved(sizes[0], 22, seed=1811)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    depth = 22 if refine else 9
    k = 5 if refine else 3
    outs = [torch.empty(sizes[0], device=DEV), torch.empty(sizes[0], device=DEV),
            torch.empty(sizes[0], dtype=torch.uint8, device=DEV)]
    if refine:
        outs += [torch.empty(sizes[0], dtype=torch.float64, device=DEV) for _ in range(2)]
    # first launches of both kernels outside the measured span
    binding.intersect_pairs_noalloc(rays[:, :64], fibers[:, :64], depth,
                                    out=[o[:64] for o in outs], refine=refine)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = []
    for n in sizes:
        say(f"[noalloc] refine={refine} n={n}")
        o = [x[:n] for x in outs]
        binding.intersect_pairs_noalloc(rays[:, :n], fibers[:, :n], depth, out=o, refine=refine)
        torch.cuda.synchronize()
        got.append([x.clone() for x in o])
    assert torch.cuda.mem_get_info()[0] == free0
    for n, g in zip(sizes, got):
        want = binding.intersect_pairs(rays[:, :n], fibers[:, :n], depth, refine=refine)
        torch.cuda.synchronize()
        assert len(want) == k
        _same(g, want)
    # a gathered call (fibers read in place) equals the workspace entry point's
    idx = torch.from_numpy(np.random.default_rng(7).permutation(sizes[1]).astype(np.int32)).to(DEV)
    g = binding.intersect_pairs_noalloc(rays, fibers, depth, idx, idx, refine=refine)
    want = binding.intersect_pairs(rays, fibers, depth, idx, idx, refine=refine)
    torch.cuda.synchronize()
    _same(g, want)
