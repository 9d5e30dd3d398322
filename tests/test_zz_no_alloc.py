"""fiber_intersect_pairs_noalloc (fiber records of gathered calls in the
library's fixed per-device scratch array) against fiber_intersect_pairs
(records in a caller workspace): bit-for-bit equal results on two gathered
calls in a row, the second with a smaller input, plain and refined, with no
change of the device's free memory across the calls."""
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
    sizes = (300_000, 70_001)                  # fibers per call; the second call is smaller
    w = W.straight_and_curved(sizes[0], 22, seed=1811)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    depth = 22 if refine else 9
    k = 5 if refine else 3
    rng = np.random.default_rng(7)
    # each call gathers its fibers (a permutation, one pair per fiber plus a
    # few repeats), so its records go to the scratch array
    idx = [torch.from_numpy(np.concatenate([rng.permutation(n), rng.integers(0, n, 1000)]).astype(np.int32)).to(DEV)
           for n in sizes]
    m_max = max(int(i.numel()) for i in idx)
    outs = [torch.empty(m_max, device=DEV), torch.empty(m_max, device=DEV),
            torch.empty(m_max, dtype=torch.uint8, device=DEV)]
    if refine:
        outs += [torch.empty(m_max, dtype=torch.float64, device=DEV) for _ in range(2)]
    # first launches of both kernels outside the measured span
    i0 = idx[1][:64].remainder(64).contiguous()
    binding.intersect_pairs_noalloc(rays[:, :64], fibers[:, :64], depth, i0, i0,
                                    out=[o[:64] for o in outs], refine=refine)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = []
    for n, ix in zip(sizes, idx):
        m = int(ix.numel())
        say(f"[noalloc] refine={refine} fibers={n} pairs={m}")
        o = [x[:m] for x in outs]
        binding.intersect_pairs_noalloc(rays[:, :n], fibers[:, :n], depth, ix, ix, out=o, refine=refine)
        torch.cuda.synchronize()
        got.append([x.clone() for x in o])
    assert torch.cuda.mem_get_info()[0] == free0
    for n, ix, g in zip(sizes, idx, got):
        want = binding.intersect_pairs(rays[:, :n], fibers[:, :n], depth, ix, ix, refine=refine)
        torch.cuda.synchronize()
        assert len(want) == k
        _same(g, want)
    # an identity call (no scratch) equals the workspace entry point's
    g = binding.intersect_pairs_noalloc(rays[:, :sizes[1]], fibers[:, :sizes[1]], depth, refine=refine)
    want = binding.intersect_pairs(rays[:, :sizes[1]], fibers[:, :sizes[1]], depth, refine=refine)
    torch.cuda.synchronize()
    _same(g, want)
