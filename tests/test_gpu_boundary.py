"""The single-call boundary: caller-sized workspaces, no device allocation
on the call path, and argument checks of the binding."""
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


def test_device_memory_unchanged_across_growing_calls():
    """With the workspace and outputs passed in, calls of growing size (plain,
    gathered, refined, counting) leave the device's free memory unchanged:
    the library allocates and frees nothing on the call path."""
    n_max = 1 << 19
    w = W.straight_and_curved(n_max, 22)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    idx = torch.arange(n_max, dtype=torch.int32, device=DEV).flip(0).contiguous()
    ws = binding.pairs_workspace(n_max, n_max, True, torch.device(DEV))
    outs = (torch.empty(n_max, device=DEV), torch.empty(n_max, device=DEV),
            torch.empty(n_max, dtype=torch.uint8, device=DEV))

    def calls(n):
        o = tuple(x[:n] for x in outs)
        binding.intersect_pairs(rays, fibers, 9, out=o, workspace=ws, pair_ray=idx[:n], pair_fiber=idx[:n])
        binding.intersect_pairs(rays[:, :n], fibers[:, :n], 22, out=o, workspace=ws)

    calls(64)                               # first launches (code objects, kernel scratch)
    binding.intersect_pairs(rays[:, :64], fibers[:, :64], 22, refine=True, workspace=ws)
    binding.intersect_pairs(rays[:, :64], fibers[:, :64], 9, counts=True, workspace=ws)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for n in (1000, 1 << 14, 100_003, 1 << 19):
        say(f"[boundary] n={n}")
        calls(n)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
    # the results with the caller's workspace equal those of per-call workspaces
    t, u, h = (x.cpu().numpy() for x in binding.intersect_pairs(rays, fibers, 22))
    assert np.array_equal(_bits(outs[0].cpu().numpy()), _bits(t))
    assert np.array_equal(_bits(outs[1].cpu().numpy()), _bits(u))
    assert np.array_equal(outs[2].cpu().numpy(), h)


def test_workspace_without_room_for_records():
    """A gathered call whose workspace holds only the root slots reads the
    fiber rows in place: same results, bit for bit."""
    n = 50_000
    w = W.straight_and_curved(n, 9)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    idx = torch.from_numpy(np.random.default_rng(3).permutation(n).astype(np.int32)).to(DEV)
    full = binding.pairs_workspace(n, n, True, torch.device(DEV))
    slots_only = binding.pairs_workspace(n, n, False, torch.device(DEV))
    assert full.numel() > slots_only.numel()
    a = [x.cpu().numpy() for x in binding.intersect_pairs(rays, fibers, 9, idx, idx, workspace=full)]
    b = [x.cpu().numpy() for x in binding.intersect_pairs(rays, fibers, 9, idx, idx, workspace=slots_only)]
    for x, y in zip(a, b):
        assert np.array_equal(_bits(x), _bits(y))


def test_workspace_errors():
    w = W.straight_and_curved(256, 9)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    small = torch.empty(4096, dtype=torch.uint8, device=DEV)
    with pytest.raises(binding.FiberHitError):
        binding.intersect_pairs(rays, fibers, 9, workspace=small)
    ws = binding.pairs_workspace(256, 256, False, torch.device(DEV))
    with pytest.raises(binding.FiberHitError):          # not 256-byte aligned
        binding.intersect_pairs(rays, fibers, 9, workspace=ws[16:])


def test_mismatched_per_pair_lengths_rejected_before_launch():
    w = W.straight_and_curved(256, 9)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    i = torch.arange(256, dtype=torch.int32, device=DEV)
    d = torch.full((200,), 9, dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):
        binding.intersect_pairs(rays, fibers, 9, i, i[:100])
    with pytest.raises(ValueError):
        binding.intersect_pairs(rays, fibers, 9, i, None, d)
    with pytest.raises(ValueError):
        binding.PreparedPairs(rays, fibers, 9, None, i[:10], d)
    with pytest.raises(ValueError):
        binding.Problem(rays, fibers, 9, i, i, d)
    with pytest.raises(ValueError):                      # identity pairing longer than the rays
        binding.intersect_pairs(rays[:, :100], fibers, 9, None, None, d)
