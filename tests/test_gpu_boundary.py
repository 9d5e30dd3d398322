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
    assert ws is not None
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
    """A gathered call without a workspace, or with one too small for the
    fiber records, reads the fiber rows in place: same results, bit for
    bit."""
    n = 50_000
    w = W.straight_and_curved(n, 9)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    idx = torch.from_numpy(np.random.default_rng(3).permutation(n).astype(np.int32)).to(DEV)
    full = binding.pairs_workspace(n, n, True, torch.device(DEV))
    assert full is not None and full.numel() == n * 64
    assert binding.pairs_workspace(n, n, False, torch.device(DEV)) is None
    small = torch.empty(4096, dtype=torch.uint8, device=DEV)
    a = [x.cpu().numpy() for x in binding.intersect_pairs(rays, fibers, 9, idx, idx, workspace=full)]
    for ws in (small, None):
        lib = binding.lib()
        t, u, h = (torch.empty(n, device=DEV), torch.empty(n, device=DEV),
                   torch.empty(n, dtype=torch.uint8, device=DEV))
        st = lib.fiber_intersect_pairs(rays.data_ptr(), rays.stride(0), n, fibers.data_ptr(), fibers.stride(0), n,
                                       idx.data_ptr(), idx.data_ptr(), None, 9, n, 0, t.data_ptr(), u.data_ptr(),
                                       h.data_ptr(), None, None, None, None if ws is None else ws.data_ptr(),
                                       0 if ws is None else ws.numel(),
                                       torch.cuda.current_stream().cuda_stream)
        assert st == 0
        torch.cuda.synchronize()
        for x, y in zip(a, (t, u, h)):
            assert np.array_equal(_bits(x), _bits(y.cpu().numpy()))


def test_workspace_errors():
    n = 256
    w = W.straight_and_curved(n, 9)
    rays = torch.from_numpy(w.rays).to(DEV)
    fibers = torch.from_numpy(w.fibers).to(DEV)
    idx = torch.arange(n, dtype=torch.int32, device=DEV)
    ws = binding.pairs_workspace(n, n, True, torch.device(DEV))
    with pytest.raises(binding.FiberHitError):          # not 256-byte aligned
        binding.intersect_pairs(rays, fibers, 9, idx, idx, workspace=ws[16:])


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
