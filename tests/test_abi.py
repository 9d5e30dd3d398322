"""C-ABI library checks that need no GPU: it loads, exports every function the
header declares, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1811_03374_amd import binding, build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fiberhit.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    names = declared_functions()
    assert {"fiber_intersect_pairs", "fiber_intersect_counts", "fi_version", "fi_strerror"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", build_lib.LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = binding.lib()
    for n in names:
        assert hasattr(L, n)
    assert set(binding.exported_symbols()) <= exported


def test_version_and_strerror():
    L = binding.lib()
    assert L.fi_version() > 0
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert len(L.fi_strerror(code)) > 0


def _call(**kw):
    a = dict(rays=1, rs=8, nr=8, fibers=1, fs=8, nf=8, pr=None, pf=None, pd=None,
             depth=9, n=8, flags=0, t=1, u=1, h=1, ws=None, wsb=0)
    a.update(kw)
    vp = lambda x: None if x is None else C.c_void_p(x)
    return binding.lib().fiber_intersect_pairs(
        vp(a["rays"]), a["rs"], a["nr"], vp(a["fibers"]), a["fs"], a["nf"], vp(a["pr"]),
        vp(a["pf"]), vp(a["pd"]), a["depth"], a["n"], a["flags"], vp(a["t"]), vp(a["u"]),
        vp(a["h"]), vp(a.get("t64")), vp(a.get("u64")), vp(a.get("nrm")), vp(a["ws"]), a["wsb"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(depth=24), -2), (dict(depth=-1), -2), (dict(n=-1), -2), (dict(flags=8), -2),
    (dict(rs=4), -2), (dict(fs=4), -2), (dict(n=9), -2),
    (dict(rays=None), -1), (dict(fibers=None), -1), (dict(t=None), -1), (dict(h=None), -1),
    (dict(flags=1), -1), (dict(flags=1, t64=1), -1), (dict(flags=9, t64=1, u64=1), -2),
    # a misaligned workspace is refused before any HIP call
    (dict(ws=0x1008, wsb=1 << 30), -4), (dict(flags=2, ws=0x1010, wsb=64), -4),
    (dict(flags=3, t64=1, u64=1, ws=0x1001, wsb=64), -4),
])
def test_argument_errors_before_launch(kw, code):
    # these return before any HIP call, so they are safe without a device
    assert _call(**kw) == code


def test_empty_batch_is_a_no_op():
    assert _call(n=0, rays=None, fibers=None, t=None, u=None, h=None) == 0


def test_counts_requires_output():
    L = binding.lib()
    r = L.fiber_intersect_counts(C.c_void_p(1), 8, 8, C.c_void_p(1), 8, 8, None, None, None,
                                 9, 8, 0, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), None, None, 0, None)
    assert r == -1
    r = L.fiber_intersect_counts(C.c_void_p(1), 8, 8, C.c_void_p(1), 8, 8, None, None, None,
                                 9, 8, 1, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), None,
                                 0, None)
    assert r == -2


def test_pair_count_rejects_mismatched_lengths():
    """Per-pair tensors of different lengths, or an identity pairing longer
    than its table, are refused by the binding before any launch (the C ABI
    cannot check a device array's length)."""
    import torch
    rays = torch.zeros(7, 300)
    fibers = torch.zeros(16, 200)
    i = torch.zeros(150, dtype=torch.int32)
    d = torch.zeros(150, dtype=torch.uint8)
    assert binding._pair_count(rays, fibers, None, None, None) == 200
    assert binding._pair_count(rays, fibers, i, i, d) == 150
    assert binding._pair_count(rays, fibers, None, None, d) == 150
    with pytest.raises(ValueError):
        binding._pair_count(rays, fibers, i, i[:149], None)
    with pytest.raises(ValueError):
        binding._pair_count(rays, fibers, i, None, d[:10])
    with pytest.raises(ValueError):
        binding._pair_count(rays, fibers, None, None, torch.zeros(250, dtype=torch.uint8))
    with pytest.raises(ValueError):
        binding._pair_count(rays[:, :100], fibers, None, i, None)


def test_workspace_sizes():
    """The single-call workspace holds the fiber records of a gathered call
    (64 bytes per fiber, 256-byte aligned) and is empty otherwise; the
    batched workspace holds the scene table. Neither needs a device."""
    L = binding.lib()
    L.fiber_batched_workspace_bytes.argtypes = [C.c_int32, C.c_int64]
    L.fiber_batched_workspace_bytes.restype = C.c_size_t
    assert L.fiber_pairs_workspace_bytes(1000, 1000, 1, 0) == 64000
    assert L.fiber_pairs_workspace_bytes(1001, 1001, 1, 0) == (1001 * 64 + 255) // 256 * 256
    assert L.fiber_pairs_workspace_bytes(1000, 1000, 0, 0) == 0
    assert L.fiber_pairs_workspace_bytes(999, 1000, 1, 0) == 0       # fewer pairs than fibers: in place
    assert L.fiber_pairs_workspace_bytes(-1, 10, 1, 0) == 0
    assert L.fiber_batched_workspace_bytes(10, 1 << 20) > 0


def test_noalloc_refuses_more_records_than_its_scratch():
    """A gathered call whose fiber records exceed the 32 MiB scratch of the
    no-allocation entry point is refused before any HIP call."""
    L = binding.lib()
    n = 600_000
    r = L.fiber_intersect_pairs_noalloc(C.c_void_p(256), n, n, C.c_void_p(256), n, n, None,
                                        C.c_void_p(256), None, 9, n, 0, C.c_void_p(256), C.c_void_p(256),
                                        C.c_void_p(256), None, None, None, None)
    assert r == -5
