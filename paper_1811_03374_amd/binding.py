"""Thin ctypes binding of the fiberhit C ABI (``include/fiberhit.h``).

Argument marshalling only: torch device tensors in, device pointers and the
current HIP stream out to the library. Every step of the intersection runs in
the HIP kernels; there is no host fallback, and a missing library is an error.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

from . import build_lib

FI_OK = 0
FI_ERR_RANGE = -2
FI_MAX_DEPTH = 23
FI_FP64_REFINE = 1
FI_COMPENSATED_PROJ = 2
FI_QUADRATIC = 4

_lib = None


class FiberHitError(RuntimeError):
    pass


def lib():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(build_lib.LIB):
            raise FiberHitError(
                f"HIP library {build_lib.LIB} is not built; run __graft_entry__.build()")
        L = C.CDLL(build_lib.LIB)
        i64, vp, u32, i32 = C.c_int64, C.c_void_p, C.c_uint32, C.c_int32
        common = [vp, i64, i64, vp, i64, i64, vp, vp, vp, i32, i64, u32, vp, vp, vp]
        L.fiber_intersect_pairs.argtypes = common + [vp, vp, vp, vp, C.c_size_t, vp]
        L.fiber_intersect_pairs.restype = C.c_int
        L.fiber_intersect_pairs_noalloc.argtypes = common + [vp, vp, vp, vp]
        L.fiber_intersect_pairs_noalloc.restype = C.c_int
        L.fiber_intersect_counts.argtypes = common + [vp, vp, C.c_size_t, vp]
        L.fiber_intersect_counts.restype = C.c_int
        L.fiber_pairs_workspace_bytes.argtypes = [i64, i64, i32, u32]
        L.fiber_pairs_workspace_bytes.restype = C.c_size_t
        L.fiber_candidates_workspace_bytes.argtypes = [i64, i64, u32]
        L.fiber_candidates_workspace_bytes.restype = C.c_size_t
        L.fiber_intersect_candidates.argtypes = [vp, i64, i64, vp, i64, i64, vp, vp, vp, i32, i32, i64, u32,
                                                 vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.fiber_intersect_candidates.restype = C.c_int
        L.fiber_validate.argtypes = [vp, i64, i64, vp, vp, vp]
        L.fiber_validate.restype = C.c_int
        L.fiber_presplit_workspace_bytes.argtypes = [i64]
        L.fiber_presplit_workspace_bytes.restype = C.c_size_t
        L.fiber_presplit_count.argtypes = [vp, i64, i64, i32, vp, vp, C.c_size_t, vp]
        L.fiber_presplit_count.restype = C.c_int
        L.fiber_presplit.argtypes = [vp, i64, i64, i32, vp, i64, vp, i64, vp, vp, vp, vp, vp]
        L.fiber_presplit.restype = C.c_int
        L.fi_init_device.restype = C.c_int
        L.fi_strerror.argtypes = [C.c_int]
        L.fi_strerror.restype = C.c_char_p
        L.fi_version.restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    return ["fi_version", "fi_strerror", "fi_init_device", "fiber_pairs_workspace_bytes",
            "fiber_intersect_pairs", "fiber_intersect_pairs_noalloc", "fiber_intersect_counts",
            "fiber_candidates_workspace_bytes", "fiber_intersect_candidates",
            "fiber_validate", "fiber_presplit_workspace_bytes", "fiber_presplit_count", "fiber_presplit",
            "fiber_batched_workspace_bytes", "fiber_intersect_batched", "fiber_batch_plan_create",
            "fiber_batch_plan_launch", "fiber_batch_plan_tuning", "fiber_batch_plan_destroy",
            "fiber_batch_autotune", "fiber_tuning_save", "fiber_tuning_load", "fiber_tuning_lookup",
            "fiber_tuning_clear"]


def _check(status: int):
    if status != FI_OK:
        raise FiberHitError(f"fiberhit error {status}: {lib().fi_strerror(status).decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _table(t: torch.Tensor, rows: int, name: str):
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != rows:
        raise ValueError(f"{name} must be a float32 tensor of shape ({rows}, n)")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.shape[1] > 0 and t.stride(1) != 1:
        raise ValueError(f"{name} rows must be contiguous")
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def _index(t: Optional[torch.Tensor], dtype, name: str):
    if t is None:
        return None
    if t.dtype != dtype or t.dim() != 1 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D {dtype} device tensor")
    return t


def _pair_count(rays, fibers, pr, pf, pd):
    """Number of pairs of a call, with every given per-pair tensor of exactly
    that length (the C ABI cannot check the length of a device array)."""
    given = [(name, x) for name, x in (("pair_ray", pr), ("pair_fiber", pf), ("pair_depth", pd))
             if x is not None]
    if given:
        n = given[0][1].shape[0]
        for name, x in given:
            if x.shape[0] != n:
                raise ValueError(f"{name} has {x.shape[0]} elements, expected {n} "
                                 f"(all per-pair tensors must have the same length)")
    else:
        n = min(rays.shape[1], fibers.shape[1])
    if pr is None and n > rays.shape[1]:
        raise ValueError(f"identity ray pairing: {n} pairs but only {rays.shape[1]} rays")
    if pf is None and n > fibers.shape[1]:
        raise ValueError(f"identity fiber pairing: {n} pairs but only {fibers.shape[1]} fibers")
    return n


def _outs(out, n: int, dev):
    """Output tensors (t, u, hit) for n pairs: new ones, or the caller's after
    a check that the kernel cannot write past them."""
    if out is None:
        return (torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.uint8, device=dev))
    t, u, hit = out
    for x, dt, name in ((t, torch.float32, "t"), (u, torch.float32, "u"), (hit, torch.uint8, "hit")):
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous() or x.numel() < n:
            raise ValueError(f"out {name} must be a contiguous {dt} device tensor of at least {n} elements")
    return t, u, hit


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def pairs_workspace(n: int, n_fibers: int, gathered: bool, device) -> Optional[torch.Tensor]:
    """Device workspace of one fiber_intersect_pairs call (the fiber records
    of a gathered call), sized by the library; None when the call needs
    none."""
    nbytes = lib().fiber_pairs_workspace_bytes(int(n), int(n_fibers), int(bool(gathered)), 0)
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _keep_for(ws: Optional[torch.Tensor], stream):
    """A workspace freed after a call on another stream than the current one
    must not be reused by the allocator before that stream passes the call."""
    if ws is not None and stream is not None and stream != torch.cuda.current_stream(ws.device):
        ws.record_stream(stream)


def _ws_args(ws: Optional[torch.Tensor]):
    return (None, 0) if ws is None else (C.c_void_p(ws.data_ptr()), ws.numel())


def _normal_tensor(normal, n, dev):
    """The (3, n) float32 normal rows: None for none, True to allocate, or a
    caller's tensor (checked)."""
    if normal is None or normal is False:
        return None
    if normal is True:
        return torch.empty((3, n), dtype=torch.float32, device=dev)
    if (normal.dtype != torch.float32 or not normal.is_cuda or not normal.is_contiguous()
            or normal.dim() != 2 or normal.shape[0] != 3 or normal.shape[1] != n):
        raise ValueError(f"normal must be a contiguous (3, {n}) float32 device tensor")
    return normal


def intersect_pairs(rays: torch.Tensor, fibers: torch.Tensor, depth: int = 9,
                    pair_ray: Optional[torch.Tensor] = None,
                    pair_fiber: Optional[torch.Tensor] = None,
                    pair_depth: Optional[torch.Tensor] = None,
                    out=None, counts: bool = False, refine: bool = False, stream=None,
                    workspace: Optional[torch.Tensor] = None, normal=None, quadratic: bool = False):
    """Nearest hit (t, u, hit) of every (ray, fiber) pair at subdivision depth
    ``depth`` (or per-pair ``pair_depth``). See ``fiber_intersect_pairs``.

    rays: (7, n_rays) float32; fibers: (16, n_fibers) float32; indices int32.
    Returns (t, u, hit) device tensors, plus an (n, 4) int32 tensor of node
    tests / splits / backtracks / leaf level when ``counts`` is set, or the
    float64 (t64, u64) of the FP64 surface refinement when ``refine`` is set,
    then the (3, n) float32 normals when ``normal`` is True (or a tensor to
    fill). ``workspace`` (uint8 device tensor, see ``pairs_workspace``) is
    allocated per call when not given and the call gathers fibers.
    ``quadratic``: fibers is a (12, n) table of quadratic curves."""
    rs = _table(rays, 7, "rays")
    fs = _table(fibers, 12 if quadratic else 16, "fibers")
    pr = _index(pair_ray, torch.int32, "pair_ray")
    pf = _index(pair_fiber, torch.int32, "pair_fiber")
    pd = _index(pair_depth, torch.uint8, "pair_depth")
    n = _pair_count(rays, fibers, pr, pf, pd)
    dev = rays.device
    t, u, hit = _outs(out, n, dev)
    if counts and refine:
        raise ValueError("counts and refine are separate passes")
    if counts and normal not in (None, False):
        raise ValueError("counts and normals are separate passes")
    nrm = _normal_tensor(normal, n, dev)
    if workspace is None:
        workspace = None if quadratic else pairs_workspace(n, fibers.shape[1], pf is not None, dev)
        _keep_for(workspace, stream)
    elif workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 device tensor")
    ws = _ws_args(workspace)
    cn = torch.empty((n, 4), dtype=torch.int32, device=dev) if counts else None
    flags = (FI_FP64_REFINE if refine else 0) | (FI_QUADRATIC if quadratic else 0)
    args = [_ptr(rays), rs, rays.shape[1], _ptr(fibers), fs, fibers.shape[1],
            _ptr(pr), _ptr(pf), _ptr(pd), int(depth), n, flags,
            _ptr(t), _ptr(u), _ptr(hit)]
    if counts:
        _check(lib().fiber_intersect_counts(*args, _ptr(cn), *ws, _stream(stream)))
        return t, u, hit, cn
    extra = (nrm,) if nrm is not None else ()
    if refine:
        t64 = torch.empty(n, dtype=torch.float64, device=dev)
        u64 = torch.empty(n, dtype=torch.float64, device=dev)
        _check(lib().fiber_intersect_pairs(*args, _ptr(t64), _ptr(u64), _ptr(nrm), *ws, _stream(stream)))
        return (t, u, hit, t64, u64) + extra
    _check(lib().fiber_intersect_pairs(*args, None, None, _ptr(nrm), *ws, _stream(stream)))
    return (t, u, hit) + extra


def intersect_pairs_noalloc(rays: torch.Tensor, fibers: torch.Tensor, depth: int = 9,
                            pair_ray: Optional[torch.Tensor] = None,
                            pair_fiber: Optional[torch.Tensor] = None,
                            pair_depth: Optional[torch.Tensor] = None,
                            out=None, refine: bool = False, stream=None, normal=None,
                            quadratic: bool = False):
    """``intersect_pairs`` through ``fiber_intersect_pairs_noalloc``: no
    workspace (the library's fixed per-device array holds the fiber records
    of gathered calls). With ``out`` (and, under ``refine``, ``out`` holding
    five tensors; ``normal`` a tensor when normals are asked for) the call
    allocates nothing. Calls on one device must not overlap."""
    rs = _table(rays, 7, "rays")
    fs = _table(fibers, 12 if quadratic else 16, "fibers")
    pr = _index(pair_ray, torch.int32, "pair_ray")
    pf = _index(pair_fiber, torch.int32, "pair_fiber")
    pd = _index(pair_depth, torch.uint8, "pair_depth")
    n = _pair_count(rays, fibers, pr, pf, pd)
    dev = rays.device
    t64 = u64 = None
    if refine:
        if out is not None:
            if len(out) != 5:
                raise ValueError("a refined call takes out=(t, u, hit, t64, u64)")
            t64, u64 = out[3], out[4]
            for x, name in ((t64, "t64"), (u64, "u64")):
                if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() < n:
                    raise ValueError(f"out {name} must be a contiguous float64 device tensor of at least {n} elements")
            out = out[:3]
        else:
            t64 = torch.empty(n, dtype=torch.float64, device=dev)
            u64 = torch.empty(n, dtype=torch.float64, device=dev)
    t, u, hit = _outs(out, n, dev)
    nrm = _normal_tensor(normal, n, dev)
    _check(lib().fiber_intersect_pairs_noalloc(
        _ptr(rays), rs, rays.shape[1], _ptr(fibers), fs, fibers.shape[1], _ptr(pr), _ptr(pf), _ptr(pd),
        int(depth), n, (FI_FP64_REFINE if refine else 0) | (FI_QUADRATIC if quadratic else 0), _ptr(t), _ptr(u),
        _ptr(hit), _ptr(t64), _ptr(u64), _ptr(nrm), _stream(stream)))
    extra = (nrm,) if nrm is not None else ()
    return ((t, u, hit, t64, u64) if refine else (t, u, hit)) + extra


def intersect_candidates(rays: torch.Tensor, fibers: torch.Tensor, offsets: torch.Tensor,
                         cand_fiber: torch.Tensor, depth: int = 9,
                         cand_depth: Optional[torch.Tensor] = None, max_candidates: Optional[int] = None,
                         refine: bool = False, normal=None, stream=None,
                         workspace: Optional[torch.Tensor] = None):
    """Nearest hit of each ray over its candidate list (see
    ``fiber_intersect_candidates``): ``offsets`` (n_rays + 1) int64 CSR over
    ``cand_fiber`` int32 (and optional per-candidate uint8 ``cand_depth``).
    Returns (t, u, hit, fiber) device tensors, then (t64, u64) when
    ``refine``, then the (3, n_rays) normals when ``normal``. Without
    ``max_candidates`` the longest list is measured (one device sync)."""
    rs = _table(rays, 7, "rays")
    fs = _table(fibers, 16, "fibers")
    n = rays.shape[1]
    off = _index(offsets, torch.int64, "offsets")
    cf = _index(cand_fiber, torch.int32, "cand_fiber")
    cd = _index(cand_depth, torch.uint8, "cand_depth")
    if off is None or off.numel() != n + 1:
        raise ValueError(f"offsets must hold n_rays + 1 = {n + 1} entries")
    if cf is None:
        raise ValueError("cand_fiber is required")
    if cd is not None and cd.numel() != cf.numel():
        raise ValueError("cand_depth must hold one depth per candidate")
    if max_candidates is None:
        max_candidates = int((off[1:] - off[:-1]).max().item()) if n else 0
    dev = rays.device
    t = torch.empty(n, dtype=torch.float32, device=dev)
    u = torch.empty(n, dtype=torch.float32, device=dev)
    hit = torch.empty(n, dtype=torch.uint8, device=dev)
    fib = torch.empty(n, dtype=torch.int32, device=dev)
    t64 = torch.empty(n, dtype=torch.float64, device=dev) if refine else None
    u64 = torch.empty(n, dtype=torch.float64, device=dev) if refine else None
    nrm = _normal_tensor(normal, n, dev)
    if workspace is None:
        nb = lib().fiber_candidates_workspace_bytes(int(cf.numel()), int(fibers.shape[1]), 0)
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None
        _keep_for(workspace, stream)
    ws = _ws_args(workspace)
    _check(lib().fiber_intersect_candidates(
        _ptr(rays), rs, n, _ptr(fibers), fs, fibers.shape[1], _ptr(off), _ptr(cf), _ptr(cd), int(depth),
        int(max_candidates), int(cf.numel()), FI_FP64_REFINE if refine else 0, _ptr(t), _ptr(u), _ptr(hit),
        _ptr(fib), _ptr(t64), _ptr(u64), _ptr(nrm), *ws, _stream(stream)))
    out = (t, u, hit, fib)
    if refine:
        out += (t64, u64)
    if nrm is not None:
        out += (nrm,)
    return out


def validate(fibers: torch.Tensor, excess: bool = False, stream=None):
    """Validity mask (int32, 0 = valid) of every fiber of a (16, n) table, and
    the (n, 2) float32 start/end cap excesses when ``excess``
    (``fiber_validate``)."""
    fs = _table(fibers, 16, "fibers")
    n = fibers.shape[1]
    mask = torch.empty(n, dtype=torch.int32, device=fibers.device)
    ex = torch.empty((n, 2), dtype=torch.float32, device=fibers.device) if excess else None
    _check(lib().fiber_validate(_ptr(fibers), fs, n, _ptr(mask), _ptr(ex), _stream(stream)))
    return (mask, ex) if excess else mask


def presplit(fibers: torch.Tensor, max_level: int = 6, stream=None):
    """Split invalid fibers into valid pieces (``fiber_presplit_count`` then
    ``fiber_presplit``; one device sync to read the piece count). Returns
    (pieces (16, k) float32, piece_fiber int32, u0, u1 float32, mask int32,
    offsets int64 (n + 1))."""
    fs = _table(fibers, 16, "fibers")
    n = fibers.shape[1]
    dev = fibers.device
    L = lib()
    nb = L.fiber_presplit_workspace_bytes(n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    _check(L.fiber_presplit_count(_ptr(fibers), fs, n, int(max_level), _ptr(off), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream(stream)))
    if stream is not None:
        stream.synchronize()
    k = int(off[-1].item())
    pieces = torch.empty((16, max(k, 1)), dtype=torch.float32, device=dev)[:, :k]
    pf = torch.empty(k, dtype=torch.int32, device=dev)
    u0 = torch.empty(k, dtype=torch.float32, device=dev)
    u1 = torch.empty(k, dtype=torch.float32, device=dev)
    mk = torch.empty(k, dtype=torch.int32, device=dev)
    _check(L.fiber_presplit(_ptr(fibers), fs, n, int(max_level), _ptr(off), k, _ptr(pieces),
                            pieces.stride(0), _ptr(pf), _ptr(u0), _ptr(u1), _ptr(mk), _stream(stream)))
    return pieces, pf, u0, u1, mk, off


class PreparedPairs:
    """One plain ``fiber_intersect_pairs`` call (no counts, no refinement),
    checked and marshalled once and then enqueued as often as needed, on any
    stream (serving loops, benchmarks): ``launch`` skips the per-call tensor
    checks and argument building of ``intersect_pairs``. The object keeps its
    input tensors alive and owns its workspace and (or takes, via ``out``)
    the output tensors t, u, hit, which every launch overwrites; launches of
    one object must not overlap (they share the workspace)."""

    def __init__(self, rays, fibers, depth=9, pair_ray=None, pair_fiber=None, pair_depth=None,
                 out=None, normal=None):
        rs = _table(rays, 7, "rays")
        fs = _table(fibers, 16, "fibers")
        pr = _index(pair_ray, torch.int32, "pair_ray")
        pf = _index(pair_fiber, torch.int32, "pair_fiber")
        pd = _index(pair_depth, torch.uint8, "pair_depth")
        n = _pair_count(rays, fibers, pr, pf, pd)
        self.t, self.u, self.hit = _outs(out, n, rays.device)
        self.normal = _normal_tensor(normal, n, rays.device)
        self.workspace = pairs_workspace(n, fibers.shape[1], pf is not None, rays.device)
        self._keep = (rays, fibers, pr, pf, pd)
        self._fn = lib().fiber_intersect_pairs
        self._args = (_ptr(rays), rs, rays.shape[1], _ptr(fibers), fs, fibers.shape[1],
                      _ptr(pr), _ptr(pf), _ptr(pd), int(depth), n, 0,
                      _ptr(self.t), _ptr(self.u), _ptr(self.hit), None, None, _ptr(self.normal),
                      *_ws_args(self.workspace))

    def launch(self, stream=None):
        _check(self._fn(*self._args, _stream(stream)))
        return (self.t, self.u, self.hit) + (() if self.normal is None else (self.normal,))


def raw_call(name: str, *args):
    """Call a C-ABI entry point with already-marshalled arguments (tests)."""
    return getattr(lib(), name)(*args)


# ---------------------------------------------------------------------------
# many problems in one launch
# ---------------------------------------------------------------------------

class FiScene(C.Structure):
    _fields_ = [("rays", C.c_void_p), ("ray_stride", C.c_int64), ("n_rays", C.c_int64),
                ("fibers", C.c_void_p), ("fiber_stride", C.c_int64), ("n_fibers", C.c_int64),
                ("pair_ray", C.c_void_p), ("pair_fiber", C.c_void_p), ("pair_depth", C.c_void_p),
                ("depth", C.c_int32), ("n_pairs", C.c_int64),
                ("t_out", C.c_void_p), ("u_out", C.c_void_p), ("hit_out", C.c_void_p),
                ("t64_out", C.c_void_p), ("u64_out", C.c_void_p), ("normal_out", C.c_void_p)]


class FiTuning(C.Structure):
    _fields_ = [("refill", C.c_int32), ("waves_per_simd", C.c_int32), ("stack", C.c_int32)]

    def as_dict(self):
        return {"refill": self.refill, "waves_per_simd": self.waves_per_simd, "stack": self.stack}


def _batched_lib():
    L = lib()
    if not getattr(L, "_batched_ready", False):
        vp = C.c_void_p
        L.fiber_batched_workspace_bytes.argtypes = [C.c_int32, C.c_int64]
        L.fiber_batched_workspace_bytes.restype = C.c_size_t
        L.fiber_intersect_batched.argtypes = [C.POINTER(FiScene), C.c_int32, C.POINTER(FiTuning),
                                              C.c_uint32, vp, C.c_size_t, vp]
        L.fiber_intersect_batched.restype = C.c_int
        L.fiber_batch_plan_create.argtypes = [C.POINTER(FiScene), C.c_int32, C.POINTER(FiTuning),
                                              C.c_uint32, C.POINTER(vp)]
        L.fiber_batch_plan_create.restype = C.c_int
        L.fiber_batch_plan_launch.argtypes = [vp, vp]
        L.fiber_batch_plan_launch.restype = C.c_int
        L.fiber_batch_plan_destroy.argtypes = [vp]
        L.fiber_batch_plan_destroy.restype = C.c_int
        L.fiber_batch_plan_tuning.argtypes = [vp, C.POINTER(FiTuning)]
        L.fiber_batch_plan_tuning.restype = C.c_int
        L.fiber_batch_autotune.argtypes = [C.POINTER(FiScene), C.c_int32, C.c_uint32, vp, C.c_size_t,
                                           vp, C.c_int32, C.POINTER(FiTuning), C.POINTER(C.c_float)]
        L.fiber_batch_autotune.restype = C.c_int
        L.fiber_tuning_save.argtypes = [C.c_char_p]
        L.fiber_tuning_load.argtypes = [C.c_char_p]
        L.fiber_tuning_lookup.argtypes = [C.c_char_p, C.c_uint32, C.c_int64, C.c_int32, C.c_int32,
                                          C.POINTER(FiTuning)]
        for f in (L.fiber_tuning_save, L.fiber_tuning_load, L.fiber_tuning_lookup, L.fiber_tuning_clear):
            f.restype = C.c_int
        L._batched_ready = True
    return L


class Problem:
    """One problem of a batch: device tensors in the layout of intersect_pairs,
    with its own outputs (allocated here; t64/u64 too when ``refine``)."""

    def __init__(self, rays, fibers, depth=9, pair_ray=None, pair_fiber=None, pair_depth=None,
                 refine=False, normal=False):
        _table(rays, 7, "rays")
        _table(fibers, 16, "fibers")
        self.rays, self.fibers = rays, fibers
        self.pair_ray = _index(pair_ray, torch.int32, "pair_ray")
        self.pair_fiber = _index(pair_fiber, torch.int32, "pair_fiber")
        self.pair_depth = _index(pair_depth, torch.uint8, "pair_depth")
        self.depth = int(depth)
        n = _pair_count(rays, fibers, self.pair_ray, self.pair_fiber, self.pair_depth)
        self.n = n
        dev = rays.device
        self.t = torch.empty(n, dtype=torch.float32, device=dev)
        self.u = torch.empty(n, dtype=torch.float32, device=dev)
        self.hit = torch.empty(n, dtype=torch.uint8, device=dev)
        self.t64 = torch.empty(n, dtype=torch.float64, device=dev) if refine else None
        self.u64 = torch.empty(n, dtype=torch.float64, device=dev) if refine else None
        self.normal = torch.empty((3, n), dtype=torch.float32, device=dev) if normal else None

    def scene(self):
        rs = _table(self.rays, 7, "rays")
        fs = _table(self.fibers, 16, "fibers")
        return FiScene(self.rays.data_ptr(), rs, self.rays.shape[1], self.fibers.data_ptr(), fs,
                       self.fibers.shape[1],
                       None if self.pair_ray is None else self.pair_ray.data_ptr(),
                       None if self.pair_fiber is None else self.pair_fiber.data_ptr(),
                       None if self.pair_depth is None else self.pair_depth.data_ptr(),
                       self.depth, self.n, self.t.data_ptr(), self.u.data_ptr(), self.hit.data_ptr(),
                       None if self.t64 is None else self.t64.data_ptr(),
                       None if self.u64 is None else self.u64.data_ptr(),
                       None if self.normal is None else self.normal.data_ptr())


def _batch_flags(problems, refine):
    if refine and any(p.t64 is None for p in problems):
        raise ValueError("a refined batch needs problems made with refine=True")
    return FI_FP64_REFINE if refine else 0


def _scene_array(problems):
    arr = (FiScene * len(problems))()
    for k, p in enumerate(problems):
        arr[k] = p.scene()
    return arr


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, FiTuning):
        return C.byref(t)
    return C.byref(FiTuning(int(t["refill"]), int(t["waves_per_simd"]), int(t.get("stack", 0))))


def workspace_for(problems, device=None):
    """Device workspace for a batched call over ``problems`` (a list of
    Problem): the scene table and pair offsets."""
    total = sum(int(p.n) for p in problems)
    nbytes = _batched_lib().fiber_batched_workspace_bytes(len(problems), total)
    if device is None:
        device = problems[0].rays.device
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def intersect_batched(problems, tuning=None, workspace=None, stream=None, refine=False):
    """All pairs of all problems in one persistent-kernel launch (results
    land in each Problem's t, u, hit, and t64, u64 when ``refine``)."""
    L = _batched_lib()
    flags = _batch_flags(problems, refine)
    arr = _scene_array(problems)
    if workspace is None:
        workspace = workspace_for(problems)
        _keep_for(workspace, stream)
    _check(L.fiber_intersect_batched(arr, len(problems), _tuning(tuning), flags,
                                     C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     _stream(stream)))
    return workspace


class BatchPlan:
    """A batch captured once into a HIP graph; ``launch`` replays it."""

    def __init__(self, problems, tuning=None, refine=False):
        L = _batched_lib()
        self.problems = problems
        flags = _batch_flags(problems, refine)
        arr = _scene_array(problems)
        h = C.c_void_p()
        _check(L.fiber_batch_plan_create(arr, len(problems), _tuning(tuning), flags, C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(_batched_lib().fiber_batch_plan_launch(self._h, _stream(stream)))

    def tuning(self):
        t = FiTuning()
        _check(_batched_lib().fiber_batch_plan_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if self._h:
            _check(_batched_lib().fiber_batch_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(problems, repeats=2, workspace=None, stream=None, refine=False):
    """Fastest tuning for this batch; returns (dict, milliseconds)."""
    L = _batched_lib()
    flags = _batch_flags(problems, refine)
    arr = _scene_array(problems)
    if workspace is None:
        workspace = workspace_for(problems)
    best = FiTuning()
    ms = C.c_float()
    _check(L.fiber_batch_autotune(arr, len(problems), flags, C.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), _stream(stream), int(repeats), C.byref(best),
                                  C.byref(ms)))
    return best.as_dict(), ms.value


def save_tuning(path):
    """Write the process's tuning table (every autotuned or loaded entry) to
    a text file."""
    _check(_batched_lib().fiber_tuning_save(os.fsencode(path)))


def load_tuning(path):
    """Merge a tuning table file into the process's table."""
    _check(_batched_lib().fiber_tuning_load(os.fsencode(path)))


def lookup_tuning(arch, total_pairs, n_scenes, max_depth, refine=False):
    """The table's tuning (dict) for a batch of this class on ``arch``
    (e.g. "gfx950"), or None."""
    t = FiTuning()
    st = _batched_lib().fiber_tuning_lookup(arch.encode(), FI_FP64_REFINE if refine else 0, int(total_pairs),
                                            int(n_scenes), int(max_depth), C.byref(t))
    if st == FI_ERR_RANGE:
        return None
    _check(st)
    return t.as_dict()


def clear_tuning():
    _check(_batched_lib().fiber_tuning_clear())
