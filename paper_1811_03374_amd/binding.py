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
FI_MAX_DEPTH = 23

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
        L.fiber_intersect_pairs.argtypes = common + [vp]
        L.fiber_intersect_pairs.restype = C.c_int
        L.fiber_intersect_counts.argtypes = common + [vp, vp]
        L.fiber_intersect_counts.restype = C.c_int
        L.fi_strerror.argtypes = [C.c_int]
        L.fi_strerror.restype = C.c_char_p
        L.fi_version.restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    return ["fi_version", "fi_strerror", "fiber_intersect_pairs", "fiber_intersect_counts"]


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


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def intersect_pairs(rays: torch.Tensor, fibers: torch.Tensor, depth: int = 9,
                    pair_ray: Optional[torch.Tensor] = None,
                    pair_fiber: Optional[torch.Tensor] = None,
                    pair_depth: Optional[torch.Tensor] = None,
                    out=None, counts: bool = False, stream=None):
    """Nearest hit (t, u, hit) of every (ray, fiber) pair at subdivision depth
    ``depth`` (or per-pair ``pair_depth``). See ``fiber_intersect_pairs``.

    rays: (7, n_rays) float32; fibers: (16, n_fibers) float32; indices int32.
    Returns (t, u, hit) device tensors, plus an (n, 4) int32 tensor of node
    tests / splits / backtracks / leaf level when ``counts`` is set."""
    rs = _table(rays, 7, "rays")
    fs = _table(fibers, 16, "fibers")
    pr = _index(pair_ray, torch.int32, "pair_ray")
    pf = _index(pair_fiber, torch.int32, "pair_fiber")
    pd = _index(pair_depth, torch.uint8, "pair_depth")
    if pr is not None:
        n = pr.shape[0]
    elif pf is not None:
        n = pf.shape[0]
    elif pd is not None:
        n = pd.shape[0]
    else:
        n = min(rays.shape[1], fibers.shape[1])
    dev = rays.device
    if out is None:
        t = torch.empty(n, dtype=torch.float32, device=dev)
        u = torch.empty(n, dtype=torch.float32, device=dev)
        hit = torch.empty(n, dtype=torch.uint8, device=dev)
    else:
        t, u, hit = out
    cn = torch.empty((n, 4), dtype=torch.int32, device=dev) if counts else None
    args = [_ptr(rays), rs, rays.shape[1], _ptr(fibers), fs, fibers.shape[1],
            _ptr(pr), _ptr(pf), _ptr(pd), int(depth), n, 0,
            _ptr(t), _ptr(u), _ptr(hit)]
    if counts:
        _check(lib().fiber_intersect_counts(*args, _ptr(cn), _stream(stream)))
        return t, u, hit, cn
    _check(lib().fiber_intersect_pairs(*args, _stream(stream)))
    return t, u, hit


def raw_call(name: str, *args):
    """Call a C-ABI entry point with already-marshalled arguments (tests)."""
    return getattr(lib(), name)(*args)
