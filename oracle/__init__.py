"""TEST INFRASTRUCTURE: ctypes front end of the FP64 CPU oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package. The HIP library and its Python binding never
do: they share no code with it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        # FIBER_ORACLE_LIB: another build of these sources (the mutation test
        # loads copies with planted mistakes through it)
        path = os.environ.get("FIBER_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.fo_intersect_d.argtypes = [dp, dp, C.c_int, dp, dp, C.POINTER(C.c_int64)]
        L.fo_intersect_d.restype = C.c_int
        L.fo_batch_d.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int64,
                                 C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_int]
        L.fo_batch_d.restype = None
        L.fo_tie_outcomes_quad.argtypes = [dp, dp, C.c_int, C.c_double, C.c_int, C.c_int, dp, dp,
                                           C.POINTER(C.c_int)]
        L.fo_tie_outcomes_quad.restype = C.c_int
        L.fo_quadratic_constraint.argtypes = [dp]
        L.fo_quadratic_constraint.restype = C.c_int
        L.fo_split_half.argtypes = [dp, dp, dp]
        L.fo_split_plane.argtypes = [dp, dp, dp]
        L.fo_split_children.argtypes = [dp, dp, dp]
        L.fo_unit_ray_cylinder.argtypes = [dp, dp, C.c_double, dp, dp]
        L.fo_unit_ray_cylinder.restype = C.c_int
        L.fo_conservative_radius.argtypes = [dp]
        L.fo_conservative_radius.restype = C.c_double
        L.fo_cap_interval.argtypes = [dp, C.c_double, dp]
        L.fo_ray_frame.argtypes = [dp, dp, dp]
        L.fo_ray_frame.restype = C.c_int
        L.fo_tie_outcomes.argtypes = [dp, dp, C.c_int, C.c_double, C.c_int, C.c_int, dp, dp,
                                      C.POINTER(C.c_int)]
        L.fo_tie_outcomes.restype = C.c_int
        L.fo_nearest_d.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_double,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_void_p]
        L.fo_nearest_d.restype = None
        L.fv_validate.argtypes = [dp, dp, dp]
        L.fv_validate.restype = C.c_int
        L.fv_presplit.argtypes = [dp, C.c_int, dp, dp, dp, C.c_void_p, C.c_int]
        L.fv_presplit.restype = C.c_int
        L.fv_validate_batch.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
        L.fv_validate_batch.restype = None
        L.fo_cubic_constraints.argtypes = [dp]
        L.fo_cubic_constraints.restype = C.c_int
        if hasattr(L, "fx_batch"):
            L.fx_batch.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
            L.fx_batch.restype = None
            L.fx_intersect.argtypes = [dp, dp, dp, dp, dp]
            L.fx_intersect.restype = C.c_int
            L.fx_nearest.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
            L.fx_nearest.restype = None
            L.fx_batch_quad.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
            L.fx_batch_quad.restype = None
            L.fx_side_polynomial.argtypes = [dp, dp]
            L.fx_side_polynomial.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def intersect_depth(rays, fibers, depth=9, pair_ray=None, pair_fiber=None,
                    pair_depth=None, radius_scale=1.0, stats=False, nthreads=0, t_err=False,
                    normal=False, quadratic=False):
    """ORACLE-D: the paper's depth-d method in FP64 for every pair.

    Returns (t float64, u float64, hit uint8[, stats int32 (n, 4)][, t_err
    float64][, normal float64 (n, 8)]). ``stats`` columns: node tests, splits,
    backtracks (second-child visits), leaf level (-1 on a miss). ``t_err``:
    error bound of each hit's t in an FP32 evaluation (reading R14's node
    error model; 0 on a miss). ``normal`` columns: the unit normal at the hit
    in world space (3), the normal of the other entry where a cap and a side
    entry tie (3, else the same), the angle bound in radians of the normal in
    an FP32 evaluation (1), how the leaf was entered (1: 0 through the
    cylinder's side, 1 through a plane on the curve's start cap plane, 2 on
    its end cap plane, 3 through another plane or at the origin); NaN on a
    miss. ``quadratic``: fibers are (12, n) quadratics (Appendix B.1)."""
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    fibers = np.ascontiguousarray(fibers, dtype=np.float32)
    pr = None if pair_ray is None else np.ascontiguousarray(pair_ray, dtype=np.int32)
    pf = None if pair_fiber is None else np.ascontiguousarray(pair_fiber, dtype=np.int32)
    pd = None if pair_depth is None else np.ascontiguousarray(pair_depth, dtype=np.uint8)
    if pr is not None:
        n = pr.shape[0]
    elif pf is not None:
        n = pf.shape[0]
    else:
        n = min(rays.shape[1], fibers.shape[1])
    t = np.empty(n, np.float64)
    u = np.empty(n, np.float64)
    hit = np.empty(n, np.uint8)
    st = np.empty((n, 4), np.int32) if stats else None
    te = np.empty(n, np.float64) if t_err else None
    nn = np.empty((n, 8), np.float64) if normal else None
    lib().fo_batch_d(_ptr(rays), rays.shape[1], rays.shape[1], _ptr(fibers), fibers.shape[1],
                     fibers.shape[1], _ptr(pr), _ptr(pf), _ptr(pd), int(depth), n,
                     float(radius_scale), _ptr(t), _ptr(u), _ptr(hit), _ptr(st), int(nthreads),
                     _ptr(te), _ptr(nn), int(bool(quadratic)))
    out = (t, u, hit) + ((st,) if stats else ()) + ((te,) if t_err else ()) + ((nn,) if normal else ())
    return out


def intersect_exact(rays, fibers, pair_ray=None, pair_fiber=None, radius_scale=1.0,
                    nthreads=0, normal=False, quadratic=False):
    """ORACLE-X: first entry of the ray into the swept-disk solid (the limit
    of the method), in FP64. Returns (t, u, hit, kind[, normal (n, 3)]) where
    kind is 0 miss, 1 side surface, 2 start cap, 3 end cap, 4 origin inside;
    ``normal`` is the outward unit normal at the entry in world space (NaN
    on a miss or with the origin inside)."""
    L = lib()
    if not hasattr(L, "fx_batch"):
        raise RuntimeError("exact oracle not built")
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    fibers = np.ascontiguousarray(fibers, dtype=np.float32)
    pr = None if pair_ray is None else np.ascontiguousarray(pair_ray, dtype=np.int32)
    pf = None if pair_fiber is None else np.ascontiguousarray(pair_fiber, dtype=np.int32)
    if pr is not None:
        n = pr.shape[0]
    elif pf is not None:
        n = pf.shape[0]
    else:
        n = min(rays.shape[1], fibers.shape[1])
    t = np.empty(n, np.float64)
    u = np.empty(n, np.float64)
    kind = np.empty(n, np.int32)
    nn = np.empty((n, 3), np.float64) if normal else None
    fn = L.fx_batch_quad if quadratic else L.fx_batch
    fn(_ptr(rays), rays.shape[1], rays.shape[1], _ptr(fibers), fibers.shape[1],
       fibers.shape[1], _ptr(pr), _ptr(pf), n, float(radius_scale),
       _ptr(t), _ptr(u), _ptr(kind), int(nthreads), _ptr(nn))
    return (t, u, (kind > 0).astype(np.uint8), kind) + ((nn,) if normal else ())


def intersect_nearest(rays, fibers, offsets, cand, depth=9, cand_depth=None, max_cand=None,
                      radius_scale=1.0, nthreads=0, t_err=False, normal=False):
    """Nearest hit over each ray's candidate list with the depth-d method
    (fo_nearest_d): candidates cand[offsets[r]:offsets[r+1]] in order, each
    against the ray shortened to the latest hit. Returns (t, u, hit, fiber[,
    t_err][, normal (n_rays, 8)])."""
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    fibers = np.ascontiguousarray(fibers, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    cd = np.ascontiguousarray(cand, dtype=np.int32)
    dd = None if cand_depth is None else np.ascontiguousarray(cand_depth, dtype=np.uint8)
    n = rays.shape[1]
    assert off.shape[0] == n + 1
    mc = int(np.diff(off).max(initial=0)) if max_cand is None else int(max_cand)
    t = np.empty(n)
    u = np.empty(n)
    hit = np.empty(n, np.uint8)
    fib = np.empty(n, np.int32)
    te = np.empty(n) if t_err else None
    nn = np.empty((n, 8)) if normal else None
    lib().fo_nearest_d(_ptr(rays), rays.shape[1], n, _ptr(fibers), fibers.shape[1], fibers.shape[1],
                       _ptr(off), _ptr(cd), _ptr(dd), int(depth), mc, float(radius_scale), _ptr(t),
                       _ptr(u), _ptr(hit), _ptr(fib), int(nthreads), _ptr(te), _ptr(nn))
    return (t, u, hit, fib) + ((te,) if t_err else ()) + ((nn,) if normal else ())


def nearest_exact(rays, fibers, offsets, cand, max_cand=None, radius_scale=1.0, nthreads=0,
                  normal=False):
    """Nearest entry over each ray's candidate list into the swept solids
    (fx_nearest). Returns (t, u, hit, kind, fiber[, normal (n_rays, 3)])."""
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    fibers = np.ascontiguousarray(fibers, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    cd = np.ascontiguousarray(cand, dtype=np.int32)
    n = rays.shape[1]
    mc = int(np.diff(off).max(initial=0)) if max_cand is None else int(max_cand)
    t = np.empty(n)
    u = np.empty(n)
    kind = np.empty(n, np.int32)
    fib = np.empty(n, np.int32)
    nn = np.empty((n, 3)) if normal else None
    lib().fx_nearest(_ptr(rays), rays.shape[1], n, _ptr(fibers), fibers.shape[1], fibers.shape[1],
                     _ptr(off), _ptr(cd), mc, float(radius_scale), _ptr(t), _ptr(u), _ptr(kind),
                     _ptr(fib), int(nthreads), _ptr(nn))
    return (t, u, (kind > 0).astype(np.uint8), kind, fib) + ((nn,) if normal else ())


def single_exact(ray, fiber, normal=False):
    """One pair through fx_intersect (float64 inputs). Returns (kind, t, u[,
    normal])."""
    r, rp = _d(ray)
    f, fp = _d(fiber)
    t = C.c_double()
    u = C.c_double()
    n = np.empty(3)
    kind = lib().fx_intersect(rp, fp, C.byref(t), C.byref(u), n.ctypes.data_as(C.POINTER(C.c_double)))
    return (kind, t.value, u.value) + ((n,) if normal else ())


def side_polynomial(q16):
    """Bernstein coefficients of the degree-10 side polynomial of a curve
    already in the ray frame."""
    q, qp = _d(q16)
    out = np.zeros(11)
    n = lib().fx_side_polynomial(qp, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out[:n + 1]


def single_depth(ray, fiber, depth):
    """One pair through fo_intersect_d (float64 inputs, no float32 rounding)."""
    r, rp = _d(ray)
    f, fp = _d(fiber)
    t = C.c_double()
    u = C.c_double()
    st = (C.c_int64 * 4)()
    hit = lib().fo_intersect_d(rp, fp, int(depth), C.byref(t), C.byref(u), st)
    return bool(hit), t.value, u.value, tuple(st)


def tie_outcomes(ray, fiber, depth, scale=1.0, max_flips=2, max_out=512, quadratic=False):
    """Results of one pair reachable by flipping at most ``max_flips`` near-tie
    comparisons: comparisons whose two sides differ by at most ``scale`` times
    the sum of their FP32 error bounds (reading R14 of the oracle). Returns
    arrays (t, u, hit), the unflipped result first."""
    r, rp = _d(ray)
    f, fp = _d(fiber)
    t = np.empty(max_out)
    u = np.empty(max_out)
    h = np.empty(max_out, np.int32)
    fn = lib().fo_tie_outcomes_quad if quadratic else lib().fo_tie_outcomes
    n = fn(rp, fp, int(depth), float(scale), int(max_flips), int(max_out),
                              t.ctypes.data_as(C.POINTER(C.c_double)),
                              u.ctypes.data_as(C.POINTER(C.c_double)),
                              h.ctypes.data_as(C.POINTER(C.c_int)))
    return t[:n], u[:n], h[:n].astype(bool)


def split_half(q16):
    q, qp = _d(q16)
    L = np.empty(16)
    R = np.empty(16)
    lib().fo_split_half(qp, L.ctypes.data_as(C.POINTER(C.c_double)),
                        R.ctypes.data_as(C.POINTER(C.c_double)))
    return L, R


def split_children(q16):
    """The two children the depth-d recursion uses (de Casteljau halves with
    the cusp rule of reading R13)."""
    q, qp = _d(q16)
    L = np.empty(16)
    R = np.empty(16)
    lib().fo_split_children(qp, L.ctypes.data_as(C.POINTER(C.c_double)),
                            R.ctypes.data_as(C.POINTER(C.c_double)))
    return L, R


def split_plane(q16):
    q, qp = _d(q16)
    s = np.empty(3)
    n = np.empty(3)
    lib().fo_split_plane(qp, s.ctypes.data_as(C.POINTER(C.c_double)),
                         n.ctypes.data_as(C.POINTER(C.c_double)))
    return s, n


def unit_ray_cylinder(o, a, r):
    o_, op = _d(o)
    a_, ap = _d(a)
    t0 = C.c_double()
    t1 = C.c_double()
    ok = lib().fo_unit_ray_cylinder(op, ap, float(r), C.byref(t0), C.byref(t1))
    return bool(ok), t0.value, t1.value


def conservative_radius(q16):
    q, qp = _d(q16)
    return lib().fo_conservative_radius(qp)


def cap_interval(q16, tmax):
    q, qp = _d(q16)
    out = np.empty(2)
    lib().fo_cap_interval(qp, float(tmax), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out[0], out[1]


def ray_frame(ray7, fiber16):
    r, rp = _d(ray7)
    f, fp = _d(fiber16)
    out = np.empty(16)
    ok = lib().fo_ray_frame(rp, fp, out.ctypes.data_as(C.POINTER(C.c_double)))
    return (out if ok else None)


def cubic_constraints(q16):
    q, qp = _d(q16)
    return lib().fo_cubic_constraints(qp)


def validate(q16):
    """Validity mask of one fiber (fv_validate; 0: valid): bits 0-4 the five
    inequalities of Section 3.4 that fail, bit 5 thick at the start, bit 6
    thick at the end, bit 7 non-finite. Returns (mask, start excess, end
    excess), the excesses relative to the fiber's extent."""
    q, qp = _d(q16)
    e0, e1 = C.c_double(), C.c_double()
    m = lib().fv_validate(qp, C.byref(e0), C.byref(e1))
    return m, e0.value, e1.value


def validate_table(fibers, nthreads=0):
    """Masks (int32) and excesses (n, 2) of every fiber of a (16, n) table."""
    f = np.ascontiguousarray(fibers, dtype=np.float32)
    n = f.shape[1]
    m = np.empty(n, np.int32)
    ex = np.empty((n, 2))
    lib().fv_validate_batch(_ptr(f), n, n, _ptr(m), _ptr(ex), int(nthreads))
    return m, ex


def presplit(q16, max_level=6):
    """Pieces of one fiber (fv_presplit): (pieces (k, 16), u0, u1, masks)."""
    q, qp = _d(q16)
    cap = 1 << max_level
    pieces = np.empty((cap, 16))
    u0 = np.empty(cap)
    u1 = np.empty(cap)
    mk = np.empty(cap, np.int32)
    k = lib().fv_presplit(qp, int(max_level), pieces.ctypes.data_as(C.POINTER(C.c_double)),
                          u0.ctypes.data_as(C.POINTER(C.c_double)), u1.ctypes.data_as(C.POINTER(C.c_double)),
                          _ptr(mk), cap)
    return pieces[:k], u0[:k], u1[:k], mk[:k]


def quadratic_constraint(p12):
    """The constraint of Appendix B.1, <p1 - p0, p1 - p2> <= 0 (bool)."""
    q, qp = _d(p12)
    return bool(lib().fo_quadratic_constraint(qp))
