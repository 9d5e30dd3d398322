"""The pins catch plausible mistakes in the oracle (CPU only).

Each mutant is a copy of the oracle's C sources with one planted mistake (a
flipped comparison, a dropped term, a wrong index or sign). It is built into
a temporary library and the pin suites run against it; every mutant must
make at least one pin fail. The mistakes are planted in copies only: the
oracle in the tree is never changed."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
D, X, V = "fiber_oracle.c", "fiber_exact.c", "fiber_validate.c"

# (name, file, text, replacement): the first occurrence of text is replaced
MUTANTS = [
    ("first child chosen the wrong way", D, "go_right = beyond_entry != (n.z > 0.0);",
     "go_right = beyond_entry == (n.z > 0.0);"),
    ("second child never visited", D, "if (!both) return 0;", "if (1) return 0;"),
    ("radius without the control-point distance", D, "return sqrt(fmax(d1, d2)) + rmax;", "return rmax;"),
    ("interval narrowed on the wrong side", D, "if (beyond_entry) { if (tpn < fhi)", "if (!beyond_entry) { if (tpn < fhi)"),
    ("leaf t without the cap plane", D, "const double t = enter;", "const double t = te;"),
    ("visibility without the cropped interval", D, "decide_vis(S, enter <= leave,", "decide_vis(S, tx >= lo && te <= hi,"),
    ("wrong sign in the ray-axis distance", D, "const double dd = a.x * o.y - a.y * o.x;",
     "const double dd = a.x * o.y + a.y * o.x;"),
    ("wrong de Casteljau split point", D, "const v4 s = scale4(add4(m012, m123), 0.5);",
     "const v4 s = scale4(add4(m012, m12), 0.5);"),
    ("chord instead of tangent as split normal", D, "v4 t = sub4(add4(q[2], q[3]), add4(q[0], q[1]));",
     "v4 t = sub4(q[3], q[0]);"),
    ("no interval recomputation after backtracking", D,
     "return visit(S, second, blo, bhi, eblo, ebhi, level + 1, s0, s1);",
     "return visit(S, second, lo, hi, elo, ehi, level + 1, s0, s1);"),
    ("tangents negligible only when exactly zero", D, "return dot3(v, v) <= 0x1p-40 * dot3(chord, chord);",
     "return zero3(v);"),
    ("grazing ties never decided together", D, "return S->ties.force_vis > 0;", "return value;"),
    ("visibility forced outside ties", D,
     "if (S->ties.force_vis != 0 && S->ties.scale > 0.0 && isfinite(diff) &&\n        fabs(diff) <= S->ties.scale * margin) {",
     "if (S->ties.force_vis != 0) {"),
    ("flipped crossing kept at its value", D,
     "if (beyond_entry != (tp > te)) tpn = beyond_entry ? tp + ep : tp - ep;", "(void)0;"),
    ("cusp children keep the noise of the split tangent", D,
     "if (!negligible(sub4(l[3], l[2]), sub4(q[3], q[0]))) return;", "return;"),
    ("tie margin 2^10 too wide", D, "return (2.0 + 2.0 * level) * 0x1p-24 * S->ties.X;",
     "return (2.0 + 2.0 * level) * 0x1p-14 * S->ties.X;"),
    ("start cap normal pointing inwards", D,
     "const v4 cap = near1 ? S->cap1 : scale4(S->cap0, -1.0);",
     "const v4 cap = near1 ? S->cap1 : S->cap0;"),
    ("side normal from the leaf's start point", D,
     "add4(N->q[0], scale4(a, ul)));", "N->q[0]);"),
    ("cap entries given the side normal", D, "const int on_cap = plane && dc <= 1.0;",
     "const int on_cap = 0;"),
    ("cap plane test without its tolerance", D, "const int on_cap = plane && dc <= 1.0;",
     "const int on_cap = plane && dc <= 0.0;"),
    ("the farther cap plane taken", D, "const int near1 = d1 < d0;", "const int near1 = d1 > d0;"),
    ("normal left in the ray frame", D,
     "normal_out[k] = hit ? S.n[0] * frame[k] + S.n[1] * frame[3 + k] + S.n[2] * frame[6 + k] : NAN;",
     "normal_out[k] = hit ? S.n[k] : NAN;"),
    ("later candidates not held to the nearest hit", D,
     "ray[6] = t;                     /* later candidates must come nearer */", "(void)0;"),
    ("candidate lists not truncated", D, "if (end - off[r] > max_cand) end = off[r] + max_cand;", "(void)0;"),
    ("cap excess with the wrong sign of the along term", V, "return r * s - along;", "return r * s + along;"),
    ("end cap normal taken at the start", V, "c[0] = end ? vsub(pt(q, 3), pt(q, 2)) : vsub(pt(q, 1), pt(q, 0));",
     "c[0] = vsub(pt(q, 1), pt(q, 0));"),
    ("cosine instead of sine of the disc tilt", V, "const double s = sqrt(vdot(x, x)) / dl;",
     "const double s = vdot(D, n) / dl;"),
    ("pieces not halved at the midpoint", V, "const double s = (m012 + m123) * 0.5;",
     "const double s = (m012 + m12) * 0.5;"),
    ("halving one level past the limit", V, "level >= max_level ||", "level > max_level ||"),
    ("quadratic bound from the elevated inner points", D, "return 1.5 * sqrt(fmax(d1, d2)) + rmax;",
     "return sqrt(fmax(d1, d2)) + rmax;"),
    ("quadratic elevation with swapped weights", D, "q[4 + c] = (p[c] + 2.0 * p[4 + c]) / 3.0;",
     "q[4 + c] = (2.0 * p[c] + p[4 + c]) / 3.0;"),
    ("stalled nodes cut short anywhere on the curve", D, "const int stalled = (u0 == 0.0 || u1 == 1.0) &&",
     "const int stalled = 1 &&"),
    ("stall without the FP32 resolution bound", D, "const int stalled = (u0 == 0.0 || u1 == 1.0) && ext <= S->stall_abs &&",
     "const int stalled = (u0 == 0.0 || u1 == 1.0) &&"),
    ("stall without the bound relative to the root", D, "ext <= ldexp(S->stall_rel, -2 * level);", "1;"),
    ("exact oracle: no side points about discs that nearly contain the ray", X,
     "    if (!eo) {\n        double bs = INFINITY, bus = NAN;", "    if (0) {\n        double bs = INFINITY, bus = NAN;"),
    ("exact oracle: side roots taken off the disc's circle", X, "if (on_circle && rest < -1e-9",
     "if (0 && rest < -1e-9"),
    ("exact oracle: edge-on side points taken where C' vanishes", X,
     "if (tok && has_disc && t >= 0.0L", "if (tok && t >= 0.0L"),
    ("exact oracle: radius term with the wrong sign", X, "F = badd(&F, &a3, -1.0);", "F = badd(&F, &a3, 1.0);"),
    ("exact oracle: no limit disc at a zero end tangent", X, "while (j < 2 && cand[j][0]", "while (0 && cand[j][0]"),
    ("exact oracle: edge-on rays through the expanded polynomial", X, "    if (eo) {\n        /* F's two roots",
     "    if (0) {\n        /* F's two roots"),
    ("exact oracle: edge-on exit taken for the entry", X, "if (t) *t = C[2] + s * sr;", "if (t) *t = C[2] + sr;"),
    ("exact oracle: taper tilt with the wrong sign", X, "const double beta = -D1[3] /",
     "const double beta = D1[3] /"),
    ("exact oracle: no curvature term in the tilt", X, "(dl - C[3] * ec2 / dl)", "(dl)"),
    ("exact oracle: start cap normal pointing inwards", X, "(kind == 2 ? -1.0 : 1.0)", "(1.0)"),
    ("exact oracle: later candidates not held to the nearest entry", X,
     "best_n[k] = nn[k];\n                ray[6] = t;", "best_n[k] = nn[k];"),
    ("exact oracle: circle point on the wrong side", X,
     "tsq = fabs((tm - C[2]) * D[2] - xy) <= fabs((tp - C[2]) * D[2] - xy) ? tm : tp;",
     "tsq = fabs((tm - C[2]) * D[2] - xy) <= fabs((tp - C[2]) * D[2] - xy) ? tp : tm;"),
]


def _run_mutant(m, tmp):
    name, fname, text, repl = m
    srcs = []
    for f in oracle_build.SOURCES:
        with open(os.path.join(oracle_build.HERE, f)) as fh:
            src = fh.read()
        if f == fname:
            assert text in src, f"mutation site gone: {name}"
            src = src.replace(text, repl, 1)
        path = os.path.join(tmp, f)
        with open(path, "w") as fh:
            fh.write(src)
        srcs.append(path)
    lib = os.path.join(tmp, "libmutant.so")
    subprocess.run(oracle_build.gcc_cmd(srcs, lib), check=True, capture_output=True)
    env = dict(os.environ, FIBER_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "tests/test_oracle_pins.py", "tests/test_oracle_exact.py",
                          "tests/test_oracle_normals.py", "tests/test_oracle_candidates.py",
                          "tests/test_oracle_validate.py", "tests/test_oracle_quadratic.py",
                          "tests/test_oracle_stall.py"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, res.returncode, res.stdout[-400:]


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as top:
        dirs = []
        for k in range(len(MUTANTS)):
            d = os.path.join(top, str(k))
            os.makedirs(d)
            dirs.append(d)
        with ThreadPoolExecutor(max_workers=max(2, min(8, os.cpu_count() or 2))) as ex:
            results = list(ex.map(_run_mutant, MUTANTS, dirs))
    survivors = [(name, out) for name, rc, out in results if rc == 0]
    assert not survivors, survivors
    # a failure must be a failed pin, not a crash or a collection error
    for name, rc, out in results:
        assert rc == 1, (name, rc, out)
