"""Algorithmic work model of the per-pair test (fixed before measurement).

Flops count add, sub, mul, min/max, div and sqrt as 1 and fma as 2, taken from
the operations the paper's listings perform (Appendix C):

  setup     130  normalise the direction, build the basis, project four
                 control points, convert to {p, d, t0, t1}, cap interval
  test       78  conservative radius (point-line distances) + unit-ray
                 cylinder (Appendix A) + overlap with the t interval
  split      57  split point and tangent (Section 3.1), split plane,
                 ordering, interval update, keep one half
  backtrack 160  re-derive the pending node (four curve evaluations) and
                 its cap interval (Section 3.3)
  finalise   21  u from the projection onto the leaf chord

The counts of tests, splits and backtracks per pair come from the traversal
itself (``fiber_intersect_counts``), whose counts equal the oracle's.

Bytes: each pair reads a ray (7 floats), a fiber (16 floats) and writes t, u
(floats) and a hit byte; a gathered pair also reads its two int32 indices.
"""
FLOPS_SETUP = 130
FLOPS_TEST = 78
FLOPS_SPLIT = 57
FLOPS_BACKTRACK = 160
FLOPS_FINAL = 21

BYTES_RAY = 7 * 4
BYTES_FIBER = 16 * 4
BYTES_OUT = 4 + 4 + 1
BYTES_INDEX = 4


def flops(n_pairs, tests, splits, backtracks, hits):
    return (FLOPS_SETUP * n_pairs + FLOPS_TEST * tests + FLOPS_SPLIT * splits
            + FLOPS_BACKTRACK * backtracks + FLOPS_FINAL * hits)


def bytes_streamed(n_pairs, indexed=False):
    """HBM bytes when every ray and fiber is read once (identity pairing)."""
    per = BYTES_RAY + BYTES_FIBER + BYTES_OUT + (2 * BYTES_INDEX if indexed else 0)
    return per * n_pairs


def bytes_gathered(n_pairs, n_fibers):
    """HBM bytes of a call with one ray per pair and fibers gathered through
    an int32 index: each pair reads its ray and index and writes its outputs
    (41 B), and the fiber table is read once (64 B per fiber)."""
    return (BYTES_RAY + BYTES_INDEX + BYTES_OUT) * n_pairs + BYTES_FIBER * n_fibers


# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3        # vector FP32, 256 CUs at 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
