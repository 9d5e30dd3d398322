"""MI355X (gfx950) ray/fiber intersection after Binder & Keller,
"Fast, High Precision Ray/Fiber Intersection using Tight, Disjoint Bounding
Volumes" (arXiv 1811.03374).

The compute path is a C-ABI shared library of hand-written HIP kernels
(``csrc/``); ``binding`` marshals torch device tensors into it.
"""
__version__ = "0.1.0"
