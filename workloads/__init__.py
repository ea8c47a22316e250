"""Seeded synthetic inputs shared by the checker's tests, the oracle and the
benchmark.  This package only builds descriptions; it holds none of the
checking arithmetic."""

from .desc import (AUX_EMOD, AUX_FLOORDIV, AUX_NONE, BARRIER_BLOCK, BARRIER_NONE, BARRIER_WARP, GLOBAL, NV,
                   SHARED, VARS, Access, Array, Aux, Builder, KernelDesc, Phase, Segment, aff, aff_from, rw)
from . import kernels, random_affine

__all__ = [
    "AUX_EMOD", "AUX_FLOORDIV", "AUX_NONE", "BARRIER_BLOCK", "BARRIER_NONE", "BARRIER_WARP", "GLOBAL", "NV", "SHARED", "VARS", "Access", "Array",
    "Aux", "Builder", "KernelDesc", "Phase", "Segment", "aff", "aff_from", "rw", "kernels",
    "random_affine",
]
