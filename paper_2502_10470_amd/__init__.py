"""MetaDE inner-DE path on AMD Instinct MI355X (gfx950).

The compute lives in ``libmetade.so`` (HIP kernels behind the C ABI declared
in ``include/metade.h``); ``metade`` is its thin Python binding.
"""
from . import metade  # noqa: F401
from .metade import Batch, MetadeError  # noqa: F401
