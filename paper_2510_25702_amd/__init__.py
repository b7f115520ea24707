"""MI355X (gfx950) implementation of the per-step particle pipeline of the
weakly compressible SPH / k-epsilon RANS method with improved bidirectional
open-boundary buffers (Wang & Hu, arXiv 2510.25702).

The compute path is the C-ABI library ``libsphx.so`` (include/sph.h) built
from ``csrc/`` with hipcc for gfx950; ``sph`` is its Python binding.
"""
from .sph import (SPH_FP32_MIXED, SPH_FP64, Simulation, SphError, lib)  # noqa: F401
