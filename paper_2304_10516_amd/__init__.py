"""MI355X (gfx950) hot path of the distributed volumetric neural representation
(DVNR): per-block multiresolution hash-grid INRs trained and decoded by hand-
written HIP kernels behind the C ABI in include/dvnr.h.

Importing the package does not load the library; `paper_2304_10516_amd.DVNR`
(or `_lib.lib()`) does, and fails loudly when libdvnr.so is not built.
"""
from __future__ import annotations

__all__ = ["DVNR", "EncodingCfg", "MlpCfg", "OptimCfg"]


def __getattr__(name):
    if name in ("DVNR", "EncodingCfg", "MlpCfg", "OptimCfg"):
        from . import dvnr as _d
        return getattr(_d, name)
    raise AttributeError(name)
