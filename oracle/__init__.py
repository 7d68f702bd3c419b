"""Float64 CPU oracle of the DVNR hot path -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never
does.
"""
from . import dvnr_oracle  # noqa: F401
