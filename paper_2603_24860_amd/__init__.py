"""Symmetry-blocked Bethe-Salpeter hot path for MI355X (gfx950).

The compute path lives in the HIP library libbse.so (include/bse.h); this
package holds the thin Python binding (bse.py) and the device-side system
container and solve sequence (system.py).
"""
from . import bse  # noqa: F401  (loads libbse.so; raises if it is missing)
