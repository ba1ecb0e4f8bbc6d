"""Symmetry-blocked Bethe-Salpeter hot path for MI355X (gfx950).

The compute path lives in the HIP library libbse.so (include/bse.h); this
package holds the thin Python binding (bse.py, which loads the library and
raises if it is missing), the device-side system container and solve sequence
(system.py), and the build script (build_lib.py).
"""
