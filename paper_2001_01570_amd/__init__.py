"""Compact 8th-order gas-kinetic scheme on MI355X (gfx950).

The hot path -- compact linear and WENO-Z reconstruction, the per-interface
gas-kinetic evolution and the two-stage fourth-order update of cell averages
and cell-averaged gradients -- runs in hand-written HIP kernels behind the
C ABI declared in include/cgks.h.  This package is the thin Python binding.
"""
