"""MI355X-native Wilson-clover / SAP / FGMRES library (HIP, gfx950).

The compute path lives in ``libddsap.so`` (C ABI declared in include/ddsap.h);
``paper_1710_07041_amd.ddsap`` is its thin ctypes binding.  Importing this
package loads nothing: ``synth`` (seeded inputs) has no GPU dependency.
"""
