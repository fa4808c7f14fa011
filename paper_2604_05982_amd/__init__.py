"""MI355X-native (gfx950) GPU-resident fork-join task runtime.

The runtime itself is the HIP library built from ``csrc/`` into
``libgtap.so``; :mod:`paper_2604_05982_amd.gtap` is its Python binding.
"""
__all__ = ["gtap"]
