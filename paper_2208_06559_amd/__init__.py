"""MI355X-native bead-rod Brownian dynamics with RPY hydrodynamic
interactions (arXiv 2208.06559): Python binding of ``libbdrpy.so``.

The binding is loaded lazily, so that ``paper_2208_06559_amd.inputs`` can be
imported without it; every compute call fails loudly if the HIP library is
missing.
"""
__all__ = ["inputs"]
