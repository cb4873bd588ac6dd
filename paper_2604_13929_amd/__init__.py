"""MI355X-native 3D Monte Carlo photon migration through voxelised pore masks.

The hot path (voxel walk, tallies, reduction) is HIP for gfx950 behind the C
ABI in ``include/photonmc.h``; ``photonmc`` is its Python binding and
``inputs`` generates seeded synthetic masks.  Importing the package loads
nothing; the library is loaded on first use.
"""
__all__ = ["inputs", "photonmc", "build"]
