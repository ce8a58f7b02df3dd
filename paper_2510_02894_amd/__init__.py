"""MI355X-native 3D shape features (marching-cubes area/volume and maximum
diameters) behind a C-ABI HIP library.

The compiled library is loaded lazily by ``paper_2510_02894_amd.shape3d`` on
first use; importing the package does not touch the GPU.
"""
__all__ = ["shape3d", "synth"]
