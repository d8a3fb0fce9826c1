"""MI355X-native global-placement hot path of analytical heterogeneous die-to-die 3D placement.

Submodules: ``place3d`` (binding to the HIP library), ``autograd`` (autograd Functions),
``synth`` (seeded synthetic netlists).  Nothing is imported eagerly.
"""
__all__ = ["place3d", "autograd", "synth"]
