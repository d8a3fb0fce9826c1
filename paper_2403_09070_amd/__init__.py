"""MI355X-native global-placement hot path of analytical heterogeneous die-to-die 3D placement.

Submodules: ``place3d`` (binding to the HIP library), ``autograd`` (torch.autograd Functions over
it), ``synth`` (seeded synthetic netlists), ``build`` (compiles the library).  Nothing is imported
eagerly.
"""
__all__ = ["place3d", "autograd", "synth"]
