"""MI355X-native hot path of the JUMP integrator (velocity jumps for MD).

The compute path lives in the HIP library libjumpmd.so (paper_2412_15073_amd/csrc);
`paper_2412_15073_amd.jumpmd` is its thin ctypes binding and `systems` builds
seeded synthetic inputs.
"""
__all__ = ["systems", "jumpmd"]
