"""MI355X-native global adaptive-velocity-space (AVS) discrete-velocity sweep.

The computation lives in the HIP library ``libavs.so`` (C ABI in
``include/avs.h``); ``paper_2212_05645_amd.avs`` is its ctypes binding.
"""
__all__ = ["avs"]
