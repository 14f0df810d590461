"""MI355X-native hot path of patch-to-volume reconstruction (PVR).

Submodules:
  synth   seeded synthetic inputs (phantoms, stacks, patches, motion draws)
  pvr     ctypes binding of the HIP library libpvr.so (loaded on first use)
  driver  the reconstruction cycle built from the library's calls
"""
__all__ = ["synth", "pvr", "driver"]
