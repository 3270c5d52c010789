"""MI355X-native hot path of a multibeam radio-transient pipeline.

RFI thresholding, brute-force incoherent dedispersion, per-DM normalisation
and n-sigma detection as HIP kernels for gfx950 behind the C ABI of
include/mbtp.h (libmbtp.so); ``api`` is the Python binding.
"""
__all__ = ["api", "synth", "build"]
