"""MI355X-native dust-particle hot path (gather, exponential-midpoint push,
deposit) of Mignone, Flock & Vaidya (2019), as hand-written HIP kernels for
gfx950 behind a C ABI (``include/dust.h``).

``paper_1908_10793_amd.dust`` is the thin Python binding (argument
marshalling only); ``paper_1908_10793_amd.synth`` draws seeded inputs.
Importing the package loads nothing native.
"""
__all__ = ["dust", "synth"]
