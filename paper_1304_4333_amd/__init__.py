"""MI355X-native hot path of the sequential posterior simulator (SPS) for
multinomial logit models (Geweke, Durham & Xu 2013).

The HIP library (libsps.so, C ABI declared in include/sps.h) is loaded lazily
by ``paper_1304_4333_amd.sps``; importing this package loads nothing.
"""
__all__ = ["synth", "sps"]
