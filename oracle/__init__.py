"""FP64 CPU oracle of the SPS hot path (test infrastructure only).

Imported only by the test suite, the smoke check and the CPU baseline of the
benchmark; the product path never imports it.
"""
