"""MI355X-native HSWO / HSEG / RHSEG hot path (hyperspectral region merging).

The product is the C-ABI library libhswo.so (include/hswo.h) built from the
HIP sources in csrc/; ``hswo`` is its thin Python binding and ``synth`` the
seeded synthetic-cube generators.
"""
