"""MI355X-native lane detection hot path (Fan & Dahnoun, arXiv 1807.02752).

The compute runs in the HIP library libld.so (see include/ld.h); `ld` is its thin Python
binding.  `synth` generates seeded synthetic stereo-road frames.
"""
