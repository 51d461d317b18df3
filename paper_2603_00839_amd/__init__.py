"""MI355X-native RTG-GMRES (randomized tensor global GMRES) hot path.

``paper_2603_00839_amd.rtg`` is the ctypes binding of the HIP library
``librtg.so`` (C ABI declared in ``include/rtg.h``); ``synth`` holds the
seeded synthetic input generators.
"""
