"""MI355X-native k-mer counting (the hot path of KMC 2, Deorowicz et al. 2014).

The counting runs in hand-written HIP kernels behind the C ABI of
``libkmc_hip.so`` (include/kmc.h); ``kmc`` is its ctypes binding and
``synth`` makes seeded synthetic read sets.
"""
