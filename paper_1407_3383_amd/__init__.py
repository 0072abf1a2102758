"""MI355X-native exact NTT, polynomial-product and integer-product library.

The compute path lives in ``libntt_mi355x.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/ntt_mi355x.h``); ``paper_1407_3383_amd.ntt`` is the thin
ctypes binding.  ``paper_1407_3383_amd.inputs`` draws seeded synthetic inputs.
"""
