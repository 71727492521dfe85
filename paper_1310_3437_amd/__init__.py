"""MI355X-native DCA collision step (arXiv:1310.3437): a C-ABI HIP library
(libkmc.so) with a thin ctypes binding.

    from paper_1310_3437_amd import kmc      # the binding (needs libkmc.so)
    from paper_1310_3437_amd import inputs   # seeded synthetic workloads
"""
