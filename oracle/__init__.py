"""CPU oracle of the DCA collision step -- test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never does.
"""
