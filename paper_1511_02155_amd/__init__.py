"""MI355X-native ternary free-energy lattice Boltzmann (arXiv:1511.02155).

The compute path is the HIP library ``libtlb.so`` (sources in ``csrc/``,
C ABI in ``include/tlb.h``); ``tlb`` is its thin ctypes binding and
``inputs`` builds seeded synthetic initial conditions.  Importing the
package does not load the library; ``paper_1511_02155_amd.tlb`` does, and
raises if it has not been built.
"""
__all__ = ["inputs", "tlb"]
