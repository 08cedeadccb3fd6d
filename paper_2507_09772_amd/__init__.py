"""MI355X-native Coulomb/exchange (J/K) matrix build.

The compute path is the HIP library under ``csrc/``; ``jk`` is its thin
ctypes binding.  ``synth`` holds the seeded synthetic workloads.
"""
__all__ = ["jk", "synth"]
