"""MI355X-native Monte-Carlo sweeps of the 3D Edwards-Anderson Heisenberg spin glass.

Yavors'kii & Weigel, "Optimized GPU simulation of continuous-spin glass models"
(arXiv:1204.6192). The compute path lives in the HIP library ``libhsg.so``
(``csrc/``), reached through the thin ctypes binding in :mod:`.hsg`. The seeded
synthetic input generators live in :mod:`.inputs`.

Importing the package loads nothing; ``from paper_1204_6192_amd import hsg``
loads the library and raises if it has not been built.
"""

__all__ = ["hsg", "inputs"]
__version__ = "0.1.0"
