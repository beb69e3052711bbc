"""MI355X-native non-LTE 3D radiative transfer: MALI smoother wrapped by FAS multigrid.

The compute path is the HIP/C-ABI library ``libnlte3d.so`` (built from ``csrc/``);
``nlte`` holds its ctypes binding and ``synth`` the seeded synthetic input generators.
Importing this package loads nothing; ``nlte.load()`` opens the library and raises if it
has not been built.
"""

__all__ = ["synth", "nlte"]
