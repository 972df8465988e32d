"""MI355X-native split-step Crank-Nicolson solver for the 3D Gross-Pitaevskii equation.

The compute path is the HIP library ``csrc/`` builds (``libgpsscn.so``, C-ABI declared in
``include/gp.h``); ``gp.py`` is its thin ctypes binding.  Importing the package loads
nothing; ``gp.load()`` loads the library and raises if it is missing.
"""
__all__ = ["gp", "inputs"]
