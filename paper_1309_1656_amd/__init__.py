"""Matrix-valued quantum lattice Boltzmann method on AMD Instinct MI355X.

The compute path is the HIP library ``libmlbm.so`` built from ``csrc/``; the
Python layer (``mlbm``) only marshals arguments.  Importing this package does
not load the library: the first call into ``mlbm`` does, and raises if the
library has not been built.
"""
