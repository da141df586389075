"""ORBGRAND on AMD Instinct MI355X: a C-ABI HIP library (liborbgrand.so) and its
ctypes binding.  Import the binding with ``from paper_2202_13951_amd import binding``."""
