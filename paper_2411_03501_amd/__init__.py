"""hjx: MI355X-native explicit Hamilton-Jacobi level-set time stepping
(the hot path of LevelSetPy, arXiv 2411.03501).

The solver itself lives in the HIP library libhjx.so behind the C-ABI
declared in include/hjx.h; `paper_2411_03501_amd.hjx` is the ctypes binding
(argument marshalling only).  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["hjx", "inputs"]
