"""CPU oracle for the MP matrix products and LU (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
anything here.  The library (paper_1410_1599_amd) never does, and the oracle
imports nothing from the library.  Modules:

* mpnum  -- p-bit round-to-nearest-even scalar arithmetic on Python ints
* gemm   -- Simple, Block, Strassen, Winograd, the recursion and its op counts
* lu     -- blocked LU with partial pivoting, solve, exact residual
* exact  -- exact products and ulp errors (yardstick for the slice path)
* cref   -- ctypes wrapper of the C twin in oracle/c/mpref.c (large sizes)
* conditioning -- exact condition numbers of the Lotkin matrix (Section 4)
"""
