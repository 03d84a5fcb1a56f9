"""hdsw: trace-transfer diagonal sweeping DDM for the Helmholtz equation with
PML on one AMD Instinct MI355X (arXiv:2003.02585, Algorithms 2.1 / 4.1).

``paper_2003_02585_amd.hdsw``     -- ctypes binding of libhdsw (C-ABI in
                                     include/hdsw.h); importing it requires
                                     the built library.
``paper_2003_02585_amd.workloads`` -- seeded synthetic inputs.
"""
