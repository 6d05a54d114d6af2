"""bnx: BFGS-preconditioned Inexact Newton eigensolver (DACG-Newton) for one MI355X.

The solver is the HIP library ``libbnx.so`` (C-ABI in ``include/bnx.h``);
``bnx`` is its ctypes binding and ``workloads`` the seeded input generators.
"""
