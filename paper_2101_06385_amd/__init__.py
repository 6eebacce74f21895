"""SP2 density matrices on AMD Instinct MI355X (gfx950).

The compute path lives in the HIP library `libsp2.so` (sources in `csrc/`, C ABI in
`include/sp2.h`); `sp2` is a thin ctypes binding with the same entry-point names.
Importing the package does not load the library; the first call does, and fails
loudly if it has not been built.
"""
__all__ = ["sp2", "workloads"]
