"""dfamin: massively parallel DFA minimization on AMD Instinct MI355X (gfx950).

Signature-based partition refinement with a parallel partial transitive
closure (Martens & Wijs, "An Evaluation of Massively Parallel Algorithms for
DFA Minimization", GandALF 2024), as hand-written HIP kernels behind the
C-ABI in ``include/dfamin.h``.

Submodules:
  ``dfamin``     ctypes binding to ``libdfamin.so`` (same names as the C-ABI)
  ``workloads``  seeded synthetic DFA generators (inputs only)
  ``build``      compiles the HIP library for gfx950

Importing the package loads nothing; ``paper_2410_22764_amd.dfamin`` loads
the native library on first use and raises if it is missing.
"""
__all__ = ["dfamin", "workloads", "build"]
