"""Plain FP64 CPU oracle for the deflated-multigrid Wilson-Dirac solve.

TEST INFRASTRUCTURE ONLY.  This package exists so that tests, the smoke check
and the CPU-baseline leg of the benchmark can check the HIP solver against an
independent, slow, obviously correct implementation written from the paper
(Whyte, Wilcox, Morgan, "Deflated GMRES with Multigrid for Lattice QCD").  No
product code imports it, and it shares no code, headers, tables or helpers with
the HIP library; the only thing both sides consume is the seeded input arrays
of the ``synth`` package.

Everything is numpy / scipy complex128.  Operators are scipy sparse matrices
built entry by entry from their definitions, and the solvers follow the steps
of the methods in the order the literature states them.

Modules
    wilson      the 2D U(1) Wilson-Dirac operator (Methods section)
    mcrit       critical mass from the low spectrum (Results section, "mass gap")
    krylov      CG, GMRES, FGMRES, GMRES-DR and GMRES-Proj (Methods section)
    precision   bfloat16 rounding of stored blocks (the BF16 preconditioner variant)
    multigrid   near-null vectors, prolongators, Galerkin operators, the cycle,
                the partial intermediate solve and the outer solve (Methods)

Parity status of each function is stated in its docstring; functions without a
pin say "parity unpinned".
"""
