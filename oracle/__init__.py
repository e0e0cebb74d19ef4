"""Plain FP64 CPU oracle of the implicit FLD radiation-energy update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes anything in this package; only
the tests, the package's smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the GPU path.

Modules
-------
fldref       coefficient stage, operator assembly, exact linear solve,
             exchange quartic, opacity law, full step (Sect. 2-3 of the paper).
linear_modes linearised static FLD + exchange response and the octic
             dispersion relation of Appendix B (used as pins).
"""
