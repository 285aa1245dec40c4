"""Plain FP64 CPU oracle for the HOTRG coarse-graining step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls anything in this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do.  It shares no code,
table or helper with the GPU path.

Modules
-------
hotrg   -- the method itself, step by step in the paper's order (Sections 2-4).
exact   -- closed forms and brute force used to pin the oracle (Onsager's 2D
           Ising free energy, exhaustive sums over tiny periodic tori).
tangent -- forward-mode derivative d(lnZ/V)/d(beta) of the oracle run.
"""
