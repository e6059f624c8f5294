"""CPU oracle for the ILU(0)-preconditioned BiCGSTAB advection-diffusion solver.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU library never
does, and this package imports nothing from it.

``oracle.core`` binds the plain FP64 C implementation (``adr_oracle.c``);
``oracle.dense`` holds the small dense helpers used to pin it (exact discrete
solutions, the appendix's truncated-LU preconditioner, discretisation error).
"""
