"""Reference oracle for replica-exchange Wang-Landau sampling.

TEST INFRASTRUCTURE ONLY: a plain, slow CPU implementation written from the
paper (arXiv:1402.2328) plus exact densities of states that pin it.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
anything from this package; the GPU library never does.
"""
