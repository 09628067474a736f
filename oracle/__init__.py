"""CPU FP64 oracle for the MPS lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library.

Two independent programs live here:

* ``dense_lbm`` - the plain definition: a dense FP64 D3Q19 BGK lattice
  Boltzmann solver (collide then stream, Section 3.1 of the paper) with the
  same inverse-density approximation, equilibrium assembly, forcing and
  boundary rules that the MPS method uses, so that an untruncated MPS run
  must reproduce it up to rounding.
* ``mps`` / ``mps_lbm`` - the method itself, step by step: matrix product
  states over scale-ordered indices (Section 2), their algebra, the
  variational compressed Hadamard product (Section 2.3), the shift MPOs
  (Section 2.5) and the MPS-LBM step (Section 3.2), in plain numpy/LAPACK.
"""
