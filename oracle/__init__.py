"""Plain, slow FP64 CPU implementation of Hierarchical Particle-Mesh (HPM).

TEST INFRASTRUCTURE ONLY. This package is the parity oracle for the HIP library. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the product code never
does, and it shares no code, tables or constants with the HIP path.

Modules:
  tables  -- gridlet nodes, Vandermonde matrix A and its inverse B (Sec. 2.2), the child-to-parent
             matrices T^C (Sec. 2.3), the exact lattice Green function (Eq. 1)
  tree    -- the oct-tree rule and the cube-complete zone geometry (Sec. 1)
  hpm     -- the method's steps in the paper's order (Sec. 1 and 2): P2M, M2M, M2L (direct gridlet
             sum or one zero-padded FFT), L2L, L2P and the near-zone direct sum
  direct  -- the O(N^2) softened direct sum used as the force-error reference
"""
