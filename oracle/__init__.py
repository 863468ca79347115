"""CPU FP64 oracle for recursive skeletonization of the 2D Stokes double layer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the GPU path: the only common
dependency is the `workloads` input generator, which holds none of the
method's arithmetic.

Contents (all plain NumPy/SciPy in float64, written from the paper):
  stokes  - the kernels of Section 3.1 (stresslet double layer with its jump
            term, the rank-one null-space completion N, Stokeslets, rotlets,
            the rigid-motion null space Psi) and the dense augmented system of
            eq. (backwardeq); dense LU solve; interior evaluation eq. (forwardeq).
  tree    - the adaptive quadtree of Section 2.3.
  cpqr    - Householder QR with column pivoting and the interpolative
            decomposition of Section 2.2 / eq. (lowrank).
  rs      - the level-parallel recursive skeletonization of Sections 2.2-2.7
            with the bordered root solve of Section 3.2 (eq. partition), and
            the box-marking update of Section 2.8.

Parity status per function is stated in each module header.
"""
