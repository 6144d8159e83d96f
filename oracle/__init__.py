"""Oracle: a plain, slow, FP64 CPU implementation of the vertex-patch smoother
with a nested p-multigrid local solver (arXiv 2510.17785), written from the
paper's statement of the method.

THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it.  The GPU library never calls it
and shares no code with it; the two meet only in the seeded inputs of the
`synth` package.

Everything here assembles matrices explicitly (element, patch, level and
global matrices) and applies them as dense or sparse matrix-vector products,
so that each step can be checked against the paper by eye:

  fe1d      -- Gauss-Lobatto-Legendre nodes, Gauss-Legendre rule, Lagrange basis
  fem       -- multilinear cell maps, element matrices of a(u,v)=int mu grad u.grad v
               (Section 2, bilinear form), patch and global assembly, coarse
               meshes (coefficient means, or box-wise coefficients integrated
               by the octant rule)
  pmg       -- p-transfers, level operators, Chebyshev-Jacobi smoothing and the
               local p-multigrid V-cycle (Section 3.1, Algorithm 2)
  smoother  -- vertex patches, colouring and the multiplicative sweep
               (Section 2.1, Algorithm 1)
  lanczos   -- eigenvalue bounds of D^{-1}A for the Chebyshev interval
  gmg       -- h-transfers, the global V-cycle and the outer CG (Section 2, Section 4)
  mlp       -- the bound-predicting network, forward/backward/Adam in FP64
  simplex   -- simplicial patches (3 quadrilaterals / 4 hexahedra around a
               vertex, Section 3.2): numbering, level matrices, transfers and
               their V-cycle
"""
