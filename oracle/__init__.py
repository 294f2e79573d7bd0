"""CPU reference oracle for the grid-overlay FD method (test infrastructure).

This package is a plain, slow, FP64 CPU implementation of what the GPU path
computes, written from the paper (Huang & Shen, "A grid-overlay finite
difference method for the fractional Laplacian on arbitrary bounded
domains").  Where the method has a plain definition (the Toeplitz product,
point location, the transfer matrix, the solution of the linear system) the
oracle writes that definition out; where it is an algorithm (the Filon
quadrature with Richardson extrapolation, incomplete Cholesky, conjugate
gradients) it takes the paper's steps in the paper's order.

It is test infrastructure only: the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library and its Python
binding never do.  It shares no code with the HIP path; both sides only read
the seeded inputs of the ``workloads`` package.

Every function cites the passage it follows.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""

__all__ = ["grid", "fdweights", "afd", "predicates", "transfer", "operator", "precond", "solve",
           "exact", "adjoint"]
