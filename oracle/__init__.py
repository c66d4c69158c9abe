"""CPU FP64 oracle for the IFGF-accelerated N-Mueller forward map.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the bench's CPU
baseline leg do.  It shares no code with the HIP path.

Modules, each citing the passage of Paul & Sideris, "Accelerated 3D Maxwell
Integral Equation Solver using the Interpolated Factored Green Function
Method" (arXiv 2408.02274) that it follows:

  cheb       open Chebyshev grid, Fejer weights, Chebyshev expansion and
             differentiation (Sec. III-A eq. cheby_nodes, Sec. III-C
             eq. fejer_weighs, Sec. III-E interpolation formula)
  greens     Helmholtz Green's function and its gradient (Sec. II)
  direct     O1: the plain O(N^2) regular sums that IFGF approximates
             (Sec. III-E eq. ifgf_sum, Sec. III-I eq. ifgf_sum_em)
  ifgf_ref   O2: the reference IFGF, step by step (Sec. III-E..III-I)
  surface    node weights, normals, tangent basis, surface derivatives
             (Sec. III-A, Sec. III intro)
  singular   rectangular-polar singular moments and local corrections
             (Sec. III-D, Sec. III-H)
  nmuller    densities, operator assembly, right-hand side (Sec. II
             eq. n_muller .. t_delta)
  gmres      plain GMRES (Sec. III-A eq. lin_system)
  mie        Mie series for the dielectric sphere (textbook; Sec. IV-B check)
  mlp        NumPy MLP forward/backward used to check the preconditioner
             kernels' gradients (project addition, not in the paper)

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
