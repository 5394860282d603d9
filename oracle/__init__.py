"""CPU oracle for the adaptive local-smoothing geometric multigrid method of
Clevenger, Heister, Kanschat and Kronbichler (arXiv:1904.03317).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or executes
this package; only the tests, the smoke entry point and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path: it is written from the
paper in plain Python, numpy and scipy.sparse, in float64 throughout, with
assembled sparse matrices and explicit hanging-node constraints.

Modules
  basis     1D Gauss-Lobatto nodes, Lagrange basis, reference mass/stiffness,
            family prolongation matrix                       (Sec. 2.1, 2.2)
  forest    forest of quad/hex trees, refinement, 2:1 closure, canonical
            (z-order) cell order                             (Sec. 2.3, 3.3)
  dofs      node identity, Dirichlet nodes, hanging constraints, leaf DoF
            numbering, level DoFs with S/I/D splitting, copy and family maps
                                                             (Sec. 2.3, Fig. 1)
  assemble  assembled leaf, level, mass and transfer matrices (Sec. 2.2, 2.3)
  mg        eigenvalue estimate, Chebyshev-Jacobi smoother, local-smoothing
            V-cycle, full-space V-cycle, preconditioned CG   (Alg. 1, Alg. 2,
                                                             Sec. 2.3, 4.1)
  problem   end-to-end driver: mesh + options -> solution, iterations, history

Functions without an independent pin say so in their docstring ("parity
unpinned").
"""
