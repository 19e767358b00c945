"""CPU FP64 oracle for the matrix-free GMG Stokes hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_1907_06696_amd/csrc`` and its Python binding) may import, call, link or
execute anything in this package.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously correct restatement of what the method
computes (Clevenger & Heister, "Comparison between algebraic and matrix-free
geometric multigrid for a Stokes problem on adaptive meshes with variable
viscosity", arXiv 1907.06696):

* ``fe``         -- Q2 / Q1 Lagrange reference element, Gauss rules, element
                    matrices of the weak form (Sec. 2.1, eq. weak_form and the
                    block system eq. stokes_linear_system).
* ``mesh``       -- unit-cube octree, 2:1 balance, global-coarsening level
                    meshes, Q2/Q1 node sets, Dirichlet and hanging-node
                    constraints.
* ``operators``  -- assembled and cellwise operators A, B, M_p, right-hand
                    side, level operators and transfers.
* ``multigrid``  -- Chebyshev smoother (Sec. 2.2.1), eigenvalue estimate,
                    coarse solve, V-cycle.
* ``krylov``     -- FGMRES with the block-triangular preconditioner (Sec. 2.2,
                    eq. stokes_precond; Sec. 2.2.2), CG, direct solve.
* ``rng``        -- SplitMix64 counter-based generator (Steele, Lea & Flood,
                    OOPSLA 2014), used for start vectors the method draws.
* ``learned``    -- MLP smoother scaling (not part of the paper; the learned
                    extension of the smoother).
* ``local_smoothing`` -- the local-smoothing level hierarchy and V-cycle.
* ``q3q2``       -- the Q3-Q2 pair (k = 2 of Sec. 2.1) on uniform meshes:
                    element, operators, transfers, GMG and the Stokes solve.

Where the paper is silent the oracle takes the readings listed in the design
notes (basis, quadrature, constraint weights, Chebyshev interval, ...); each
function names the reading it relies on.
"""
