"""Plain CPU FP64 oracle of the HHG P1 multigrid hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path.

It works on one global vector per level (every micro-vertex once, in the
canonical order) with sparse matrices assembled element by element, which is
the plain definition of what the structured, ghost-layered, matrix-free HIP
path computes:

  mesh.py       macro mesh -> refined levels, canonical numbering (paper
                sec. 2.1, 3.1, 3.2)
  assemble.py   P1 stiffness / mass matrices from element matrices (sec. 4.1,
                4.2: a stencil is a row of the stiffness matrix), injection
                of the coefficient, and one-row-at-a-time evaluation
                (rows_at) for sampled checks at full size
  mg.py         staged multicolour Gauss-Seidel, residual, restriction,
                prolongation, Jacobi-PCG coarse solve, V-cycle, solve loop
                (sec. 4.3)
  net.py        the learned smoother's forward/backward (not in the paper)
  partition.py  the same level stored as one block per macro-primitive with
                explicit ghost copies and a packer for the four exchange
                directions (sec. 2.2, Alg. 3), checked against the global
                vector
  stokes.py     equal-order P1-P1 Stokes with pressure stabilisation, the
                block-diagonal multigrid preconditioner and preconditioned
                MINRES (sec. 4.3, 5.2)
  transport.py  finite-volume upwind transport of the temperature on the
                micro-triangles and its coupling to Stokes (sec. 3.1, 5.2)
  p2.py         quadratic elements on the refined faces and p-multigrid with
                the P1 hierarchy (sec. 3.1, 4.2, 4.3)

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
from .mesh import MacroMesh, Level  # noqa: F401
