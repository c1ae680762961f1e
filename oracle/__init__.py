"""Plain FP64 CPU oracle for the wedge Stokes operator of TERRA-NG (arXiv 2609.21633).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP path; it is
imported only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  The product path never calls it and
shares no code with it (the one common module is ``synthetic``, which draws
seeded inputs and holds none of the method's arithmetic).

What it computes, and from which passage of the paper:

* ``oracle.mesh``    -- icosahedral shell mesh: 12-vertex icosahedron, recursive
  geodesic midpoint refinement of its 20 spherical triangles, radial extrusion
  (Sec. 2 "Grid and Parallelization").  Built as a plain triangle mesh with no
  diamond index space, so it can be matched to the library only by coordinates.
* ``oracle.stokes``  -- per-wedge element matrices of eq:elemmat at the single
  quadrature point q_c = (1/3, 1/3, 0) (Sec. 3 eq:wedgebasis, eq:elemmat; Sec. 4
  eq:oneptenergy), the divergence coupling B, the iso-W1 pressure interpolation,
  assembly into a global sparse matrix (eq:matfree is the matrix-free form of
  exactly this sum), Dirichlet rows, SpMV and a sparse direct solve of the
  saddle-point system of Sec. 7.
* ``oracle.energy``  -- assembled lumped mass, diffusion, advection and SUPG
  matrices of the W1 temperature step (Sec. 6 scheme list).
* ``oracle.solver_ref`` -- textbook reference pieces used only to pin the
  preconditioner (eq:block-precond, eq:pmass).

Every function cites the passage it follows.  Readings of silent or ambiguous
passages are listed in the module docstrings.
"""
