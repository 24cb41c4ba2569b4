"""CPU FP64 oracle for the HDG local solve / static condensation / recovery path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  It shares
no code with the HIP library (``paper_1807_00086_amd``): the two are written
independently from the paper's formulation, and only the seeded input generator in
``synth`` serves both.

Plain, slow and direct: every local matrix is built by quadrature in physical
coordinates, every local solve uses ``numpy.linalg.solve`` (partial pivoting), the global
trace system is assembled with ``scipy.sparse`` and solved with a sparse direct solver.

Modules
  polynomials  Jacobi polynomials, orthonormal simplex bases, collapsed Gauss rules
  mesh         faces, adjacency, canonical face parametrisations, outward normals
  physics      local HDG matrices for acoustics, elastodynamics and Maxwell (with and without
               the GLM multiplier), and the paper's velocity / deformation-gradient elastic
               form used to pin the velocity / stress form
  postprocess  element-wise post-processing of the acoustic pressure (superconvergence pin)
  hdg          condensation, assembly, trace solve, recovery, full uncondensed solve,
               projections, norms, DIRK(3,3) stepping
"""
