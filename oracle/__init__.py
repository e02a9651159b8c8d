"""Plain FP64 CPU oracle for the matrix-free Poisson / multigrid-CG path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two meet
only through the seeded inputs of ``fem_inputs``.

Every function follows a definition from the paper (Betteridge, Farrell and
Ham, "Code generation for productive portable scalable finite element
simulation in Firedrake"):

* Section 2, eq. (1): -lap(u) = f in the unit cube, u = 0 on the boundary,
  generalised to -div(k grad u) = f with k a continuous piecewise-linear field.
* Section 2, eq. (4): the weak form, find u in V with
  int grad(u).grad(v) = int f v for all v in V.
* Section 2, Listing 1: UnitCubeMesh(N,N,N), MeshHierarchy(mesh, 2),
  FunctionSpace(mesh, "CG", degree), DirichletBC on all six faces.
* Section 4, Listing 2: multigrid with 2 Chebyshev smoothing steps per level
  and a direct coarse solve.

Arithmetic is float64 except the reference-element tensors, which are exact
rationals (fractions.Fraction) converted to float64 once.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""
