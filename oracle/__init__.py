"""Plain, slow, FP64 CPU oracle of the FNPF-SEM per-stage Laplace-solve path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package; the
product path (the HIP library and its Python binding) never does, and this
package never imports the product.  It shares no code with the HIP path:
the only common dependency is the seeded input package ``workloads`` (meshes
and analytic data, no method arithmetic).

Each module follows the paper (Visbech, Melander, Engsig-Karup, "FNPF-SEM: A
parallel spectral element model in Firedrake for fully nonlinear water wave
simulations"), citing the section/equation it implements:

* ``gll``       GLL nodes, weights, derivative matrix (nodal Lagrange P^p, Sec. 3.1)
* ``geometry``  extruded, surface-following mesh and per-point factors (Sec. 3.1.2)
* ``operator``  Laplace bilinear form a[phi; nu] (Eq. 4): assembled and matrix-free
* ``solve``     Dirichlet lift at the free surface, Neumann data, CG solve (Eq. 1, Sec. 4),
                and the vertical line blocks of A_II with their block solve
* ``surface``   vertical-velocity recovery (Sec. 3.4 Steps 4.4-4.5) and the
                Zakharov free-surface right-hand side (Eqs. 2-3, 5)
* ``timestep``  ERK4 (Sec. 3.2), relaxation zones (Sec. 3.3), mass and energy

All arithmetic is written so that it also runs in complex128, which lets
``timestep`` provide complex-step directional derivatives (a tangent-linear
reference that shares nothing with a hand-written adjoint).
"""
