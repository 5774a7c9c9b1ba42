"""Plain, slow, FP64 CPU oracle of the Acc-FEM hot path.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the bench's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never
calls it, and it shares no code with that path: the two meet only through the
seeded input generators in ``workloads``.

It follows the paper's formulation (Sec. II, Sec. III) step by step, with numpy,
scipy (LAPACK banded LU, scipy.spatial.transform) and plain Python loops:

* ``beam``      - co-rotational 3D beam element: deformation measures, internal
                  force as the exact gradient of the element strain energy,
                  reference configuration (Sec. II-B, Sec. III-A eq. 20).
* ``actuation`` - cable tensions carried to the tip node as a follower wrench
                  (Sec. II-E, eq. 16-18).
* ``collision`` - brute-force node-versus-triangle contact detection and the
                  constraint rows and gaps (Sec. II-C eq. 3, 8-10; Sec. III-C).
* ``lcp``       - Lemke's complementary pivoting and brute-force enumeration for
                  the contact complementarity (eq. 12-13).
* ``solver``    - Newton iteration of the linearised contact problem with the
                  step-size limit (eq. 20-23, 25-27) and quasi-static load
                  stepping.
* ``adjoint``   - gradient of a tip-sensor loss with respect to the cable tensions
                  at a converged equilibrium (with the curvature of edge/vertex
                  contact constraints).
* ``admm``      - the operator-splitting (OSQP) iteration on the linear step's QP,
                  the solver Sec. III-B uses, as an alternative linear step.

Parity pins: every function is checked in tests/test_oracle_*.py against closed
forms (cantilever tip deflection, exact circular arc under a pure tip moment,
uniform axial shortening), invariances, finite differences and brute force.
"""
from . import beam, actuation, collision, lcp, solver, adjoint, admm  # noqa: F401
