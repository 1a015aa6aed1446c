"""CPU FP64 oracle for the direction-split ("phisplit") exponential integrators.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (no kernels, headers, helpers, tables or constant
generators); the two meet only in the seeded problem definitions of the
``workloads`` package, which hold none of the method's arithmetic.

Contents (plain NumPy / SciPy, float64 / complex128, written for reading
against the paper rather than for speed):

* ``phi``       -- phi_l(X) of small dense matrices (section 1, eqs. integraldef
                   and seriesdef), via the exponential of an augmented block
                   matrix (a textbook identity, not the paper's phiquad).
* ``tensor``    -- mu-mode product, Tucker operator, Kronecker-sum action,
                   dense Kronecker sum and the element loop (eqs. kronsum,
                   vecexp, tuckerexp, forloop).
* ``nonlinear`` -- the nonlinearities g of the workloads.
* ``schemes``   -- Lawson-Euler, Lawson2b, exponential Euler and ETD2RK in
                   the tensor (phisplit) form of section 3.2, and exponential
                   Rosenbrock-Euler for Riccati-type matrix equations (eq.
                   expRosEulertensor with the Kronecker-sum Jacobian).
* ``norms``     -- error measures and the observed order.

Parity status: every function is pinned by the tests under
``tests/test_oracle_*.py`` (brute force on tiny sizes, closed forms, the
paper's printed errors of section 4.2, invariants; for Rosenbrock-Euler the
Jacobian against central differences, the unsplit step with the exact phi_1 of
the assembled Jacobian, and the order against a Runge-Kutta reference).  The
Riccati steppers have no printed values to reproduce (the paper's Riccati
experiment needs a reference solution it does not specify); their pins are
dense brute force on small instances, the matrix form against the vec form,
and these invariants.
"""

from . import phi, tensor, nonlinear, schemes, norms  # noqa: F401
