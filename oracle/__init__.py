"""Plain, slow, FP64 CPU oracle for the DEC beam-propagation method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it, links it or reads its output, and it shares no code
with the library (no kernels, headers, helpers or tables).

What it computes, in the paper's order and notation:

* ``dec``        topology (incidence matrices D0, D1), Hodge stars H0 and the
                 Galerkin/Whitney H1, stiffness D0^T H1 D0, the potential
                 stars H0(V), the averaging matrix Q and Q^T D Q, and the
                 operators of the semi-discrete ODE (Eqs. 10-14).
* ``stepper``    z-marching: exact Kerr/absorber flow, classical RK4 for the
                 linear part, Strang composition (half steps are never merged).
* ``unsplit``    z-marching of the whole right-hand side (Kerr term inside
                 every stage): classical RK4 at a fixed step and the adaptive
                 Dormand-Prince 5(4) pair with its step-size controller.
* ``soliton``    nonlinear eigenmodes (soliton launches) by imaginary-z
                 propagation with power renormalisation.
* ``diagnostics`` power, Hamiltonian, overlap, the paper's intensity error
                 (Eq. 15) and the plain relative L2 error.
* ``adjoint``    the exact reverse of ``stepper.propagate`` for the overlap objective,
                 with gradients w.r.t. the launch field and a per-vertex index
                 perturbation.

Readings of the paper where it is silent or inconsistent are stated in the
functions that take them.  Every function here is pinned by a CPU test
against a closed form, invariant, hand-computed value or brute-force result.
"""
from .dec import Operators, assemble  # noqa: F401
from .stepper import propagate, strang_step, nl_flow, lin_rk4  # noqa: F401
from .unsplit import rhs, rk4_step, propagate_rk4, propagate_dp54  # noqa: F401
from .soliton import find_mode  # noqa: F401
from .diagnostics import power, hamiltonian, overlap, e_rel, rel_l2  # noqa: F401
