"""FP64 CPU oracle for the collision-aware local/global soft-robot solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path (the HIP library
and its Python binding) never does, and the two share no code.

It follows the paper's method step by step (Sections II-III, Eqs. 1-9 and
the inner loop of Algorithm 1) in double precision:

* ``mesh``     - set-up: oriented tets, rest shapes, weights, surface, A_el.
* ``local``    - the local projection of every element onto its target
                 (Section III-A; Eqs. 6 and 7).
* ``collide``  - brute-force collision detection and the virtual-spring
                 active set (Sections II-B, II-C, III-A.3; Eqs. 3-5, 8).
* ``solve``    - right-hand side, exact sparse direct global step, energy
                 (Eq. 9) and the local/global iteration.
* ``adjoint``  - gradients w.r.t. the per-chamber volume ratios: implicit
                 (at a fixed point with the contact set frozen) and unrolled
                 (through K recorded iterations), by automatic
                 differentiation of the plain definitions.

Readings of passages the paper leaves open are listed where they are used.
"""
from .mesh import Params, Problem, orient, ORIENT_SWAP
from .local import local_step, mooney_rivlin_weight
from .collision import collide, Contacts
from .solver import solve, global_step, energy, residual_rhs
from .adjoint import grad, unrolled_grad, record_path

__all__ = ["Params", "Problem", "orient", "ORIENT_SWAP", "local_step", "mooney_rivlin_weight",
           "collide", "Contacts", "solve", "global_step", "energy", "residual_rhs", "grad",
           "unrolled_grad", "record_path"]
