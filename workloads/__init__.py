"""Seeded synthetic inputs for the circuit-contraction hot path.

This package only *generates inputs*: Fermi-Hubbard Hamiltonians and their
time-evolution targets, brick-wall circuit topologies, Haar-random gates and
tangent directions, and Trotter gate lists.  It holds none of the arithmetic of
the method itself (no cost, gradient, Hessian or contraction code), so both the
CPU oracle and the GPU path may import it without sharing any method code.
"""

from .hubbard import (  # noqa: F401
    spinful_fh_hamiltonian,
    target_unitary,
    strang_trotter_gates,
    hop_gate,
    fswap_gate,
    onsite_gate,
    local_hop_bond_operator,
)
from .circuits import (  # noqa: F401
    brickwall_pairs,
    haar_unitary,
    random_states,
    haar_gates,
    parity_haar_gates,
    number_haar_gates,
    NUMBER_MASK,
    tangent_direction,
    PARITY_MASK,
)
from .configs import CONFIGS, make_problem, Problem  # noqa: F401
