"""CPU FP64 oracle for the circuit-contraction hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The
product path (``paper_2506_23775_amd``) never imports this package and shares
no code with it; the two meet only in the seeded input generators of
``workloads`` (which hold none of the method's arithmetic).

Everything is plain numpy in complex128 / float64: dense matrices, explicit
Kronecker embeddings, ``tensordot`` for the action of an embedded gate, and
dual numbers for directional derivatives.  Each function cites the passage of
the paper (arXiv 2506.23775) it follows.

Parity status of the functions (see the tests under ``tests/test_oracle_*``):
all functions are pinned by closed forms, brute force, exact Taylor
coefficients (FFT of the polynomial h(G + zX)) or finite differences, except
the conventions listed as "parity unpinned" in ``riemann.py`` (choice of the
orthonormal real tangent basis) and ``trust_region.py`` (trust-region
constants), which no value printed in the paper fixes.
"""

from .dense import (  # noqa: F401
    apply_gate,
    embed_kron,
    circuit_matrix_kron,
    circuit_matrix,
    cost,
    h_trace,
    forward_states,
    backward_states,
    hole_contraction,
    euclidean_T,
    tangent_T,
    hessian_holomorphic,
    hessian_by_holes,
    reference_columns,
    sector_columns,
)
from .riemann import (  # noqa: F401
    per_param,
    egrad,
    proj,
    rgrad,
    rhvp,
    real_basis,
    hessian_real,
    gradient_real,
    tangent_from_real,
    polar,
)
from .trust_region import tcg, tr_solve, tr_step  # noqa: F401
from .evaluate import evaluate  # noqa: F401
