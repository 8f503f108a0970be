"""The five workload configurations (seeded, synthetic).

Each workload is a spinful Fermi-Hubbard ring (J = 1, periodic, interleaved
spins) whose time-evolution operator is the target U, and a brick-wall circuit
of two-qubit gates whose cost f, Riemannian gradient, Hessian-vector product
and Hessian blocks are evaluated.

Seeds: numpy ``default_rng([250623775, cfg])``.  Draw order per configuration:
gates in parameter order (each gate: real part, then imaginary part of its
Gaussian matrix), then the tangent direction.

=====  ==  ======  =======  ========================================================
 cfg    k  layers  gates    target / notes
=====  ==  ======  =======  ========================================================
  1     8    3     12 Haar  dense exp(-iHt), U=4, t=0.25
  2    12    5     30 Haar  dense exp(-iHt), U=4, t=0.5
  3    16    7     56 inst. Strang Trotter (200 steps, t=1.0); one shared parity
                   7 params gate per layer; two parity sectors of 2^15
  4    16    9     72 Haar  same Trotter target as 3; general gates
  5     -    -     -        serving mix (see ``serving_requests``)
=====  ==  ======  =======  ========================================================
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .circuits import (brickwall_pairs, haar_gates, parity_haar_gates,
                       tangent_direction)
from .hubbard import strang_trotter_gates, target_unitary

SEED = 250623775

CONFIGS = {
    1: dict(k=8, n_layers=3, U=4.0, t=0.25, parity=False, shared=False,
            target="dense"),
    2: dict(k=12, n_layers=5, U=4.0, t=0.5, parity=False, shared=False,
            target="dense"),
    3: dict(k=16, n_layers=7, U=4.0, t=1.0, parity=True, shared=True,
            target="trotter", trotter_steps=200),
    4: dict(k=16, n_layers=9, U=4.0, t=1.0, parity=False, shared=False,
            target="trotter", trotter_steps=200),
}


@dataclass
class Problem:
    name: str
    k: int
    n_layers: int
    pairs: List[Tuple[int, int]]
    layer_of: np.ndarray
    param_of: np.ndarray
    gates: np.ndarray          # [P,4,4] complex128 (one per parameter)
    direction: np.ndarray      # [P,4,4] complex128 tangent direction
    parity: bool
    U: float
    t: float
    J: float = 1.0
    U_ref: Optional[np.ndarray] = None            # dense target (k <= 12)
    trotter: Optional[list] = None                # target as a gate list
    extra: dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return len(self.pairs)

    @property
    def n_params(self) -> int:
        return self.gates.shape[0]

    def instance_gates(self) -> np.ndarray:
        return self.gates[self.param_of]


def make_problem(cfg: int, *, k: Optional[int] = None, n_layers: Optional[int] = None,
                 dense_target: Optional[bool] = None, trotter_steps: Optional[int] = None,
                 seed_tag: Optional[int] = None) -> Problem:
    """Build configuration ``cfg`` (1..4).  ``k`` / ``n_layers`` /
    ``trotter_steps`` override the sizes (reduced-size variants for tests keep
    every other recipe unchanged); ``dense_target`` forces a dense exp(-iHt)."""
    c = dict(CONFIGS[cfg])
    if k is not None:
        c["k"] = k
    if n_layers is not None:
        c["n_layers"] = n_layers
    if trotter_steps is not None:
        c["trotter_steps"] = trotter_steps
    if dense_target is not None:
        c["target"] = "dense" if dense_target else "trotter"
    rng = np.random.default_rng([SEED, cfg if seed_tag is None else seed_tag])
    kq = c["k"]
    pairs, layer_of = brickwall_pairs(kq, c["n_layers"])
    layer_of = np.asarray(layer_of, dtype=np.int32)
    if c["shared"]:
        param_of = layer_of.copy()
        n_params = c["n_layers"]
    else:
        param_of = np.arange(len(pairs), dtype=np.int32)
        n_params = len(pairs)
    gates = parity_haar_gates(rng, n_params) if c["parity"] else haar_gates(rng, n_params)
    direction = tangent_direction(rng, gates, parity=c["parity"])
    n_sites = kq // 2
    prob = Problem(name=f"cfg{cfg}", k=kq, n_layers=c["n_layers"], pairs=pairs,
                   layer_of=layer_of, param_of=param_of, gates=gates,
                   direction=direction, parity=c["parity"], U=c["U"], t=c["t"])
    if c["target"] == "dense":
        prob.U_ref = target_unitary(n_sites, c["t"], 1.0, c["U"])
    else:
        prob.trotter = strang_trotter_gates(n_sites, c["t"], c["trotter_steps"], 1.0, c["U"])
    return prob


def serving_requests(n_requests: int, rate_hz: float, *, ks=(8, 10, 12, 14, 16),
                     depths=(3, 5, 7, 9), ops=("f", "grad", "hvp")):
    """Configuration 5: a Poisson stream of f / grad / HVP requests.

    Returns dicts with arrival time, k, depth, U in [2,8], t in [0.25,2], op
    and a per-request seed tag; gates and directions are generated from
    ``default_rng([SEED, 5, r])`` by :func:`request_problem`."""
    rng = np.random.default_rng([SEED, 5, 0])
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        out.append(dict(rid=r, arrival=t, k=int(rng.choice(ks)),
                        depth=int(rng.choice(depths)),
                        U=float(rng.uniform(2.0, 8.0)), t=float(rng.uniform(0.25, 2.0)),
                        op=str(rng.choice(ops))))
    return out


def request_problem(req: dict, trotter_steps: int = 40, dense_max_k: int = 12) -> Problem:
    """Circuit, gates and target of one serving request.  Targets are dense
    exp(-iHt) for k <= dense_max_k and a Strang Trotter gate list beyond."""
    rng = np.random.default_rng([SEED, 5, req["rid"] + 1])
    k = req["k"]
    pairs, layer_of = brickwall_pairs(k, req["depth"])
    gates = haar_gates(rng, len(pairs))
    direction = tangent_direction(rng, gates)
    prob = Problem(name=f"req{req['rid']}", k=k, n_layers=req["depth"], pairs=pairs,
                   layer_of=np.asarray(layer_of, dtype=np.int32),
                   param_of=np.arange(len(pairs), dtype=np.int32), gates=gates,
                   direction=direction, parity=False, U=req["U"], t=req["t"])
    if k <= dense_max_k:
        prob.U_ref = target_unitary(k // 2, req["t"], 1.0, req["U"])
    else:
        prob.trotter = strang_trotter_gates(k // 2, req["t"], trotter_steps, 1.0, req["U"])
    return prob
