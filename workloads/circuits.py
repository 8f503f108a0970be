"""Circuit topologies and random gate / direction generators.

* Brick wall on a ring of k qubits: layer l even holds the pairs (2s, 2s+1),
  layer l odd the pairs (2s+1, 2s+2 mod k); gates are listed layer by layer
  (the paper's sequentialisation of a brick wall, Sec. "Brick wall circuit
  layout").  Pairs are given as (q_hi, q_lo); a gate's row/column index is
  2*bit(q_hi) + bit(q_lo), so the wrap gate (k-1, 0) is the translate of the
  bulk gates.
* Haar-random U(m) by QR of a complex Gaussian matrix with the phases of R's
  diagonal moved into Q (Mezzadri's construction).  Draw order: the real part
  (m x m), then the imaginary part.
* Parity-conserving gates (paper eq. for the parity gate matrix): nonzeros at
  rows/columns {0,3} (even block) and {1,2} (odd block).  The even block is
  drawn first, then the odd block, each Haar on U(2).
"""

from __future__ import annotations

import numpy as np

#: 4x4 boolean mask of the parity-conserving gate pattern.
PARITY_MASK = np.array([[1, 0, 0, 1],
                        [0, 1, 1, 0],
                        [0, 1, 1, 0],
                        [1, 0, 0, 1]], dtype=bool)


def brickwall_pairs(k: int, n_layers: int):
    """List of (q_hi, q_lo) in application order and the layer of each gate."""
    if k % 2 or k < 2:
        raise ValueError("k must be even and >= 2")
    pairs, layer_of = [], []
    for l in range(n_layers):
        for s in range(k // 2):
            if l % 2 == 0:
                p = (2 * s, 2 * s + 1)
            else:
                p = (2 * s + 1, (2 * s + 2) % k)
            pairs.append(p)
            layer_of.append(l)
    return pairs, layer_of


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def haar_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    z = _complex_gaussian(rng, (m, m))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def random_states(rng: np.random.Generator, dim: int, n: int) -> np.ndarray:
    """n Haar-random unit vectors of dimension dim, as the columns of a
    [dim, n] complex128 array (normalised complex Gaussians)."""
    z = _complex_gaussian(rng, (dim, n))
    return z / np.linalg.norm(z, axis=0, keepdims=True)


def haar_gates(rng: np.random.Generator, n: int) -> np.ndarray:
    return np.stack([haar_unitary(rng, 4) for _ in range(n)])


def parity_haar_gates(rng: np.random.Generator, n: int) -> np.ndarray:
    out = np.zeros((n, 4, 4), dtype=np.complex128)
    ev, od = [0, 3], [1, 2]
    for p in range(n):
        be = haar_unitary(rng, 2)
        bo = haar_unitary(rng, 2)
        out[p][np.ix_(ev, ev)] = be
        out[p][np.ix_(od, od)] = bo
    return out


def number_haar_gates(rng: np.random.Generator, n: int) -> np.ndarray:
    """Particle-number-conserving gates U(1) x U(2) x U(1) on {00}, {01, 10},
    {11}: a Haar U(2) block on the odd states, then two uniform phases."""
    out = np.zeros((n, 4, 4), dtype=np.complex128)
    od = [1, 2]
    for p in range(n):
        out[p][np.ix_(od, od)] = haar_unitary(rng, 2)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=2)
        out[p][0, 0] = np.exp(1j * ph[0])
        out[p][3, 3] = np.exp(1j * ph[1])
    return out


NUMBER_MASK = np.array([[1, 0, 0, 0],
                        [0, 1, 1, 0],
                        [0, 1, 1, 0],
                        [0, 0, 0, 1]], dtype=bool)


def tangent_direction(rng: np.random.Generator, gates: np.ndarray,
                      parity=False) -> np.ndarray:
    """Seeded random tangent vector X_p = G_p A_p with A_p the anti-Hermitian
    part of a complex Gaussian matrix (restricted to the parity pattern in
    parity mode, to the particle-number pattern for parity="number"),
    normalised so that sum_p ||X_p||_F^2 = 1."""
    out = np.empty_like(gates)
    for p in range(gates.shape[0]):
        z = _complex_gaussian(rng, (4, 4))
        if parity == "number":
            z = np.where(NUMBER_MASK, z, 0)
        elif parity:
            z = np.where(PARITY_MASK, z, 0)
        a = 0.5 * (z - z.conj().T)
        out[p] = gates[p] @ a
    return out / np.sqrt(np.sum(np.abs(out) ** 2))
