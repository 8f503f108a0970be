"""Pins of the oracle's input-state path (trace over vectors other than the
basis, Sec. "Conclusions"): the sum over any orthonormal basis equals the
basis-state trace (Tr A = sum_r v_r^dagger A v_r), for f, the gradients, the
HVP and the Hessian; and the random-vector (Hutchinson) estimate is unbiased
(E[z z^dagger] = I)."""

import numpy as np

import oracle as O
import workloads as w
from gpu_helpers import sector_full_index


def _problem(rng, k, layers, parity=False):
    pairs, _ = w.brickwall_pairs(k, layers)
    P = len(pairs)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    direction = w.tangent_direction(rng, gates, parity=parity)
    return pairs, np.arange(P), gates, direction


def _close(a, b, tol):
    for key in b:
        x, y = np.asarray(a[key]), np.asarray(b[key])
        assert np.abs(x - y).max() <= tol * max(1.0, np.abs(y).max()), key


def test_orthonormal_inputs_equal_basis_trace():
    rng = np.random.default_rng(31)
    k = 6
    pairs, param_of, gates, direction = _problem(rng, k, 3)
    U = w.haar_unitary(rng, 1 << k)
    V = w.haar_unitary(rng, 1 << k)
    full = O.evaluate(k, pairs, gates, param_of, direction, U, None)
    rot = O.evaluate(k, pairs, gates, param_of, direction, U @ V, None, inputs=V)
    _close(rot, full, 1e-12)


def test_orthonormal_inputs_equal_basis_trace_parity_sectors():
    rng = np.random.default_rng(32)
    k = 6
    pairs, param_of, gates, direction = _problem(rng, k, 3, parity=True)
    U = w.target_unitary(3, 0.5, 1.0, 4.0)
    full = O.evaluate(k, pairs, gates, param_of, direction, U, None, parity=True)
    n = 1 << (k - 1)
    vin = np.zeros((1 << k, 2 * n), dtype=complex)
    for p in (0, 1):
        rows = sector_full_index(k, p, np.arange(n))
        vin[rows, p * n:(p + 1) * n] = w.haar_unitary(rng, n)
    rot = O.evaluate(k, pairs, gates, param_of, direction, U @ vin, None, parity=True,
                     inputs=vin)
    _close(rot, full, 1e-12)


def test_orthonormal_inputs_hessian():
    rng = np.random.default_rng(33)
    k = 4
    pairs = [(0, 1), (2, 3), (1, 2)]
    gates = w.haar_gates(rng, 3)
    U = w.haar_unitary(rng, 1 << k)
    V = w.haar_unitary(rng, 1 << k)
    H = O.hessian_holomorphic(k, pairs, gates, U, None)
    Hv = O.hessian_holomorphic(k, pairs, gates, U @ V, None, inputs=V)
    assert np.abs(Hv - H).max() <= 1e-12 * np.abs(H).max()


def test_random_vector_estimate_is_unbiased():
    """Mean of the complex-Rademacher estimate over 2000 vectors (fixed seed)
    against the exact trace, within 5 standard errors, for f and every
    gradient entry; a global phase of z does not change a summand."""
    rng = np.random.default_rng(34)
    k = 4
    pairs, param_of, gates, _ = _problem(rng, k, 2)
    U = w.haar_unitary(rng, 1 << k)
    exact = O.evaluate(k, pairs, gates, param_of, None, U, None)
    R = 2000
    Z = (1j ** rng.integers(0, 4, size=(1 << k, R))).astype(complex)
    fs, egs = [], []
    for c in range(R):
        z = Z[:, c:c + 1]
        e = O.evaluate(k, pairs, gates, param_of, None, U @ z, None, inputs=z)
        fs.append(e["f"])
        egs.append(e["egrad"])
    fs = np.asarray(fs)
    egs = np.asarray(egs)
    se = fs.std(ddof=1) / np.sqrt(R)
    assert abs(fs.mean() - exact["f"]) <= 5 * se + 1e-12
    m = egs.mean(axis=0)
    se_g = np.sqrt(egs.real.var(axis=0, ddof=1) + egs.imag.var(axis=0, ddof=1)) / np.sqrt(R)
    assert np.all(np.abs(m - exact["egrad"]) <= 5 * se_g + 1e-12)
    # the sum over the R vectors at once equals the sum of the single summands
    tot = O.evaluate(k, pairs, gates, param_of, None, U @ Z, None, inputs=Z)
    assert abs(tot["f"] - fs.sum()) <= 1e-9 * max(1.0, abs(tot["f"]))
    z = Z[:, :1]
    a = O.evaluate(k, pairs, gates, param_of, None, U @ z, None, inputs=z)["f"]
    b = O.evaluate(k, pairs, gates, param_of, None, U @ (1j * z), None, inputs=1j * z)["f"]
    assert abs(a - b) <= 1e-12 * max(1.0, abs(a))
