"""rq_hess_blocks with a declared translation symmetry (only translation-
unique hole pairs swept, Sec. "Exploiting translational invariance") against
the same call without it and against the oracle; sub-ranges and input states
ignore the symmetry."""

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import rel

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-6}


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


def _np(t):
    return t.detach().cpu().numpy()


def _hess(rq, k, pairs, layer, gates, tgt, parity, shift, **kw):
    circ = rq.Circuit(k, pairs, param_of=layer, parity=parity, shift=shift)
    return [None if x is None else _np(x) for x in rq.rq_hess_blocks(circ, tgt, gates, **kw)]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("case", ["parity_exact", "dense_exact", "parity_trotter"])
def test_shift_equals_full_hole_set(rq, dtype, case):
    rng = np.random.default_rng([101, dtype, len(case)])
    k = 8
    parity = case.startswith("parity")
    layers = 5 if parity else 4
    pairs, layer = w.brickwall_pairs(k, layers)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, layers)
    if case.endswith("trotter"):
        gl = w.strang_trotter_gates(4, 0.5, 4, 1.0, 4.0)
        tgt = rq.build_trotter_target(k, gl, dtype=dtype, parity=True)
        shift = 4
    else:
        tgt = rq.Target.from_dense(w.target_unitary(4, 0.5, 1.0, 4.0), dtype, parity=parity)
        shift = 2
    a = _hess(rq, k, pairs, layer, gates, tgt, parity, 0, chunk=64)
    b = _hess(rq, k, pairs, layer, gates, tgt, parity, shift, chunk=64)
    for x, y in zip(a, b):
        assert rel(y, x) <= TOL[dtype], rel(y, x)


def test_shift_against_oracle(rq):
    rng = np.random.default_rng(102)
    k = 6
    pairs, layer = w.brickwall_pairs(k, 3)
    layer = np.asarray(layer)
    gates = w.parity_haar_gates(rng, 3)
    U = w.target_unitary(3, 0.5, 1.0, 4.0)
    tgt = rq.Target.from_dense(U, rq.RQ_C128, parity=True)
    _, eg, _, hh, hr = _hess(rq, k, pairs, layer, gates, tgt, True, 2, chunk=64)
    inst = gates[layer]
    Hi = O.hessian_holomorphic(k, pairs, inst, U, mask=O.riemann.PARITY_MASK)
    P, N = 3, len(pairs)
    Hp = np.zeros((P, 4, 4, P, 4, 4), dtype=complex)
    for l in range(N):
        for m in range(N):
            Hp[layer[l], :, :, layer[m]] += Hi[l, :, :, m]
    pidx = [0, 3, 12, 15, 5, 6, 9, 10]
    Hh = Hp.reshape(P, 16, P, 16)[:, pidx][:, :, :, pidx]
    assert rel(hh, Hh) <= 1e-10
    T = np.where(O.riemann.PARITY_MASK, O.per_param(O.euclidean_T(k, pairs, inst, U), layer, P), 0)
    assert rel(hr, O.hessian_real(gates, O.egrad(T), Hp, True)) <= 1e-10


def test_shift_ignored_for_subrange_and_inputs(rq):
    import torch
    rng = np.random.default_rng(103)
    k = 8
    pairs, layer = w.brickwall_pairs(k, 3)
    gates = w.parity_haar_gates(rng, 3)
    U = w.target_unitary(4, 0.5, 1.0, 4.0)
    tgt = rq.Target.from_dense(U, rq.RQ_C128, parity=True)
    a = _hess(rq, k, pairs, layer, gates, tgt, True, 0, range=(1, 7, 90), chunk=64)
    b = _hess(rq, k, pairs, layer, gates, tgt, True, 2, range=(1, 7, 90), chunk=64)
    for x, y in zip(a, b):
        assert rel(y, x) <= 1e-13
    Z = torch.from_numpy(w.random_states(rng, 1 << (k - 1), 2 * 20).reshape(-1, 2, 20)
                         .transpose(1, 0, 2).copy()).cuda()
    ref = torch.stack([tgt.ref[p] @ Z[p] for p in (0, 1)]).contiguous()
    ti = rq.Target(ref, rq.RQ_C128, True, inputs=Z.contiguous())
    a = _hess(rq, k, pairs, layer, gates, ti, True, 0, range=(-1, 0, 20), chunk=64)
    b = _hess(rq, k, pairs, layer, gates, ti, True, 2, range=(-1, 0, 20), chunk=64)
    for x, y in zip(a, b):
        assert rel(y, x) <= 1e-13


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("case", ["parity_exact", "dense_exact", "parity_trotter"])
def test_orbit_reduced_basis_sum_equals_full(rq, dtype, case):
    """One basis state per translation orbit, weighted by the orbit size
    (rq.orbit_target), reproduces the full basis sum of f, both gradients
    and the HVP."""
    rng = np.random.default_rng([104, dtype, len(case)])
    k = 8
    parity = case.startswith("parity")
    layers = 5 if parity else 4
    pairs, layer = w.brickwall_pairs(k, layers)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, layers)
    direction = w.tangent_direction(rng, gates, parity=parity)
    if case.endswith("trotter"):
        gl = w.strang_trotter_gates(4, 0.5, 4, 1.0, 4.0)
        tgt = rq.build_trotter_target(k, gl, dtype=dtype, parity=True)
        shift = 4
    else:
        tgt = rq.Target.from_dense(w.target_unitary(4, 0.5, 1.0, 4.0), dtype, parity=parity)
        shift = 2
    circ = rq.Circuit(k, pairs, param_of=layer, parity=parity, shift=shift)
    full = [_np(x) for x in rq.rq_hvp(circ, tgt, gates, direction, chunk=64)]
    ot = rq.orbit_target(circ, tgt)
    R = ot.ref.shape[-1]
    assert R < (1 << (k - 1 if parity else k)) * (3 if shift == 4 else 2) // 4
    red = [_np(x) for x in rq.rq_hvp(circ, ot, gates, direction, range=(-1, 0, R), chunk=64)]
    tol = 1e-12 if dtype == 0 else 1e-5
    assert abs(red[0] - full[0]) <= tol * max(1.0, abs(full[0]))
    for x, y in zip(red[1:], full[1:]):
        assert rel(x, y) <= tol, rel(x, y)


def test_orbit_reduced_config3(rq):
    """Configuration 3 at k = 16 (Strang target, two-site symmetry): the
    orbit-reduced evaluation (8264 + 8192 representatives instead of 2 x 2^15
    basis states) agrees with the full one in c64 and c128."""
    prob = w.make_problem(3, trotter_steps=20)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, parity=True, shift=4)
    for dtype, tol in ((rq.RQ_C128, 1e-11), (rq.RQ_C64, 1e-5)):
        tgt = rq.build_trotter_target(prob.k, prob.trotter, dtype=dtype, parity=True)
        full = [_np(x) for x in rq.rq_hvp(circ, tgt, prob.gates, prob.direction, chunk=2048)]
        ot = rq.orbit_target(circ, tgt)
        R = ot.ref.shape[-1]
        assert R == 8264
        red = [_np(x) for x in rq.rq_hvp(circ, ot, prob.gates, prob.direction, range=(-1, 0, R),
                                          chunk=2048)]
        assert abs(red[0] - full[0]) <= tol * max(1.0, abs(full[0]))
        for x, y in zip(red[1:], full[1:]):
            assert rel(x, y) <= tol, (dtype, rel(x, y))
        del tgt, ot


def _orbits_bits(k, s):
    """Orbit representatives (smallest index) and sizes of the basis states
    under q -> q + s, by explicit bit lists (no library code)."""
    seen = {}
    for x in range(1 << k):
        b = [(x >> (k - 1 - q)) & 1 for q in range(k)]
        orb = set()
        for _ in range(k):
            b = [b[(q - s) % k] for q in range(k)]
            orb.add(sum(v << (k - 1 - q) for q, v in enumerate(b)))
        seen[min(orb)] = len(orb)
    reps = np.array(sorted(seen))
    return reps, np.array([seen[r] for r in reps])


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("parity", [False, True])
def test_orbit_target_abi_vs_oracle_weighted_sum(rq, dtype, parity):
    """rq_orbit_target (orbit representatives filled on the device through
    the C ABI) followed by rq_hvp equals the oracle's orbit-weighted sum: the
    oracle evaluates the input states sqrt(w_r)|rep_r> (representatives and
    weights from explicit bit lists) against U sqrt(w_r)|rep_r>."""
    rng = np.random.default_rng([105, dtype, parity])
    k, layers, shift = 8, 4, 2
    pairs, layer = w.brickwall_pairs(k, layers)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, layers)
    direction = w.tangent_direction(rng, gates, parity=parity)
    U = w.target_unitary(k // 2, 0.5, 1.0, 4.0)
    circ = rq.Circuit(k, pairs, param_of=layer, parity=parity, shift=shift)
    tgt = rq.Target.from_dense(U, dtype, parity=parity)
    ot = rq.orbit_target(circ, tgt)
    R = ot.ref.shape[-1]
    got = rq.rq_hvp(circ, ot, gates, direction, range=(-1, 0, R), chunk=64)
    reps, wts = _orbits_bits(k, shift)
    Z = np.zeros((1 << k, len(reps)), dtype=complex)
    Z[reps, np.arange(len(reps))] = np.sqrt(wts)
    ref = O.evaluate(k, pairs, gates, layer, direction, U @ Z, None, parity=parity, inputs=Z)
    tol = 1e-12 if dtype == 0 else 1e-5
    assert abs(float(got[0]) - ref["f"]) <= tol * max(1.0, abs(ref["f"]))
    for key, x in zip(["egrad", "rgrad", "ehvp", "rhvp"], got[1:]):
        assert rel(_np(x), ref[key]) <= tol, key
    # the device slabs hold exactly the weighted representatives
    inp = _np(ot.inputs)
    if parity:
        par = np.array([bin(int(v)).count("1") & 1 for v in reps])
        for p in (0, 1):
            rp, wp = reps[par == p] >> 1, wts[par == p]
            assert np.allclose(inp[p][rp, np.arange(len(rp))], np.sqrt(wp))
            assert np.count_nonzero(inp[p]) == len(rp)
    else:
        assert np.allclose(inp[reps, np.arange(len(reps))], np.sqrt(wts))
        assert np.count_nonzero(inp) == len(reps)
