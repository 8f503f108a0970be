"""C-ABI library checks that need no GPU: exported symbols, argument
validation, the sweep scheduler, and the host FP64 trust-region step."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rq():
    from paper_2506_23775_amd import rq as _rq
    if not os.path.exists(_rq.LIB_PATH):
        pytest.fail("librq.so not built (run paper_2506_23775_amd/build.py)")
    _rq.lib()
    return _rq


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(rq_[a-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(rq):
    L = rq.lib()
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(rq.EXPORTS)


def _circ(rq, k, pairs, **kw):
    return rq.Circuit(k, pairs, **kw)


def test_invalid_arguments(rq):
    L = rq.lib()
    bad = [
        (4, [(0, 0)]),      # q_hi == q_lo
        (4, [(0, 4)]),      # out of range
        (4, [(-1, 2)]),
    ]
    for k, pairs in bad:
        c = _circ(rq, k, pairs)
        assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
        assert b"invalid qubit pair" in L.rq_last_error()
    c = _circ(rq, 4, [(0, 1), (1, 2)], param_of=[0, 3], n_params=2)
    assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
    assert b"param_of" in L.rq_last_error()
    c = _circ(rq, 4, [(0, 1)])
    assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_GRAD, rq.RQ_C128, 65) == 0
    assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_GRAD, 7, 64) == 0
    c = _circ(rq, 3, [(0, 1)], parity=True)           # parity needs k >= 4
    assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
    # the Hessian workspace has its own sizing call: 0 and a message, never
    # the (too small) gradient layout
    c = _circ(rq, 4, [(0, 1), (1, 2)])
    assert L.rq_workspace_bytes(C.byref(c._c), rq.RQ_OP_HESS, rq.RQ_C128, 64) == 0
    assert b"rq_hess_workspace_bytes" in L.rq_last_error()
    assert L.rq_hess_workspace_bytes(C.byref(c._c), rq.RQ_C128, 64) > 0


def test_singular_gate_rejected_before_any_device_work(rq):
    L = rq.lib()
    c = _circ(rq, 4, [(0, 1), (2, 3)])
    g = np.zeros((2, 4, 4), dtype=np.complex128)
    g[0] = np.eye(4)
    # fake, never dereferenced device pointers: validation fails first
    t = rq._Target(rq.RQ_C128, 0, 0x1000, 16, 0)
    ex = rq._Exec(0x100000, 1 << 40, 64, None)
    f = C.c_double()
    st = L.rq_cost(C.byref(c._c), C.byref(t), rq._dptr(g), None, C.byref(ex), C.addressof(f))
    assert st == rq.RQ_ESINGULAR
    # range out of bounds is rejected too
    g[1] = np.eye(4)
    rg = rq._Range(-1, 0, 10, 10)
    st = L.rq_cost(C.byref(c._c), C.byref(t), rq._dptr(g), C.byref(rg), C.byref(ex), C.addressof(f))
    assert st == rq.RQ_EINVAL and b"range" in L.rq_last_error()
    # workspace too small
    ex2 = rq._Exec(0x100000, 16, 64, None)
    st = L.rq_cost(C.byref(c._c), C.byref(t), rq._dptr(g), None, C.byref(ex2), C.addressof(f))
    assert st == rq.RQ_ESPACE


def _check_plan(k, pairs, pass_of, parity, nt_max):
    n = len(pairs)
    # order of gates sharing a qubit is preserved across passes
    for q in range(k):
        seq = [pass_of[g] for g in range(n) if q in pairs[g]]
        assert seq == sorted(seq)
    # every pass fits a tile
    for p in set(pass_of):
        qs = set()
        for g in range(n):
            if pass_of[g] == p:
                qs |= set(pairs[g])
        if parity:
            qs.discard(k - 1)
        assert len(qs) <= nt_max


@pytest.mark.parametrize("k,layers,parity", [(8, 3, False), (12, 5, False), (16, 7, True),
                                             (16, 9, False), (6, 4, True)])
def test_scheduler_valid_and_fused(rq, k, layers, parity):
    pairs, _ = w.brickwall_pairs(k, layers)
    c = _circ(rq, k, pairs, parity=parity)
    for op, dt in [(rq.RQ_OP_HVP, rq.RQ_C64), (rq.RQ_OP_GRAD, rq.RQ_C128), (rq.RQ_OP_COST, rq.RQ_C64)]:
        n, pass_of = c.plan(op, dt)
        _check_plan(k, pairs, list(pass_of), parity, 5)
        assert n < len(pairs)        # several gates per pass


def test_scheduler_arbitrary_pairs(rq):
    rng = np.random.default_rng(3)
    k = 9
    pairs = []
    for _ in range(60):
        a, b = rng.choice(k, 2, replace=False)
        pairs.append((int(a), int(b)))
    c = _circ(rq, k, pairs)
    n, pass_of = c.plan(rq.RQ_OP_HVP, rq.RQ_C128)
    _check_plan(k, pairs, list(pass_of), False, 5)


def test_tangent_basis_matches_oracle(rq):
    for par in (False, True):
        B = rq.rq_tangent_basis(par)
        ref = np.stack(O.real_basis(par))
        assert np.abs(B - ref).max() < 1e-15


def test_tr_step_matches_oracle(rq):
    rng = np.random.default_rng(11)
    for par in (False, True):
        P = 3
        gates = (w.parity_haar_gates if par else w.haar_gates)(rng, P)
        d = 8 if par else 16
        n = P * d
        A = rng.standard_normal((n, n))
        H = A @ A.T / n - 0.3 * np.eye(n)
        g = rng.standard_normal(n)
        for delta in (0.05, 0.5, 5.0):
            eta, cand, md, stop = rq.rq_tr_step(gates, g, H, delta, parity=par)
            e_ref, why = O.tcg(g, H, delta)
            assert np.abs(eta - e_ref).max() < 1e-10
            X = O.tangent_from_real(gates, e_ref, par)
            cref = np.stack([O.polar(gates[p] + X[p]) for p in range(P)])
            assert np.abs(cand - cref).max() < 1e-12
            assert abs(md + (g @ e_ref + 0.5 * e_ref @ H @ e_ref)) < 1e-12
            assert {0: "converged", 1: "boundary", 2: "negative_curvature",
                    3: "max_iter", 4: "zero_gradient"}[stop] == why


def test_tr_accept_rule(rq):
    # rho < 1/4: radius quartered, rejected when rho <= 0.1
    nd, acc, rho = rq.rq_tr_accept(1.0, 0.99, 0.5, 1.0, 10.0, 1.0)
    assert nd == 0.25 and not acc and abs(rho - 0.02) < 1e-15
    nd, acc, rho = rq.rq_tr_accept(1.0, 0.5, 0.5, 1.0, 10.0, 1.0)
    assert nd == 2.0 and acc
    nd, acc, rho = rq.rq_tr_accept(1.0, 0.5, 0.5, 1.0, 10.0, 0.3)
    assert nd == 1.0 and acc


@pytest.mark.parametrize("parity", [False, True])
def test_tangent_coords_vs_oracle(rq, parity):
    """rq_tangent_coords (host) against the oracle's tangent coordinates of
    the Euclidean gradient."""
    rng = np.random.default_rng([61, parity])
    P = 5
    G = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    Y = rng.standard_normal((P, 4, 4)) + 1j * rng.standard_normal((P, 4, 4))
    if parity:
        Y = np.where(O.riemann.PARITY_MASK, Y, 0)
    got = rq.rq_tangent_coords(G, Y, parity=parity)
    ref = O.gradient_real(G, Y, parity)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_tr_solve_rejects_bad_arguments(rq):
    circ = rq.Circuit(4, [(0, 1), (2, 3)])
    t = rq._Target(rq.RQ_C128, 0, 8, 16, 0, None, 0, 0)
    ex = rq._Exec(256, 1 << 20, 64, None, 0, 0)
    G = np.stack([np.eye(4, dtype=complex)] * 2)
    n = C.c_int32(0)
    L = rq.lib()
    st = L.rq_tr_solve(C.byref(circ._c), C.byref(t), rq._dptr(G), None, C.byref(ex), -1, 0.0,
                       None, C.byref(n))
    assert st == rq.RQ_EINVAL
    st = L.rq_tr_solve(C.byref(circ._c), C.byref(t), rq._dptr(G), None, C.byref(ex), 3, 0.0,
                       None, C.byref(n))
    assert st == rq.RQ_ESPACE          # 1 MiB is below rq_tr_workspace_bytes
    assert L.rq_tr_workspace_bytes(C.byref(circ._c), rq.RQ_C128, 64) > (1 << 20)


def test_number_mode_host_functions(rq):
    """Particle-number mode on the host: tangent basis, coordinates and one
    trust-region step against the oracle; RQ_NUMBER needs RQ_PARITY."""
    B = rq.rq_tangent_basis("number")
    ref = np.stack(O.real_basis("number"))
    assert np.abs(B - ref).max() < 1e-15
    rng = np.random.default_rng(62)
    P = 4
    G = w.number_haar_gates(rng, P)
    Y = np.where(w.NUMBER_MASK, rng.standard_normal((P, 4, 4)) + 1j * rng.standard_normal((P, 4, 4)), 0)
    assert np.abs(rq.rq_tangent_coords(G, Y, "number") - O.gradient_real(G, Y, "number")).max() < 1e-13
    n = 6 * P
    A = rng.standard_normal((n, n))
    H = A @ A.T / n + 0.1 * np.eye(n)
    g = rng.standard_normal(n)
    delta = 0.7
    eta, cand, md, stop = rq.rq_tr_step(G, g, H, delta, "number")
    ref = O.tr_step(G, 0.0, g, H, delta, lambda X: 0.0, parity="number")
    assert np.abs(eta - ref["eta"]).max() < 1e-10
    assert np.abs(cand - ref["candidate"]).max() < 1e-10
    assert np.all(np.abs(cand[:, ~w.NUMBER_MASK]) < 1e-14)
    L = rq.lib()
    k = 6
    pairs, _ = w.brickwall_pairs(k, 2)
    bad = rq._Circuit(k, len(pairs), len(pairs), rq.RQ_NUMBER,
                      np.ascontiguousarray(np.asarray(pairs, dtype=np.int32)).ctypes.data_as(
                          C.POINTER(C.c_int32)), None, 0, 0)
    assert L.rq_workspace_bytes(C.byref(bad), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
    assert b"RQ_NUMBER" in L.rq_last_error()


def test_missing_library_fails_loudly(monkeypatch):
    """Without librq.so the binding raises instead of falling back."""
    from paper_2506_23775_amd import rq as _rq
    monkeypatch.setattr(_rq, "_lib", None)
    monkeypatch.setattr(_rq, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librq.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _rq.lib()
