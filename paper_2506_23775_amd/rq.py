"""Thin ctypes binding of librq (argument marshalling only).

Every computation runs in librq's HIP kernels; this module only converts
numpy / torch arguments to the C structures of ``include/rq.h``, owns the
device workspace and returns device results as torch tensors.  It raises
``RuntimeError`` when the library is missing or a call fails (there is no
fallback implementation).

Conventions follow ``include/rq.h``: gates are complex [P, 4, 4] arrays
indexed by 2*bit(q_hi) + bit(q_lo); qubit 0 is the most significant bit of a
basis index; in parity mode states are sector-compressed (row x >> 1).
"""

from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librq.so")

RQ_OK, RQ_EINVAL, RQ_EHIP, RQ_ESPACE, RQ_ESINGULAR = 0, 1, 2, 3, 4
RQ_C128, RQ_C64 = 0, 1
RQ_PARITY = 1
RQ_NUMBER = 2
RQ_SECTORS = 4
RQ_OP_COST, RQ_OP_GRAD, RQ_OP_HVP, RQ_OP_HESS, RQ_OP_APPLY = 0, 1, 2, 3, 4


class _Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_gates", C.c_int32), ("n_params", C.c_int32),
                ("flags", C.c_uint32), ("pairs", C.POINTER(C.c_int32)),
                ("param_of", C.POINTER(C.c_int32)), ("shift", C.c_int32),
                ("reserved", C.c_int32)]


class _Target(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("reserved", C.c_int32), ("ref", C.c_void_p),
                ("ld", C.c_int64), ("sector_stride", C.c_int64), ("inputs", C.c_void_p),
                ("in_ld", C.c_int64), ("in_sector_stride", C.c_int64)]


class _Range(C.Structure):
    _fields_ = [("sector", C.c_int32), ("reserved", C.c_int32), ("begin", C.c_int64),
                ("count", C.c_int64)]


class _Exec(C.Structure):
    _fields_ = [("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("chunk", C.c_int64), ("stream", C.c_void_p), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]

RQ_EXEC_ACCUMULATE = 1


_lib = None

EXPORTS = ["rq_workspace_bytes", "rq_cost", "rq_grad", "rq_hvp", "rq_hess_blocks",
           "rq_hess_workspace_bytes", "rq_apply_circuit", "rq_tr_step", "rq_tr_accept",
           "rq_tangent_coords", "rq_tr_workspace_bytes", "rq_tr_solve",
           "rq_tangent_basis", "rq_plan_passes", "rq_profile_enable", "rq_profile_read",
           "rq_stream_copy", "rq_hvp_static", "rq_orbit_reps", "rq_orbit_workspace_bytes",
           "rq_orbit_target", "rq_sector_rows", "rq_strerror", "rq_last_error"]


def lib():
    """Load librq.so (built in-tree by ``paper_2506_23775_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: run paper_2506_23775_amd/build.py "
                           "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.rq_workspace_bytes.restype = C.c_size_t
    L.rq_workspace_bytes.argtypes = [C.POINTER(_Circuit), C.c_int32, C.c_int32, C.c_int64]
    L.rq_hess_workspace_bytes.restype = C.c_size_t
    L.rq_hess_workspace_bytes.argtypes = [C.POINTER(_Circuit), C.c_int32, C.c_int64]
    common = [C.POINTER(_Circuit), C.POINTER(_Target), dp]
    L.rq_cost.argtypes = common + [C.POINTER(_Range), C.POINTER(_Exec), P]
    L.rq_grad.argtypes = common + [C.POINTER(_Range), C.POINTER(_Exec), P, P, P]
    L.rq_hvp.argtypes = common + [dp, C.POINTER(_Range), C.POINTER(_Exec), P, P, P, P, P]
    L.rq_hess_blocks.argtypes = common + [C.POINTER(_Range), C.POINTER(_Exec), P, P, P, P, P]
    L.rq_apply_circuit.argtypes = [C.POINTER(_Circuit), dp, P, C.c_int64, C.c_int64,
                                   C.c_int32, C.c_int32, C.POINTER(_Exec)]
    L.rq_tr_step.argtypes = [C.c_int32, C.c_uint32, dp, dp, dp, C.c_double, dp, dp, dp,
                             C.POINTER(C.c_int32)]
    L.rq_tr_accept.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                               C.c_double, dp, C.POINTER(C.c_int32), dp]
    L.rq_tangent_basis.argtypes = [C.c_uint32, dp]
    L.rq_tangent_coords.argtypes = [C.c_int32, C.c_uint32, dp, dp, dp]
    L.rq_tr_workspace_bytes.restype = C.c_size_t
    L.rq_tr_workspace_bytes.argtypes = [C.POINTER(_Circuit), C.c_int32, C.c_int64]
    L.rq_tr_solve.argtypes = [C.POINTER(_Circuit), C.POINTER(_Target), dp, C.POINTER(_Range),
                              C.POINTER(_Exec), C.c_int32, C.c_double, dp,
                              C.POINTER(C.c_int32)]
    L.rq_plan_passes.argtypes = [C.POINTER(_Circuit), C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.rq_profile_enable.argtypes = [C.c_int]
    L.rq_profile_read.argtypes = [dp, C.POINTER(C.c_int64), dp, dp]
    L.rq_stream_copy.argtypes = [P, P, C.c_size_t, C.c_int32, C.c_int32, P]
    L.rq_orbit_reps.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), dp]
    L.rq_orbit_workspace_bytes.restype = C.c_size_t
    L.rq_orbit_workspace_bytes.argtypes = [C.POINTER(_Circuit), C.c_int64]
    L.rq_orbit_target.argtypes = [C.POINTER(_Circuit), C.POINTER(_Target), P, P, C.c_int64,
                                  C.POINTER(_Exec)]
    L.rq_hvp_static.argtypes = common + [dp, C.POINTER(_Range), P, C.c_uint32,
                                         C.POINTER(C.c_int64), P, P, P, P, P]
    L.rq_sector_rows.argtypes = [C.c_int32, C.POINTER(C.c_int64)]
    L.rq_strerror.restype = C.c_char_p
    L.rq_last_error.restype = C.c_char_p
    for name in ["rq_sector_rows", "rq_cost", "rq_grad", "rq_hvp", "rq_hess_blocks", "rq_apply_circuit",
                 "rq_tr_step", "rq_tr_accept", "rq_tangent_basis", "rq_plan_passes",
                 "rq_tangent_coords", "rq_tr_solve", "rq_stream_copy", "rq_hvp_static",
                 "rq_orbit_reps", "rq_orbit_target",
                 "rq_profile_enable", "rq_profile_read"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class RQError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.rq_last_error().decode()
        super().__init__(f"{where}: {L.rq_strerror(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status, where):
    if status != RQ_OK:
        raise RQError(status, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _gates_host(g) -> np.ndarray:
    g = g.detach().cpu().numpy() if isinstance(g, torch.Tensor) else np.asarray(g)
    g = np.ascontiguousarray(g.astype(np.complex128)).reshape(-1, 4, 4)
    return g


# ---------------------------------------------------------------------------
# Circuit / target descriptions
# ---------------------------------------------------------------------------

class Circuit:
    """Gate topology: k qubits, pairs [(q_hi, q_lo)], optional param_of."""

    def __init__(self, k: int, pairs: Sequence, param_of=None, n_params: Optional[int] = None,
                 parity: bool = False, shift: int = 0, number: bool = False,
                 sectors: bool = False):
        self.k = int(k)
        self.pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        self.n_gates = self.pairs.shape[0]
        if param_of is None:
            self.param_of = None
            self.n_params = self.n_gates if n_params is None else int(n_params)
        else:
            self.param_of = np.ascontiguousarray(np.asarray(param_of, dtype=np.int32))
            self.n_params = int(self.param_of.max()) + 1 if n_params is None else int(n_params)
        self.parity = bool(parity) or bool(number)
        self.number = bool(number)      # particle-number-conserving gates (implies parity)
        # states stored per particle-number sector (requires number)
        self.sectors = bool(sectors)
        self.shift = int(shift)   # translation symmetry (qubits), 0: none
        self.flags = (RQ_PARITY if self.parity else 0) | (RQ_NUMBER if self.number else 0) | \
            (RQ_SECTORS if self.sectors else 0)
        self._c = _Circuit(self.k, self.n_gates, self.n_params, self.flags,
                           self.pairs.ctypes.data_as(C.POINTER(C.c_int32)),
                           None if self.param_of is None
                           else self.param_of.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.shift, 0)

    @property
    def kq(self):
        return self.k - 1 if self.parity else self.k

    @property
    def ncols(self):
        """Basis columns of the largest sector (parity: 2^(k-1); particle
        number: C(k, k // 2); general: 2^k)."""
        if self.sectors:
            return math.comb(self.k, self.k // 2)
        return 1 << self.kq

    def plan(self, op: int, dtype: int):
        pass_of = np.zeros(self.n_gates, dtype=np.int32)
        n = lib().rq_plan_passes(C.byref(self._c), op, dtype,
                                 pass_of.ctypes.data_as(C.POINTER(C.c_int32)))
        if n < 0:
            raise RQError(-n, "rq_plan_passes")
        return n, pass_of


def torch_dtype(dtype: int):
    return torch.complex128 if dtype == RQ_C128 else torch.complex64


def sector_rows(k: int, p: int) -> np.ndarray:
    """Full basis indices of the compressed rows x' of parity sector p."""
    xp = np.arange(1 << (k - 1), dtype=np.int64)
    par = np.zeros_like(xp)
    v = xp.copy()
    while np.any(v):
        par ^= v & 1
        v >>= 1
    return (xp << 1) | (par ^ p)


def sector_order(k: int) -> np.ndarray:
    """Stacked particle-number-sector row of every basis index x < 2^k
    (rq_sector_rows): sectors by particle number, states of a sector in
    increasing order."""
    rows = np.zeros(1 << k, dtype=np.int64)
    _check(lib().rq_sector_rows(k, rows.ctypes.data_as(C.POINTER(C.c_int64))), "rq_sector_rows")
    return rows


def sector_bounds(k: int):
    """[(first stacked row, size)] of the particle-number sectors n = 0..k."""
    sizes = [math.comb(k, n) for n in range(k + 1)]
    first = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return [(int(f), int(d)) for f, d in zip(first, sizes)]


@dataclass
class Target:
    """Device target columns.  ``ref``: general [2^k, width] (U[x][j]) or
    parity [2, 2^(k-1), width] sector blocks, complex64 / complex128 on cuda.
    ``inputs`` (optional, same shape as ref): input states psi_j replacing the
    basis states |j>; ref column j then holds U psi_j."""

    ref: torch.Tensor
    dtype: int
    parity: bool
    col_offset: int = 0     # ref holds the columns [col_offset, col_offset + width)
    inputs: Optional[torch.Tensor] = None

    @staticmethod
    def _geometry(t: torch.Tensor, parity: bool):
        if t.dtype not in (torch.complex64, torch.complex128) or not t.is_contiguous():
            raise ValueError("target / input slabs must be contiguous complex tensors")
        if parity:
            if t.dim() != 3 or t.shape[0] != 2:
                raise ValueError("parity slabs are [2, 2^(k-1), width]")
            return t.shape[2], t.shape[1] * t.shape[2]
        if t.dim() != 2:
            raise ValueError("general slabs are [2^k, width]")
        return t.shape[1], 0

    def struct(self):
        ld, ss = self._geometry(self.ref, self.parity)
        esize = self.ref.element_size()
        # the C ABI addresses column j at ref + x*ld + j: shift the base so that
        # a window of columns starting at col_offset is addressed by global j
        ref = self.ref.data_ptr() - self.col_offset * esize
        if self.inputs is None:
            return _Target(self.dtype, 0, ref, ld, ss, None, 0, 0)
        if self.inputs.shape != self.ref.shape or self.inputs.dtype != self.ref.dtype:
            raise ValueError("inputs must have the shape and dtype of ref")
        ild, iss = self._geometry(self.inputs, self.parity)
        return _Target(self.dtype, 0, ref, ld, ss,
                       self.inputs.data_ptr() - self.col_offset * esize, ild, iss)

    @staticmethod
    def from_dense_sectors(U: np.ndarray, dtype: int = RQ_C128, device="cuda"):
        """Particle-number-sector target (RQ_SECTORS) from a dense U that
        conserves particle number: [2^k, C(k, k//2)] with the block of sector
        n at rows [first(n), first(n) + C(k, n)), columns [0, C(k, n))."""
        U = np.asarray(U)
        k = int(np.log2(U.shape[0]))
        order = np.argsort(sector_order(k))          # stacked row -> basis index
        width = math.comb(k, k // 2)
        ref = np.zeros((1 << k, width), dtype=np.complex128)
        for first, size in sector_bounds(k):
            idx = order[first:first + size]
            ref[first:first + size, :size] = U[np.ix_(idx, idx)]
        t = torch.from_numpy(ref).to(torch_dtype(dtype))
        return Target(t.to(device), dtype, False)

    @staticmethod
    def from_dense(U: np.ndarray, dtype: int = RQ_C128, parity: bool = False, device="cuda"):
        U = np.asarray(U)
        k = int(np.log2(U.shape[0]))
        if parity:
            blocks = np.stack([U[np.ix_(sector_rows(k, p), sector_rows(k, p))] for p in (0, 1)])
            t = torch.from_numpy(np.ascontiguousarray(blocks)).to(torch_dtype(dtype))
        else:
            t = torch.from_numpy(np.ascontiguousarray(U)).to(torch_dtype(dtype))
        return Target(t.to(device), dtype, parity)


# ---------------------------------------------------------------------------
# Workspace
# ---------------------------------------------------------------------------

class Workspace:
    """Caller-owned device workspace (the library allocates no device memory)."""

    def __init__(self, nbytes: int, device="cuda"):
        self.buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.offset = (-base) % 256
        self.ptr = base + self.offset
        self.nbytes = int(nbytes)


_ws_cache = {}


def _workspace(nbytes: int, stream, key=()) -> Workspace:
    """Default workspace of calls that pass none: one cached buffer per
    (device, stream, key).  Calls on one stream run in order, so they may
    share it; calls on different streams never do (concurrent calls need
    distinct workspaces).  A larger request replaces the stream's buffer;
    the old one is released to torch's caching allocator on the current
    stream, which orders its reuse after the work already enqueued there."""
    k = (torch.cuda.current_device(), int(stream.cuda_stream)) + tuple(key)
    ws = _ws_cache.get(k)
    if ws is None or ws.nbytes < nbytes:
        _ws_cache.pop(k, None)
        with torch.cuda.stream(stream):
            ws = Workspace(nbytes)
        _ws_cache[k] = ws
    return ws


def release_workspaces():
    """Drop the cached default workspaces (their memory returns to torch's
    caching allocator once the work enqueued on their streams is done)."""
    _ws_cache.clear()


def default_chunk(circuit: Circuit, op: int, dtype: int, ncols: int,
                  budget_bytes: int = 24 << 30) -> int:
    """Largest power-of-two chunk (>= 64, <= padded column count) whose
    workspace fits the budget."""
    L = lib()
    top = max(64, 1 << int(np.ceil(np.log2(max(ncols, 64)))))
    chunk = top
    while chunk > 64:
        if op == RQ_OP_HESS:
            need = L.rq_hess_workspace_bytes(C.byref(circuit._c), dtype, chunk)
        else:
            need = L.rq_workspace_bytes(C.byref(circuit._c), op, dtype, chunk)
        if need and need <= budget_bytes:
            break
        chunk //= 2
    return chunk


def _exec(circuit: Circuit, op: int, dtype: int, chunk, workspace, stream, flags=0):
    L = lib()
    if chunk is None:
        chunk = default_chunk(circuit, op, dtype, circuit.ncols)
    if op == RQ_OP_HESS:
        need = L.rq_hess_workspace_bytes(C.byref(circuit._c), dtype, chunk)
    else:
        need = L.rq_workspace_bytes(C.byref(circuit._c), op, dtype, chunk)
    if need == 0:
        raise RQError(RQ_EINVAL, "rq_workspace_bytes")
    s = stream if stream is not None else torch.cuda.current_stream()
    ws = workspace if workspace is not None else _workspace(need, s)
    if ws.nbytes < need:
        raise RuntimeError(f"workspace too small: {ws.nbytes} < {need}")
    return _Exec(ws.ptr, ws.nbytes, chunk, s.cuda_stream, flags, 0), ws


def _range(rng):
    if rng is None:
        return None
    sector, begin, count = rng
    return C.byref(_Range(sector, 0, begin, count))


def _out(shape, want=True):
    if not want:
        return None
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def _ptr(t):
    return None if t is None else t.data_ptr()


def _cplx(t):
    return None if t is None else torch.view_as_complex(t)


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def _outputs(out, n, P):
    """Caller-provided float64 device outputs (f [1], then [P,4,4,2] arrays)
    or fresh zero tensors."""
    if out is not None:
        assert len(out) == n
        return list(out)
    return [_out((1,))] + [_out((P, 4, 4, 2)) for _ in range(n - 1)]


def rq_cost(circuit: Circuit, target: Target, gates, range=None, chunk=None, workspace=None,
            stream=None, out=None, accumulate=False) -> torch.Tensor:
    """f over the basis range (device float64 scalar).  With ``out`` (a
    1-element float64 device tensor) and ``accumulate``, f is added to it."""
    g = _gates_host(gates)
    ex, ws = _exec(circuit, RQ_OP_COST, target.dtype, chunk, workspace, stream,
                   RQ_EXEC_ACCUMULATE if accumulate else 0)
    (f,) = _outputs(None if out is None else (out,), 1, circuit.n_params)
    t = target.struct()
    _check(lib().rq_cost(C.byref(circuit._c), C.byref(t), _dptr(g), _range(range), C.byref(ex),
                         _ptr(f)), "rq_cost")
    return f[0]


def rq_grad(circuit: Circuit, target: Target, gates, range=None, chunk=None, workspace=None,
            stream=None, out=None, accumulate=False):
    """Returns (f, egrad [P,4,4] complex, rgrad [P,4,4] complex) on the device.
    ``out``: (f [1], egrad [P,4,4,2], rgrad [P,4,4,2]) float64 device tensors
    to write (or, with ``accumulate``, to add) the results into."""
    g = _gates_host(gates)
    ex, ws = _exec(circuit, RQ_OP_GRAD, target.dtype, chunk, workspace, stream,
                   RQ_EXEC_ACCUMULATE if accumulate else 0)
    f, eg, rg = _outputs(out, 3, circuit.n_params)
    t = target.struct()
    _check(lib().rq_grad(C.byref(circuit._c), C.byref(t), _dptr(g), _range(range), C.byref(ex),
                         _ptr(f), _ptr(eg), _ptr(rg)), "rq_grad")
    return f[0], _cplx(eg), _cplx(rg)


def rq_hvp(circuit: Circuit, target: Target, gates, direction, range=None, chunk=None,
           workspace=None, stream=None, out=None, accumulate=False):
    """Returns (f, egrad, rgrad, ehvp, rhvp) on the device (see rq_grad for
    ``out`` / ``accumulate``; here five tensors)."""
    g = _gates_host(gates)
    d = _gates_host(direction)
    ex, ws = _exec(circuit, RQ_OP_HVP, target.dtype, chunk, workspace, stream,
                   RQ_EXEC_ACCUMULATE if accumulate else 0)
    f, eg, rg, eh, rh = _outputs(out, 5, circuit.n_params)
    t = target.struct()
    _check(lib().rq_hvp(C.byref(circuit._c), C.byref(t), _dptr(g), _dptr(d), _range(range),
                        C.byref(ex), _ptr(f), _ptr(eg), _ptr(rg), _ptr(eh), _ptr(rh)), "rq_hvp")
    return f[0], _cplx(eg), _cplx(rg), _cplx(eh), _cplx(rh)


def rq_hvp_static(circuit: Circuit, target: Target, gates, direction, range=None, stream=None,
                  out=None, accumulate=False):
    """rq_hvp with the library's static scratch as workspace (no device
    allocation inside the call).  Returns (f, egrad, rgrad, ehvp, rhvp,
    chunk used).  Pass preallocated ``out`` tensors to allocate nothing."""
    g = _gates_host(gates)
    d = _gates_host(direction)
    s = stream if stream is not None else torch.cuda.current_stream()
    f, eg, rg, eh, rh = _outputs(out, 5, circuit.n_params)
    t = target.struct()
    used = C.c_int64(0)
    _check(lib().rq_hvp_static(C.byref(circuit._c), C.byref(t), _dptr(g), _dptr(d), _range(range),
                               s.cuda_stream, RQ_EXEC_ACCUMULATE if accumulate else 0,
                               C.byref(used), _ptr(f), _ptr(eg), _ptr(rg), _ptr(eh), _ptr(rh)),
           "rq_hvp_static")
    return f[0], _cplx(eg), _cplx(rg), _cplx(eh), _cplx(rh), used.value


def rq_hess_blocks(circuit: Circuit, target: Target, gates, range=None, chunk=None,
                   workspace=None, stream=None, holomorphic=True, out=None, accumulate=False):
    """Returns (f, egrad, rgrad, hess_holo [P,d,P,d] complex or None,
    hess_real [P*d, P*d]) on the device.  ``out``: float64 device tensors
    (f [1], egrad [P,4,4,2], rgrad [P,4,4,2], hess_holo [P,d,P,d,2] or None,
    hess_real [P*d,P*d]) to write, or with ``accumulate`` to add, into."""
    g = _gates_host(gates)
    ex, ws = _exec(circuit, RQ_OP_HESS, target.dtype, chunk, workspace, stream,
                   RQ_EXEC_ACCUMULATE if accumulate else 0)
    P = circuit.n_params
    d = 6 if circuit.number else 8 if circuit.parity else 16
    if out is not None:
        f, eg, rg, hh, hr = out
    else:
        f, eg, rg = _out((1,)), _out((P, 4, 4, 2)), _out((P, 4, 4, 2))
        hh = _out((P, d, P, d, 2), holomorphic)
        hr = _out((P * d, P * d))
    t = target.struct()
    _check(lib().rq_hess_blocks(C.byref(circuit._c), C.byref(t), _dptr(g), _range(range),
                                C.byref(ex), _ptr(f), _ptr(eg), _ptr(rg), _ptr(hh), _ptr(hr)),
           "rq_hess_blocks")
    return f[0], _cplx(eg), _cplx(rg), _cplx(hh), hr


def rq_apply_circuit(circuit: Circuit, gates, states: torch.Tensor, dtype: Optional[int] = None,
                     sector: int = -1, workspace=None, stream=None) -> torch.Tensor:
    """Apply the circuit in place to ``states`` ([rows, n] complex on cuda,
    column c = one state).  Returns ``states``."""
    if dtype is None:
        dtype = RQ_C128 if states.dtype == torch.complex128 else RQ_C64
    if states.dtype != torch_dtype(dtype) or states.dim() != 2 or states.stride(1) != 1:
        raise ValueError("states must be a row-major [rows, n] tensor of the given dtype")
    g = _gates_host(gates)
    L = lib()
    need = L.rq_workspace_bytes(C.byref(circuit._c), RQ_OP_APPLY, dtype, 0)
    if need == 0:
        raise RQError(RQ_EINVAL, "rq_workspace_bytes")
    s = stream if stream is not None else torch.cuda.current_stream()
    ws = workspace if workspace is not None else _workspace(need, s, key=("apply",))
    ex = _Exec(ws.ptr, ws.nbytes, 0, s.cuda_stream)
    _check(L.rq_apply_circuit(C.byref(circuit._c), _dptr(g), states.data_ptr(), states.shape[1],
                              states.stride(0), dtype, sector, C.byref(ex)), "rq_apply_circuit")
    return states


def _structure_flags(parity):
    """Circuit flags and tangent dimension for parity False / True / "number"."""
    if parity == "number":
        return RQ_PARITY | RQ_NUMBER, 6
    return (RQ_PARITY, 8) if parity else (0, 16)


def rq_tangent_basis(parity=False) -> np.ndarray:
    flags, d = _structure_flags(parity)
    out = np.zeros((d, 4, 4), dtype=np.complex128)
    n = lib().rq_tangent_basis(flags, _dptr(out))
    assert n == d
    return out


def rq_tr_step(gates, g: np.ndarray, H: np.ndarray, delta: float, parity=False):
    """Host FP64 truncated-CG step and polar retraction; returns
    (eta, candidate gates [P,4,4], model_decrease, stop_code)."""
    G = _gates_host(gates)
    P = G.shape[0]
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
    eta = np.zeros_like(g)
    cand = np.zeros_like(G)
    md = C.c_double(0)
    stop = C.c_int32(0)
    _check(lib().rq_tr_step(P, _structure_flags(parity)[0], _dptr(G), _dptr(g), _dptr(H),
                            float(delta), _dptr(eta), _dptr(cand), C.byref(md), C.byref(stop)),
           "rq_tr_step")
    return eta, cand, md.value, stop.value


def rq_tr_accept(f0, f1, model_decrease, delta, delta_bar, eta_norm):
    nd = C.c_double(0)
    acc = C.c_int32(0)
    rho = C.c_double(0)
    _check(lib().rq_tr_accept(f0, f1, model_decrease, delta, delta_bar, eta_norm, C.byref(nd),
                              C.byref(acc), C.byref(rho)), "rq_tr_accept")
    return nd.value, bool(acc.value), rho.value


def rq_stream_copy(dst: torch.Tensor, src: torch.Tensor, unroll: int = 4, blocks: int = 0,
                   stream=None):
    """Diagnostic streaming copy of src into dst (same byte size, a multiple
    of 16) by librq's hand-written copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous with the same byte size")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().rq_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, int(unroll), int(blocks),
                                s.cuda_stream), "rq_stream_copy")
    return dst


def rq_tangent_coords(gates, Y, parity=False) -> np.ndarray:
    """Coordinates Re Tr[(G_p A_mu)^dagger Y_p] in the tangent basis (host)."""
    G = _gates_host(gates)
    Yh = _gates_host(Y)
    flags, d = _structure_flags(parity)
    out = np.zeros(G.shape[0] * d)
    _check(lib().rq_tangent_coords(G.shape[0], flags, _dptr(G), _dptr(Yh),
                                   _dptr(out)), "rq_tangent_coords")
    return out


def rq_tr_solve(circuit: Circuit, target: Target, gates, max_iter: int = 20, gtol: float = 0.0,
                range=None, chunk=None, workspace=None, stream=None):
    """Riemannian trust-region optimisation on the device (rq_tr_solve).
    Returns (gates [P,4,4] complex128 host, history [n_iter, 6]: f, |grad|,
    delta, rho, accepted, tCG stop code)."""
    G = _gates_host(gates).copy()
    L = lib()
    if chunk is None:
        chunk = default_chunk(circuit, RQ_OP_HESS, target.dtype, circuit.ncols)
    need = L.rq_tr_workspace_bytes(C.byref(circuit._c), target.dtype, chunk)
    if need == 0:
        raise RQError(RQ_EINVAL, "rq_tr_workspace_bytes")
    s = stream if stream is not None else torch.cuda.current_stream()
    ws = workspace if workspace is not None else _workspace(need, s, key=("tr",))
    ex = _Exec(ws.ptr, ws.nbytes, chunk, s.cuda_stream)
    hist = np.zeros((max(1, max_iter), 6))
    n = C.c_int32(0)
    t = target.struct()
    _check(L.rq_tr_solve(C.byref(circuit._c), C.byref(t), _dptr(G), _range(range), C.byref(ex),
                         int(max_iter), float(gtol), _dptr(hist), C.byref(n)), "rq_tr_solve")
    return G, hist[:n.value]


def apply_workspace(k: int, gate_list, dtype: int, parity: bool = False,
                    sectors: bool = False) -> Workspace:
    """Workspace for rq_apply_circuit with a gate list (its gate
    coefficients), for callers that run several applications concurrently on
    different streams and must not share one."""
    circ = Circuit(k, [p for p, _ in gate_list], parity=parity, number=sectors, sectors=sectors)
    need = lib().rq_workspace_bytes(C.byref(circ._c), RQ_OP_APPLY, dtype, 0)
    if need == 0:
        raise RQError(RQ_EINVAL, "rq_workspace_bytes")
    return Workspace(need)


def build_trotter_target(k: int, gate_list, dtype: int = RQ_C128, parity: bool = True,
                         device="cuda", workspace=None, stream=None,
                         sectors: bool = False) -> Target:
    """Target columns U|j> for every basis state, built on the device by
    applying a gate list (e.g. a Trotter circuit) to the identity columns with
    rq_apply_circuit.  Parity mode returns the two sector blocks.  The work is
    enqueued on ``stream`` (default: the current stream) with ``workspace``
    (default: the stream's cached apply workspace)."""
    pairs = [p for p, _ in gate_list]
    gates = np.stack([G for _, G in gate_list])
    circ = Circuit(k, pairs, parity=parity, number=sectors, sectors=sectors)
    td = torch_dtype(dtype)
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        if sectors:
            # particle-number sectors (the gate list must conserve particle
            # number): the identity block of every sector, then the circuit
            ref = torch.zeros((1 << k, math.comb(k, k // 2)), dtype=td, device=device)
            for n, (first, size) in enumerate(sector_bounds(k)):
                blk = ref[first:first + size, :size]
                blk.fill_diagonal_(1.0)
                rq_apply_circuit(circ, gates, blk, dtype=dtype, sector=n, workspace=workspace,
                                 stream=s)
            return Target(ref, dtype, False)
        if parity:
            n = 1 << (k - 1)
            ref = torch.zeros((2, n, n), dtype=td, device=device)
            for p in (0, 1):
                ref[p].fill_diagonal_(1.0)
                rq_apply_circuit(circ, gates, ref[p], dtype=dtype, sector=p, workspace=workspace,
                                 stream=s)
        else:
            n = 1 << k
            ref = torch.eye(n, dtype=td, device=device)
            rq_apply_circuit(circ, gates, ref, dtype=dtype, sector=-1, workspace=workspace,
                             stream=s)
    return Target(ref, dtype, parity)


def sampled_target(k: int, n_samples: int, rng: np.random.Generator, *, dtype: int = RQ_C128,
                   parity: bool = False, gate_list=None, U: Optional[np.ndarray] = None,
                   kind: str = "rademacher", device="cuda") -> Target:
    """Input states and target columns for estimating the trace over random
    vectors instead of the 2^k basis states (the follow-up outlined in Sec.
    "Conclusions").  Column r holds z_r with independent entries, either
    complex Rademacher (uniform on {1, i, -1, -i}) or standard complex
    Gaussian, so that E[z z^dagger] = I and E[z^dagger A z] = Tr A; in parity
    mode each sector block gets its own n_samples vectors of the sector
    dimension.  The random numbers are drawn on the host from ``rng`` and
    passed in; the target columns U z_r are built on the device by applying
    ``gate_list`` with rq_apply_circuit, or (small k) from a dense host ``U``.
    Scale the library's sums by 1 / n_samples for the estimate."""
    dim = 1 << (k - 1) if parity else 1 << k
    shape = (2, dim, n_samples) if parity else (dim, n_samples)
    if kind == "rademacher":
        Z = (1j ** rng.integers(0, 4, size=shape)).astype(np.complex128)
    elif kind == "gaussian":
        Z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    else:
        raise ValueError("kind must be 'rademacher' or 'gaussian'")
    td = torch_dtype(dtype)
    inputs = torch.from_numpy(np.ascontiguousarray(Z)).to(td).to(device)
    if gate_list is not None:
        pairs = [p for p, _ in gate_list]
        gates = np.stack([G for _, G in gate_list])
        circ = Circuit(k, pairs, parity=parity)
        ref = inputs.clone()
        if parity:
            for p in (0, 1):
                rq_apply_circuit(circ, gates, ref[p], dtype=dtype, sector=p)
        else:
            rq_apply_circuit(circ, gates, ref, dtype=dtype, sector=-1)
    elif U is not None:
        U = np.asarray(U)
        if parity:
            Y = np.stack([U[np.ix_(sector_rows(k, p), sector_rows(k, p))] @ Z[p] for p in (0, 1)])
        else:
            Y = U @ Z
        ref = torch.from_numpy(np.ascontiguousarray(Y)).to(td).to(device)
    else:
        raise ValueError("give the target as gate_list or U")
    return Target(ref, dtype, parity, inputs=inputs)


def translation_orbits(k: int, shift: int, parity: bool = False):
    """Orbit representatives of the basis states under the cyclic qubit
    translation q -> q + shift, with their orbit sizes (rq_orbit_reps).
    Returns a list of (compressed columns, weights) per sector (one entry
    without parity)."""
    L = lib()
    out = []
    for sector in ((0, 1) if parity else (-1,)):
        n = C.c_int64(0)
        _check(L.rq_orbit_reps(k, shift, sector, C.byref(n), None, None), "rq_orbit_reps")
        reps = np.zeros(n.value, dtype=np.int64)
        wts = np.zeros(n.value)
        _check(L.rq_orbit_reps(k, shift, sector, C.byref(n),
                               reps.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(wts)),
               "rq_orbit_reps")
        out.append((reps, wts.astype(np.int64)))
    return out


def orbit_target(circuit: Circuit, target: Target, stream=None) -> Target:
    """Input states and target columns that reduce the trace sum to one basis
    state per translation orbit, weighted by the orbit size (rq_orbit_target):
    summand r starts from sqrt(w_r)|r> and its target column is
    sqrt(w_r) U|r>, so every output (bilinear in the two) is
    sum_r w_r (summand of r), which equals the sum over all basis states when
    the circuit and the target are invariant under circuit.shift.  Use with
    range (-1, 0, R) (R = width of the returned slabs; parity sectors are
    padded with zero columns to a common width)."""
    if not circuit.shift:
        raise ValueError("the circuit declares no translation symmetry")
    if target.col_offset != 0 or target.inputs is not None:
        raise ValueError("orbit reduction needs the full target columns")
    L = lib()
    counts = []
    for sector in ((0, 1) if circuit.parity else (-1,)):
        n = C.c_int64(0)
        _check(L.rq_orbit_reps(circuit.k, circuit.shift, sector, C.byref(n), None, None),
               "rq_orbit_reps")
        counts.append(n.value)
    R = max(counts)
    rows = target.ref.shape[-2]
    shape = (2, rows, R) if circuit.parity else (rows, R)
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        inputs = torch.empty(shape, dtype=target.ref.dtype, device=target.ref.device)
        ref = torch.empty(shape, dtype=target.ref.dtype, device=target.ref.device)
        need = L.rq_orbit_workspace_bytes(C.byref(circuit._c), R)
        if need == 0:
            raise RQError(RQ_EINVAL, "rq_orbit_workspace_bytes")
        ws = Workspace(need)
    ex = _Exec(ws.ptr, ws.nbytes, 0, s.cuda_stream, 0, 0)
    t = target.struct()
    _check(L.rq_orbit_target(C.byref(circuit._c), C.byref(t), inputs.data_ptr(), ref.data_ptr(),
                             R, C.byref(ex)), "rq_orbit_target")
    return Target(ref, target.dtype, circuit.parity, inputs=inputs)


STAGES = ("fwd", "last", "bwd")
OPS = ("cost", "grad", "hvp", "apply")


def rq_profile_enable(on: bool = True):
    _check(lib().rq_profile_enable(1 if on else 0), "rq_profile_enable")


def rq_profile_read():
    """Per (op, stage) kernel time (ms), launches, algorithmic bytes, flops
    since the last read (HIP events on the launch streams)."""
    ms = np.zeros(16)
    n = np.zeros(16, dtype=np.int64)
    by = np.zeros(16)
    fl = np.zeros(16)
    _check(lib().rq_profile_read(_dptr(ms), n.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(by),
                                 _dptr(fl)), "rq_profile_read")
    out = {}
    hess = {12: ("hess", "sweep"), 13: ("hess", "states"), 14: ("hess", "hole"),
            15: ("copy", "stream")}
    for i in range(16):
        if n[i]:
            key = (OPS[i // 3], STAGES[i % 3]) if i < 12 else hess[i]
            out[key] = dict(ms=float(ms[i]), launches=int(n[i]), bytes=float(by[i]),
                            flops=float(fl[i]))
    return out


def build_target_window(k: int, gate_list, j0: int, n: int, dtype: int = RQ_C128,
                        device="cuda") -> Target:
    """Columns U|j>, j0 <= j < j0 + n, of the target given by a gate list
    (general mode), built on the device with rq_apply_circuit.  Use with a
    basis range inside the window."""
    pairs = [p for p, _ in gate_list]
    gates = np.stack([G for _, G in gate_list])
    circ = Circuit(k, pairs)
    ref = torch.zeros((1 << k, n), dtype=torch_dtype(dtype), device=device)
    idx = torch.arange(n, device=device)
    ref[j0 + idx, idx] = 1.0
    rq_apply_circuit(circ, gates, ref, dtype=dtype, sector=-1)
    return Target(ref, dtype, False, col_offset=j0)
