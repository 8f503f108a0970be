"""torch.autograd.Function around the gradient and HVP kernels, checked
against central finite differences (FP64 path, step 1e-4)."""

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2506_23775_amd import autograd as ag
    from paper_2506_23775_amd import rq
    assert torch.cuda.is_available()
    return torch, rq, ag


def test_torch_complex_gradient_convention(mods):
    # PyTorch accumulates d_x L + i d_y L for a real loss L(z): the paper's
    # gradient convention.  Pin it on |z|^2, whose gradient is 2z.
    torch, _, _ = mods
    z = torch.tensor([1.0 + 2.0j, -0.5 + 0.25j], dtype=torch.complex128, requires_grad=True)
    (z.abs() ** 2).sum().backward()
    assert torch.allclose(z.grad, 2 * z.detach())


def _fd_checks(torch, rq, ag, circ, tgt, gates_np, rng, rng_range=None, n_dirs=10, h=1e-4):
    gates = torch.tensor(gates_np, dtype=torch.complex128, requires_grad=True)
    f = ag.circuit_cost(gates, circ, tgt, range=rng_range)
    (g,) = torch.autograd.grad(f, gates, create_graph=True)
    gnp = g.detach().numpy()
    for _ in range(n_dirs):
        X = rng.standard_normal(gates_np.shape) + 1j * rng.standard_normal(gates_np.shape)
        X /= np.linalg.norm(X)
        fp = float(rq.rq_cost(circ, tgt, gates_np + h * X, range=rng_range))
        fm = float(rq.rq_cost(circ, tgt, gates_np - h * X, range=rng_range))
        fd = (fp - fm) / (2 * h)
        an = np.real(np.sum(np.conj(gnp) * X))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # Hessian-vector product through double backward vs FD of the gradient
    V = rng.standard_normal(gates_np.shape) + 1j * rng.standard_normal(gates_np.shape)
    V /= np.linalg.norm(V)
    (hv,) = torch.autograd.grad(g, gates, torch.tensor(V))
    _, egp, _ = rq.rq_grad(circ, tgt, gates_np + h * V, range=rng_range)
    _, egm, _ = rq.rq_grad(circ, tgt, gates_np - h * V, range=rng_range)
    fdv = (egp.cpu().numpy() - egm.cpu().numpy()) / (2 * h)
    err = np.linalg.norm(hv.detach().numpy() - fdv) / np.linalg.norm(fdv)
    assert err < 1e-6, err


def test_autograd_fd_small(mods):
    torch, rq, ag = mods
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, rq.RQ_C128)
    _fd_checks(torch, rq, ag, circ, tgt, prob.gates, np.random.default_rng(31))


def test_autograd_fd_config4_basis_window(mods):
    """Configuration 4 shape (k=16, 9 layers, 72 gates, Strang-200 target) on
    a window of 256 basis states (the finite-difference check needs 24 cost
    and gradient evaluations)."""
    torch, rq, ag = mods
    prob = w.make_problem(4)
    j0, n = 4096, 256
    tgt = rq.build_target_window(prob.k, prob.trotter, j0, n, rq.RQ_C128)
    circ = rq.Circuit(prob.k, prob.pairs)
    _fd_checks(torch, rq, ag, circ, tgt, prob.gates, np.random.default_rng(32),
               rng_range=(-1, j0, n), n_dirs=10)
