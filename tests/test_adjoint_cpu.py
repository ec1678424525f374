"""The differentiable rollout (paper_0709_3331_amd/adjoint.py) on the CPU.

The library's adjoint walk needs a GPU; here the same autograd and
checkpointing code runs against a stand-in solver made of the FP64 oracle's
direct sum and its analytic vector-Jacobian product (the negative Hessian of U
times u).  This checks the wrapper logic: recomputed segments give the same
gradient as a stored graph, and the gradient matches central finite
differences of the loss.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0709_3331_amd import adjoint, inputs


class DirectSolver:
    def __init__(self, eps):
        self.eps = eps
        self.x = None
        self.calls = 0

    def tree_forces(self, x, q):
        self.calls += 1
        f, _ = oracle.direct(x.numpy(), q.numpy(), self.eps)
        return torch.from_numpy(f)

    def build(self, x, q):
        self.x, self.q = x.numpy().copy(), q.numpy().copy()

    def vjp(self, u):
        return torch.from_numpy(oracle.direct_vjp(self.x, self.q, self.eps, u.numpy()))

    def check(self):
        pass


class FlaggingSolver(DirectSolver):
    """Reports a device flag (as the library's sticky word would) once a
    given number of force evaluations has happened."""

    def __init__(self, eps, flag_after):
        super().__init__(eps)
        self.flag_after = flag_after

    def check(self):
        if self.calls >= self.flag_after:
            raise RuntimeError("device flag raised")


def _setup(n=64, seed=3):
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, seed)
    z = torch.from_numpy(cl.x)             # sigma = 1: x0 = sigma z
    v0 = torch.from_numpy(cl.v)
    q = torch.from_numpy(cl.q)
    m = torch.from_numpy(cl.m)
    return z, v0, q, m


def _loss(solver, sigma, z, v0, q, m, dt, steps, every):
    xT, vT = adjoint.rollout(solver, sigma * z, v0, q, m, dt, steps, checkpoint_every=every)
    return adjoint.ion_kinetic_energy(vT, q, m)


def test_checkpointed_rollout_gradient_equals_stored_graph():
    z, v0, q, m = _setup()
    grads = []
    for every in (0, 3):
        solver = DirectSolver(0.05)
        sigma = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        v = v0.clone().requires_grad_(True)
        loss = _loss(solver, sigma, z, v, q, m, 1e-3, 7, every)
        loss.backward()
        grads.append((sigma.grad.item(), v.grad.clone()))
    assert grads[0][0] == pytest.approx(grads[1][0], rel=1e-13)
    torch.testing.assert_close(grads[0][1], grads[1][1], rtol=1e-12, atol=1e-14)


def test_rollout_gradient_matches_finite_differences():
    z, v0, q, m = _setup()
    dt, steps, eps = 1e-3, 6, 0.05
    sigma = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    v = v0.clone().requires_grad_(True)
    loss = _loss(DirectSolver(eps), sigma, z, v, q, m, dt, steps, 2)
    loss.backward()
    # the electrons' motion is stiff (mass 1/1836, eps = 0.05): the central
    # difference converges to the gradient only below h ~ 1e-6
    h = 1e-7
    with torch.no_grad():
        lp = _loss(DirectSolver(eps), torch.tensor(1.0 + h, dtype=torch.float64), z, v0, q, m, dt, steps, 2)
        lm = _loss(DirectSolver(eps), torch.tensor(1.0 - h, dtype=torch.float64), z, v0, q, m, dt, steps, 2)
    fd = (lp - lm).item() / (2 * h)
    assert sigma.grad.item() == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # directional derivative in v0
    d = torch.from_numpy(np.random.default_rng(0).normal(size=v0.shape))
    with torch.no_grad():
        lp = _loss(DirectSolver(eps), torch.tensor(1.0, dtype=torch.float64), z, v0 + h * d, q, m, dt, steps, 2)
        lm = _loss(DirectSolver(eps), torch.tensor(1.0, dtype=torch.float64), z, v0 - h * d, q, m, dt, steps, 2)
    fdv = (lp - lm).item() / (2 * h)
    assert (v.grad * d).sum().item() == pytest.approx(fdv, rel=1e-6, abs=1e-12)


def test_tree_force_backward_rebuilds_at_saved_positions():
    # the backward of an earlier force call must use that call's positions,
    # whatever the solver built since
    z, v0, q, m = _setup(32, 5)
    solver = DirectSolver(0.05)
    x1 = z.clone().requires_grad_(True)
    f1 = adjoint.TreeForce.apply(x1, q, solver)
    solver.build(z + 0.3, q)               # an unrelated later build
    u = torch.from_numpy(np.random.default_rng(1).normal(size=z.shape))
    (f1 * u).sum().backward()
    want = oracle.direct_vjp(z.numpy(), q.numpy(), 0.05, u.numpy())
    np.testing.assert_allclose(x1.grad.numpy(), want, rtol=1e-13, atol=1e-13)


def test_rollout_forward_and_backward_check_the_device_flags():
    # a flag raised by any step of the forward is seen once the forward ends
    z, v0, q, m = _setup()
    with pytest.raises(RuntimeError):
        _loss(FlaggingSolver(0.05, 3), torch.tensor(1.0, dtype=torch.float64), z, v0, q, m,
              1e-3, 5, 0)
    # and a flag raised while the backward recomputes a segment is seen there
    solver = FlaggingSolver(0.05, 10 ** 9)
    sigma = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    loss = _loss(solver, sigma, z, v0, q, m, 1e-3, 5, 2)
    solver.flag_after = 0
    with pytest.raises(RuntimeError):
        loss.backward()
