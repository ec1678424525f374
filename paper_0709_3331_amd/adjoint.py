"""Differentiable tree forces and Verlet rollouts.

`TreeForce` is the force map F(x) of the TREE method (Sec. 3) as a
torch.autograd.Function.  Its backward is the library's adjoint walk
(ucp_force_vjp): the vector-Jacobian product (dF/dx)^T u with the topology,
the interaction lists and the cube's side of the build at x held fixed (they
are piecewise constant in x).  The box centres are not: they are the cube
origin, the per-axis minimum of the positions, plus fixed offsets, and the
adjoint carries their derivative to the minimum particles.  The backward
rebuilds the tree at the saved positions first, because later builds (the
next Verlet steps) replace the context's tree, and checks the library's
device flags (a raised flag raises UcpError).

`rollout` integrates velocity Verlet (kick-drift-kick, Sec. 2) with TreeForce
and recomputes each segment of `checkpoint_every` steps during the backward
pass instead of storing it (torch.utils.checkpoint).  Gradients reach the
initial positions and velocities, and through them any parameter they were
made from (e.g. the cloud width sigma with x0 = sigma z).

The solver object needs `tree_forces(x, q)`, `build(x, q)`, `vjp(u)` and
`check()` (raises if the device flagged a problem since the last check), as
`tree.TreeSolver` provides.  The forward of a rollout checks once at its end:
the library keeps every flag raised since the last check.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint


class TreeForce(torch.autograd.Function):
    """F = TreeForce.apply(x, q, solver); gradient flows to x only."""

    @staticmethod
    def forward(ctx, x, q, solver):
        xd = x.detach().contiguous()
        f = solver.tree_forces(xd, q)
        ctx.solver = solver
        ctx.save_for_backward(xd, q)
        return f

    @staticmethod
    def backward(ctx, fbar):
        x, q = ctx.saved_tensors
        solver = ctx.solver
        solver.build(x, q)   # the lists of this x
        xbar = solver.vjp(fbar.contiguous())
        solver.check()
        return xbar, None, None


def kdk_segment(solver, x, v, f, q, inv_m, dt, nsteps):
    """nsteps of kick-drift-kick from (x, v) with F(x) = f given."""
    for _ in range(nsteps):
        v = v + (0.5 * dt) * f * inv_m
        x = x + dt * v
        f = TreeForce.apply(x, q, solver)
        v = v + (0.5 * dt) * f * inv_m
    return x, v, f


def rollout(solver, x0, v0, q, m, dt, nsteps, checkpoint_every=20):
    """Differentiable KDK rollout; returns (x, v) after nsteps.

    x0, v0: (N, 3) float64 on the GPU (may require grad); q, m: (N,).
    checkpoint_every <= 0 keeps the whole graph (no recomputation)."""
    inv_m = (1.0 / m)[:, None]
    f = TreeForce.apply(x0, q, solver)
    x, v = x0, v0
    done = 0
    while done < nsteps:
        k = nsteps - done if checkpoint_every <= 0 else min(checkpoint_every, nsteps - done)
        if checkpoint_every > 0 and torch.is_grad_enabled():
            x, v, f = checkpoint(kdk_segment, solver, x, v, f, q, inv_m, dt, k,
                                 use_reentrant=False)
        else:
            x, v, f = kdk_segment(solver, x, v, f, q, inv_m, dt, k)
        done += k
    solver.check()
    return x, v


def ion_kinetic_energy(v, q, m):
    """Sum over ions (q > 0) of m |v|^2 / 2."""
    ion = (q > 0).to(v.dtype)
    return 0.5 * (ion * m * (v * v).sum(dim=1)).sum()
