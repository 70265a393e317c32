"""Gradients of a flame-front objective through the discrete adjoint of the step.

The objective is the smooth front position of a flame after n steps (the integral form
of the front position of Sec. 5.1):

    J = sum over nodes of (T - T_u) / (T_b - T_u),

a function of the Arrhenius parameters theta = (ln A_k, b_k, Ta_k) of every reaction and
of the initial temperature field T_0 (with the other initial fields held).  ``FlameFront``
is a torch.autograd.Function: its forward runs the n steps on the GPU, keeping a
snapshot every K steps; its backward walks the segments from the last, recomputes the
K - 1 states of each after its snapshot and applies the library's adjoint step to each in
reverse order.  K = 1 keeps every state resident (about 1.1 kB per node and step in FP32
storage with nine species: 9 GB for the 2048-cell flame's 4000 steps) and recomputes
nothing (lbm_adjoint_macros for the seed, lbm_adjoint_step per step,
lbm_adjoint_init for T_0).  By default K is the smallest spacing whose snapshots (and
the ring of recomputed states) fit in half of the device memory free at the call
(``snapshot_spacing``): on a GPU of 288 GB that keeps every state of such runs, and
recomputation only starts where memory runs short.  Only argument marshalling happens
here: every step and every adjoint step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np


def _torch():
    import torch
    return torch


def snapshot_spacing(n_steps: int, state_bytes: int, budget_bytes: float) -> int:
    """Smallest K >= 1 for which ceil(n / K) snapshots and a ring of K - 1 recomputed
    states, each of state_bytes, fit in budget_bytes (n_steps when none does)."""
    n = max(int(n_steps), 1)
    for k in range(1, n + 1):
        if (-(-n // k) + k - 1) * state_bytes <= budget_bytes:
            return k
    return n


class FlameFront:
    """Autograd function J(theta, T_0) over a Solver created with adjoint=True."""

    @staticmethod
    def apply(solver, theta, T0, n_steps: int, every=None, T_u: float = 300.0, T_b: float = 2000.0):
        torch = _torch()
        if every is None:
            free, _ = torch.cuda.mem_get_info(solver.device)
            every = snapshot_spacing(n_steps, solver.state_size(), 0.5 * free)
        every = int(every)
        if every < 1:
            raise ValueError("every must be >= 1")

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, th, t0):
                arr = th.detach().cpu().numpy().astype(np.float64).copy()
                arr[:, 0] = np.exp(arr[:, 0])
                solver.set_arrhenius(arr)
                solver.init(T=t0.detach())
                snaps = []
                done = 0
                while done < n_steps:
                    k = min(every, n_steps - done)
                    snaps.append((solver.state_save(), k))
                    solver.step_graph(k)
                    done += k
                final = solver.state_save()
                T = solver.macros(to_numpy=False)["T"]
                J = ((T - T_u) / (T_b - T_u)).sum()
                ctx.snaps, ctx.final = snaps, final
                ctx.t0 = t0.detach().clone()
                return J.to(th.device)

            @staticmethod
            def backward(ctx, gJ):
                R = solver.prob.mech.R
                w = torch.full((solver.N,), float(gJ) / (T_b - T_u), dtype=torch.float64, device=solver.device)
                lam = solver.adjoint_macros(state=ctx.final, w_T=w)
                grad = torch.zeros(max(R, 1), 3, dtype=torch.float64, device=solver.device)
                ring = [solver.new_state_buffer() for _ in range(max(every - 1, 0))]
                for snap, k in reversed(ctx.snaps):
                    # the segment's states: its snapshot, then k - 1 recomputed steps
                    states = [snap]
                    if k > 1:
                        solver.state_load(snap)
                        for j in range(k - 1):
                            solver.step(1)
                            states.append(solver.state_save(ring[j]))
                    for st in reversed(states):
                        solver.adjoint_step(lam, state=st, grad=grad)
                g0 = solver.adjoint_init(lam, T=ctx.t0)
                return grad[:R].to(theta.device), g0["T"].to(T0.device)

        return _Fn.apply(theta, T0)


def front_position(solver, T_u: float = 300.0, T_b: float = 2000.0) -> float:
    """J of the solver's current state."""
    T = solver.macros()["T"]
    return float(((T - T_u) / (T_b - T_u)).sum())


def theta_of(mech) -> np.ndarray:
    """(ln A, b, Ta) per reaction of a mechanism."""
    arr = np.asarray(mech.arrhenius, dtype=np.float64)
    return np.stack([np.log(arr[:, 0]), arr[:, 1], arr[:, 2]], axis=1)
