"""Gradients of a window objective through the discrete adjoint of the step.

`AdjointWindow` binds the adjoint workspace of a running `Sim` (torch owns
the memory), runs a window of steps with the bond topology frozen and
checkpoints every `ckpt_every` steps, and returns the gradient of

    J = mean over particle vertices of the distance to the nearer wall

with respect to every body's strain constant k_s, bending constant k_b and
bond spring constant sigma.  `WindowObjective` wraps it as a
torch.autograd.Function of a (n_bodies, 3) parameter tensor: each forward
call restores the window's initial state, applies the parameters and runs
the window; backward runs the library's reverse sweep.

Every step and every derivative runs in the HIP library.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np


class AdjointWindow:
    def __init__(self, sim, nsteps: int, ckpt_every: int = 100):
        import torch
        self.sim = sim
        self.nsteps = int(nsteps)
        self.ckpt_every = int(ckpt_every)
        lib = sim.lib
        nb = ctypes.c_size_t()
        sim.check(lib.lbib_adjoint_workspace_query(sim.h, self.nsteps, self.ckpt_every,
                                                   ctypes.byref(nb)))
        dev = sim.ws.device
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        aligned = (self.ws.data_ptr() + 255) & ~255
        sim.check(lib.lbib_adjoint_bind(sim.h, ctypes.c_void_p(aligned), nb.value, self.nsteps,
                                        self.ckpt_every))
        self.workspace_bytes = nb.value
        self.n_bodies = len(sim.nv)

    def forward(self):
        """Run the window; returns (J, number of bonds held)."""
        J = ctypes.c_double()
        nb = ctypes.c_int32()
        self.sim.check(self.sim.lib.lbib_adjoint_forward(self.sim.h, ctypes.byref(J),
                                                         ctypes.byref(nb)))
        return J.value, nb.value

    def backward(self, dJ: float = 1.0) -> np.ndarray:
        """dJ * (dJ/dk_s, dJ/dk_b, dJ/dsigma) per body, shape (n_bodies, 3)."""
        g = np.zeros(3 * max(self.n_bodies, 1))
        self.sim.check(self.sim.lib.lbib_adjoint_backward(
            self.sim.h, float(dJ), g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return g[: 3 * self.n_bodies].reshape(self.n_bodies, 3)


class WindowObjective:
    """torch.autograd.Function over body parameters (n_bodies, 3) = (k_s, k_b, sigma).

    Usage: obj = WindowObjective(sim, nsteps, ckpt_every); J = obj(params);
    J.backward() fills params.grad.  The state at construction is the
    initial state of every evaluation.
    """

    def __init__(self, sim, nsteps: int, ckpt_every: int = 100, window: Optional[AdjointWindow] = None):
        import torch

        self.window = window if window is not None else AdjointWindow(sim, nsteps, ckpt_every)
        self.sim = sim
        self.state0 = sim.get_state()
        win = self.window
        state0 = self.state0

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, params):
                p = params.detach().to("cpu", torch.float64).numpy()
                sim.set_state(state0)
                for b in range(p.shape[0]):
                    sim.set_body_params(b, p[b, 0], p[b, 1], p[b, 2])
                J, _ = win.forward()
                ctx.save_for_backward(params)
                return torch.tensor(J, dtype=params.dtype)

            @staticmethod
            def backward(ctx, gJ):
                (params,) = ctx.saved_tensors
                g = win.backward(float(gJ))
                return torch.as_tensor(g, dtype=params.dtype, device=params.device)

        self._fn = _Fn

    def __call__(self, params):
        return self._fn.apply(params)
