"""torch.autograd.Function over the library's taped run and hand-written reverse kernels.

`micro_steps(...)` runs n micro-steps on the GPU from psi0 with the given rates and fluid
schedule and returns (sigma, moments) at the final time.  Its backward calls
mmk_tape_backward, which recomputes checkpoint segments and runs the reverse HIP kernels;
gradients flow to psi0, k_on, k_off and v0 (dt held fixed).  No torch operation takes part
in the step itself.
"""
from __future__ import annotations

import torch

from . import mmk


class MicroSteps(torch.autograd.Function):
    @staticmethod
    def forward(fctx, psi0, k_on, k_off, v0, p, fluids, K, n, dt, ckpt_every, precision, M0):
        lib_ctx = mmk.Context(p, precision=precision, ckpt_every=ckpt_every, max_tape_steps=n,
                              device=psi0.device)
        lib_ctx.set_params(float(k_on), float(k_off), float(v0))
        lib_ctx.set_state(psi0.detach(), None if M0 is None else M0.detach())
        done, e = 0, 0
        lib_ctx.set_fluid(*fluids[0])
        lib_ctx.tape_begin(ckpt_every)
        while done < n:
            if e > 0:
                lib_ctx.set_fluid(*fluids[min(e, len(fluids) - 1)])
            k = min(K, n - done)
            lib_ctx.step(k, dt)
            done += k
            e += 1
        sigma = lib_ctx.get_stress()
        moments = lib_ctx.get_moments()
        fctx.lib_ctx = lib_ctx
        fctx.param_dtype = k_on.dtype if torch.is_tensor(k_on) else torch.float64
        fctx.param_device = k_on.device if torch.is_tensor(k_on) else torch.device("cpu")
        return sigma, moments

    @staticmethod
    def backward(fctx, g_sigma, g_moments):
        lib_ctx = fctx.lib_ctx
        g_psi0, gp = lib_ctx.tape_backward(None if g_sigma is None else g_sigma.contiguous(),
                                           None if g_moments is None else g_moments.contiguous())
        lib_ctx.tape_end()
        mk = lambda v: torch.tensor(v, dtype=fctx.param_dtype, device=fctx.param_device)
        return (g_psi0, mk(gp[0]), mk(gp[1]), mk(gp[2]), None, None, None, None, None, None, None, None)


def micro_steps(p, psi0, k_on, k_off, v0, fluids, K, n, dt, ckpt_every, precision=mmk.FP64, M0=None):
    """(sigma, moments) after n micro-steps; differentiable in psi0, k_on, k_off, v0.

    fluids: list of (u [2][nx][ny], gradu [4][nx][ny]) device tensors, one per exchange of K
    steps.  k_on, k_off, v0: 0-dim tensors (or floats)."""
    t = lambda x: x if torch.is_tensor(x) else torch.tensor(float(x), dtype=torch.float64)
    return MicroSteps.apply(psi0, t(k_on), t(k_off), t(v0), p, fluids, K, n, dt, ckpt_every, precision, M0)
