"""torch.autograd wrapper of the shooting: J_1 = I_0 o phi_1^{-1}(v0).

Forward shoots with trajectory store (a linearization of the context).
Backward is the hand-written adjoint Jacobi sweep of the library
(``lddmm_vjp``): with U^(1) = -gbar grad J_1 it returns L w_0, the gradient of
the loss with respect to the plain array v0 (optimise-then-discretise: the
Jacobi-field linearization of the state equation, Section 3 of the paper).

The context keeps one linearization; if another forward (or any other
linearizing call) ran in between, backward re-linearizes at the saved v0.
The trajectory memory policy of the context (store-all, checkpointing,
recompute) applies unchanged.
"""

from __future__ import annotations

import torch


class ShootImage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v0, reg):
        v0c = v0.detach().contiguous()
        J1 = reg.empty_scalar()
        reg.linearize(v0c, J1_out=J1)
        ctx.reg = reg
        ctx.epoch = reg.get_option("lin.epoch")
        ctx.save_for_backward(v0c)
        return J1

    @staticmethod
    def backward(ctx, gbar):
        reg = ctx.reg
        if reg.get_option("lin.epoch") != ctx.epoch:
            (v0c,) = ctx.saved_tensors
            reg.linearize(v0c)
        return reg.vjp(gbar.contiguous()), None


def shoot_image(reg, v0):
    """Differentiable J_1(v0) for a ``Registration`` context ``reg``."""
    return ShootImage.apply(v0, reg)
