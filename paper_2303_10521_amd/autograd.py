"""torch.autograd binding of the channel computation and its adjoint.

``channels(tracer, frame, eps, tx_pos, tx_orient, discover)`` runs one step of
the GPU library with the given permittivities and transmitter pose and
returns the complex channel sums H [n_freq, n_links] and the coherent powers
P_coh [n_freq, n_links] as differentiable tensors.  The backward pass calls
the library's adjoint (emrt_backward): gradients with respect to the complex
permittivities (PyTorch convention dL/dRe + j dL/dIm), the transmitter
positions and the dipole orientation, with the path topology of the step
held fixed.  The tracer must be created with ``adjoint_materials`` >= the
number of materials.  The library differentiates the tracer's last step, so a
forward's backward must run before the tracer steps again (it raises
otherwise).
"""
from __future__ import annotations

import torch


class _FrameOverride:
    def __init__(self, fr, tx_pos, tx_orient) -> None:
        for name in ("t", "obj_xform", "obj_vel", "tx_vel", "rx_pos", "rx_vel"):
            setattr(self, name, getattr(fr, name))
        self.tx_pos = tx_pos
        self.tx_orient = tx_orient


class ChannelFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, tx_pos, tx_orient, tracer, frame, discover):
        tracer.set_materials(eps.detach().cpu().numpy())
        fr = _FrameOverride(frame, tx_pos.detach().to(torch.float64), tx_orient.detach().to(torch.float64))
        tracer.set_frame(fr, getattr(frame, "index", 0))
        tracer.step(bool(discover))
        ch = tracer.channels()
        ctx.tracer = tracer
        ctx.generation = tracer.generation
        ctx.devices = (eps.device, tx_pos.device, tx_orient.device)
        return ch["H"], ch["P_coh"]

    @staticmethod
    def backward(ctx, gH, gP):
        if ctx.tracer.generation != ctx.generation:
            # the library differentiates its last step; a later step, frame or
            # material change would silently give another graph's gradients
            raise RuntimeError("the tracer stepped (or changed frame or materials) after this forward; its "
                               "adjoint would belong to the later state: run backward before the next step, "
                               "or use one tracer per recorded forward")
        g = ctx.tracer.backward(gH, gP)
        de, dp, do = ctx.devices
        return (g["grad_eps"].to(de), g["grad_tx_pos"].to(dp), g["grad_tx_orient"].to(do), None, None, None)


def channels(tracer, frame, eps: torch.Tensor, tx_pos: torch.Tensor, tx_orient: torch.Tensor, discover: bool = True):
    """Differentiable (H, P_coh) of one step; see the module docstring."""
    return ChannelFunction.apply(eps, tx_pos, tx_orient, tracer, frame, discover)
