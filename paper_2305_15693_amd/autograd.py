"""torch.autograd wrappers around the library's forward and backward passes.

The library computes on its context's HIP stream; these wrappers order that
stream after the caller's current stream before a call and the caller's stream
after the library's stream afterwards, so that they compose with ordinary torch
operations.  Every numeric step runs in the library's kernels:

  structure_factor(ctx, pos)  -> S on the mode cube.  Backward: the type-2
      field-derivative pass with dF/dS as coefficients (the derivative of S with
      respect to a position, Methods, "Analytical gradients"), so any spectral
      loss written in torch on S differentiates through the library.
  loss(ctx, pos)              -> L_S = sum_K W (S - S0)^2 (0-dim, float64).
      Backward: the gradient the forward already produced (Eq. gradient).
  soft_core(pctx, pos)        -> pair energy of the soft-core repulsion (0-dim,
      float64).  Backward: the pair forces the forward already produced.

Terms built from these share one backward, e.g.
  total = loss(ctx, pos) + soft_core(pctx, pos);  total.backward().
"""
from __future__ import annotations

import torch


class _StreamScope:
    """Order the library stream after the current stream on entry, and the current
    stream after the library stream on exit."""

    def __init__(self, lib_stream):
        self.lib = lib_stream

    def __enter__(self):
        self.cur = torch.cuda.current_stream(self.lib.device)
        if self.cur.cuda_stream != self.lib.cuda_stream:
            self.lib.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        if self.cur.cuda_stream != self.lib.cuda_stream:
            self.cur.wait_stream(self.lib)
        return False


def _keep(t, stream):
    # a tensor written on the library stream and freed on another must not be
    # reused before the library stream is done with it
    if t is not None and t.is_cuda and torch.cuda.current_stream(t.device).cuda_stream != stream.cuda_stream:
        t.record_stream(stream)
    return t


class StructureFactorFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fctx, pos):
        pos = pos.detach().contiguous()
        with _StreamScope(fctx.stream):
            S = _keep(fctx.structure_factor(_keep(pos, fctx.stream)), fctx.stream)
        ctx.fctx = fctx
        # the backward reuses rho and the point order when no other call ran on
        # fctx in between; torch's version check guards pos against in-place edits
        ctx.token = fctx.sf_token()
        ctx.save_for_backward(pos)
        return S

    @staticmethod
    def backward(ctx, gS):
        (pos,) = ctx.saved_tensors
        fctx = ctx.fctx
        gS = gS.contiguous().to(fctx.torch_dtype)
        with _StreamScope(fctx.stream):
            grad = _keep(fctx.structure_factor_backward(pos, _keep(gS, fctx.stream), token=ctx.token),
                         fctx.stream)
        return None, grad


class LossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fctx, pos):
        pos = pos.detach().contiguous()
        loss = torch.zeros((), dtype=torch.float64, device=pos.device)
        grad = torch.empty_like(pos)
        with _StreamScope(fctx.stream):
            fctx.loss_grad_async(_keep(pos, fctx.stream), _keep(loss, fctx.stream),
                                 _keep(grad, fctx.stream))
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (grad,) = ctx.saved_tensors
        return None, grad * gl.to(grad.dtype)


class SoftCoreFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pctx, pos):
        pos = pos.detach().contiguous()
        energy = torch.zeros((), dtype=torch.float64, device=pos.device)
        grad = torch.empty_like(pos)
        with _StreamScope(pctx.stream):
            pctx.energy_grad_async(_keep(pos, pctx.stream), _keep(energy, pctx.stream),
                                   _keep(grad, pctx.stream))
        ctx.save_for_backward(grad)
        return energy

    @staticmethod
    def backward(ctx, ge):
        (grad,) = ctx.saved_tensors
        return None, grad * ge.to(grad.dtype)


def structure_factor(fctx, pos):
    """S(n) on the mode cube of ``fctx`` (a ``fresco.Context``), differentiable in pos."""
    return StructureFactorFn.apply(fctx, pos)


def loss(fctx, pos):
    """L_S of ``fctx``'s problem at pos (float64 scalar), differentiable in pos."""
    return LossFn.apply(fctx, pos)


def soft_core(pctx, pos):
    """Soft-core pair energy of ``pctx`` (a ``fresco.PairContext``) at pos, differentiable."""
    return SoftCoreFn.apply(pctx, pos)
