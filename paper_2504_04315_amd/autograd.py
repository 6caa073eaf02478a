"""Differentiation form: the hot path behind torch.autograd.

`NPMFunction.apply(params, pos, dir, radiance, pdf, model, aux)` returns the
surrogate KL loss of the batch (Sec. 4.2: -(1/N) sum w log V, whose gradient
is eq. mcgradients) as a float64 device scalar.  Its backward runs the
library's hand-written backward kernels -- KL-gradient head, MLP backward,
weight gradients on MFMA, FP32 atomic scatter into the grid -- with the
grid encoding recomputed from the saved positions rather than stored.
`params` is a tensor aliasing the library's own FP32 parameter buffer, so
autograd accumulates its gradient into `params.grad`, and `NPMAdam.step()`
applies the library's fused Adam to that gradient (and zeroes it).  aux: the
NPM-product inputs [7][n] (omega_o, normal, roughness) of a network that
takes them (Sec. 4.3), else None.

Only argument marshalling happens here; every step runs in libnpm.
"""
import torch

from . import npm as B


class NPMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, pos, dir, radiance, pdf, model, aux=None):
        loss = torch.zeros(1, dtype=torch.float64, device=pos.device)
        model.loss(pos, dir, radiance, pdf, out=loss, aux=aux)
        ctx.model = model
        ctx.aux = aux
        ctx.save_for_backward(pos, dir, radiance, pdf)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        pos, dir, radiance, pdf = ctx.saved_tensors
        model = ctx.model
        g = torch.zeros(model.n_params, dtype=torch.float32, device=pos.device)
        model.backward(pos, dir, radiance, pdf, grad=g, aux=ctx.aux)
        if grad_out is not None:
            g.mul_(grad_out.to(torch.float32))
        return g, None, None, None, None, None, None


class NPM(torch.nn.Module):
    """A guiding network as a module: parameters live in libnpm."""

    def __init__(self, cfg):
        super().__init__()
        self.model = B.NPM(cfg)
        p = self.model.state_tensor(B.STATE_PARAMS)
        self.params = torch.nn.Parameter(p, requires_grad=True)

    def forward(self, pos, dir, radiance, pdf, aux=None):
        return NPMFunction.apply(self.params, pos, dir, radiance, pdf, self.model, aux)

    def query(self, pos, dir=None, **kw):
        return self.model.query(pos, dir, **kw)


class NPMAdam:
    """Adam (Sec. 5.3) on an NPM module through the library's fused kernel."""

    def __init__(self, module):
        self.module = module

    def zero_grad(self):
        if self.module.params.grad is not None:
            self.module.params.grad.zero_()

    @torch.no_grad()
    def step(self, gradnorm=None):
        g = self.module.params.grad
        if g is None:
            raise RuntimeError("no gradient: call backward() first")
        g = g.contiguous()
        self.module.model.optimizer_step(grad=g, gradnorm=gradnorm)
        self.module.params.grad = None
