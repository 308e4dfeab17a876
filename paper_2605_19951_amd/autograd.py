"""torch.autograd.Function for the forward map d(m), m = ln sigma on the
parameter cells (section "The Inverse Problem"), whose backward is the
adjoint J^T w through the cached pole factors (section "Jacobian
computation").  All arithmetic runs in libtem; torch supplies memory and
the autograd graph."""
from __future__ import annotations

import torch

from .tem import FP32_IR, Tem


class TEMProblem:
    """A factored survey: mesh, sources, receivers, poles/residues."""

    def __init__(self, tem: Tem, F, q_ptr, q_col, q_val, xi, alpha, precision=FP32_IR, ir=None):
        self.tem = tem
        self.F = F
        self.q = (q_ptr, q_col, q_val)
        self.xi = xi
        self.alpha = alpha
        self.precision = precision
        self.ir = ir
        self.version = 0        # bumped by every forward; backward must match

    def data_shape(self):
        return (self.F.shape[0], len(self.alpha), len(self.q[0]) - 1)


class TEMForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, problem: TEMProblem):
        t = problem.tem
        t.set_model(m.detach().contiguous())
        t.factor_poles(problem.xi, problem.precision)
        d = torch.empty(problem.data_shape(), dtype=torch.float64, device=m.device)
        t.forward(problem.F, *problem.q, problem.alpha, d, ir=problem.ir)
        problem.version += 1
        ctx.problem = problem
        ctx.version = problem.version
        return d

    @staticmethod
    def backward(ctx, grad_d):
        problem = ctx.problem
        if problem.version != ctx.version:
            raise RuntimeError("the factors were replaced by a later forward; backward needs the "
                               "factors of its own forward")
        g = torch.empty(problem.tem.n_params, dtype=torch.float64, device=grad_d.device)
        problem.tem.vjp(grad_d.contiguous(), g, ir=problem.ir)
        return g, None


def tem_forward(m, problem: TEMProblem):
    return TEMForward.apply(m, problem)
