"""torch.autograd wrappers of the FMM product, the BEM application and the
solve, with hand-written adjoints (marshalling only: every product runs in the
library's kernels).

For a C-linear map y = A x, torch's complex autograd passes back
grad_x = A^H grad_y, so:
* `fmm_matvec(plan, a, b)`: backward is `fmm_matvec_adjoint`;
* `bem_apply(problem, x)`: backward is `bem_apply_adjoint`;
* `bem_solve(problem, rhs, ...)`: x = A^{-1} rhs, backward solves the adjoint
  system A^H g = grad_x with the same fGMRES (right-preconditioned by M^{-H});
* `far_field(problem, x, dirs)`: F = L x at unit directions, backward is
  `bem_far_field_adjoint`.
"""

import torch


class _FmmMatvec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, plan):
        ctx.plan = plan
        return plan.matvec(a.contiguous(), b.contiguous())

    @staticmethod
    def backward(ctx, gy):
        ga, gb = ctx.plan.matvec_adjoint(gy.contiguous())
        return ga, gb, None


class _BemApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, problem):
        ctx.problem = problem
        return problem.apply(x.contiguous())

    @staticmethod
    def backward(ctx, gr):
        return ctx.problem.apply_adjoint(gr.contiguous()), None


class _BemSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhs, problem, kw):
        ctx.problem = problem
        ctx.kw = kw
        x, _ = problem.solve(rhs.contiguous(), **kw)
        return x

    @staticmethod
    def backward(ctx, gx):
        g, _ = ctx.problem.solve(gx.contiguous(), adjoint=True, **ctx.kw)
        return g, None, None


class _FarField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, problem, dirs):
        ctx.problem = problem
        ctx.dirs = dirs
        return problem.field(x.contiguous(), dirs, far=True)

    @staticmethod
    def backward(ctx, gF):
        return ctx.problem.far_field_adjoint(gF.contiguous(), ctx.dirs), None, None


def fmm_matvec(plan, a, b):
    """y = Op_k(a, b), differentiable in a and b."""
    return _FmmMatvec.apply(a, b, plan)


def bem_apply(problem, x):
    """A x, differentiable in x."""
    return _BemApply.apply(x, problem)


def bem_solve(problem, rhs, **solve_kw):
    """x = A^{-1} rhs by fGMRES, differentiable in rhs (the backward pass is an
    adjoint solve with the same options)."""
    return _BemSolve.apply(rhs, problem, dict(solve_kw))


def far_field(problem, x, dirs):
    """Far-field amplitudes F [nrhs, nd, 3] at unit directions dirs [nd, 3],
    differentiable in x."""
    return _FarField.apply(x, problem, dirs)
