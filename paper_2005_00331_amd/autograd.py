"""torch.autograd.Function around the residual of eq. (residual).

Forward: R(u, phi; Gc, eps) with phi~ a non-differentiable input (it
replaces phi in the degradation of the displacement equation, Section
3.2).  Backward, written by hand: the transposed Jacobian of eq. (G)
applied to the cotangent (unconstrained, since the residual itself has no
constraints) and the two parameter cotangents <v, dR/dGc>, <v, dR/deps>.
The context must be created without Dirichlet rows (dirichlet = 0): the
forward raises otherwise, since the product of such a context has identity
rows and columns at the Dirichlet dofs and would give a wrong u gradient.
The backward sets the context's point with an empty active set, so that its
operator is the plain Jacobian; this drops the context's linearisation, and
a V-cycle or GMRES solve on it afterwards needs set_linearization again (the
library reports MFPFF_ERR_STATE until then).
"""
import torch

from .binding import OP_GT, F64


class ResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, phi, Gc, eps, phi_tilde, solver):
        """u: (dim*n_nodes,), phi, phi_tilde: (n_nodes,), Gc/eps: 0-d tensors that
        must equal the values the solver was created with."""
        p = solver.problem
        if p.dirichlet:
            raise ValueError("the residual's backward needs a context created with dirichlet = 0 "
                             "(a Dirichlet context's transposed product has identity rows at the fixed dofs)")
        if abs(float(Gc) - p.Gc) > 0 or abs(float(eps) - p.eps) > 0:
            raise ValueError("Gc and eps must match the solver's problem description")
        R = solver.residual(u.detach(), phi.detach(), phi_tilde.detach())
        ctx.save_for_backward(u.detach(), phi.detach(), phi_tilde.detach())
        ctx.solver = solver
        return R

    @staticmethod
    def backward(ctx, v):
        u, phi, phit = ctx.saved_tensors
        s = ctx.solver
        v = v.contiguous()
        zeros = torch.zeros(s.n_nodes, dtype=torch.uint8, device=u.device)
        s.set_point(u, phi, phi, zeros, phit)
        gT = s.apply_jacobian(-1, v, prec=F64, op=OP_GT)
        dGc, deps = s.residual_param_vjp(u, phi, phit, v)
        nu = s.dim * s.n_nodes
        gu = gT[:nu] if ctx.needs_input_grad[0] else None
        gp = gT[nu:] if ctx.needs_input_grad[1] else None
        tGc = torch.tensor(dGc, dtype=torch.float64) if ctx.needs_input_grad[2] else None
        teps = torch.tensor(deps, dtype=torch.float64) if ctx.needs_input_grad[3] else None
        return gu, gp, tGc, teps, None, None


def residual(u, phi, Gc, eps, phi_tilde, solver):
    return ResidualFn.apply(u, phi, Gc, eps, phi_tilde, solver)
