"""HMC pseudofermion force behind torch.autograd.

``OvForce.apply(lattice, phi, xi)`` returns S = sum_rhs Re xi^dag (M^dag M)^-1 xi
(M depends on phi through the Yukawa term).  Its backward returns
grad_out * G with G_x = dS/dRe phi_x + i dS/dIm phi_x, which is torch's
convention for the gradient of a real function of a complex tensor.  Both S
and G come from one ``ov_force`` call (solve, recomputed M X, site-local force
kernel) in the forward pass.
"""
import torch


class OvForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lattice, phi, xi):
        S, G, _ = lattice.force(xi.detach(), phi.detach())
        ctx.save_for_backward(G)
        return torch.tensor(sum(S), dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        return None, grad_out.to(G.dtype) * G, None
