"""torch.autograd.Function over the library's smeared-field MCG functional.

L(U, rho, eps) = R(S_n(U; rho, eps)^{G*}) with S_n the n-step stout
(eps = 1) or over-improved stout smearing (Sec. II.B) and G* held fixed (at a
converged maximum this is the derivative of the fixed functional, by the
envelope theorem).  The backward pass is the library's hand-written adjoint
(mcg_smear_mcg_backward), with checkpoint-and-recompute of the smeared
fields; U.grad follows torch's convention for a real loss of a complex input,
dL/dRe U + i dL/dIm U.
"""
import torch

from . import api


class StoutMCGLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, rho, eps, n, Gstar, ckpt_every=5):
        """U: complex interchange tensor [Lt, Lz, Ly, Lx, 4, 3, 3] on the GPU
        (complex128 -> FP64 path, complex64 -> FP32 links); rho, eps: floats
        or 0-dim tensors; Gstar: api.GaugeField."""
        r, e = float(rho), float(eps)
        Ul = api.to_links(U.detach())
        L = api.functional(api.apply_gauge(api.smear(Ul, r, e, int(n)), Gstar))
        ctx.save_for_backward(U.detach())
        ctx.params = (r, e, int(n), Gstar, int(ckpt_every), torch.is_tensor(rho), torch.is_tensor(eps))
        return torch.tensor(L, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gL):
        (U,) = ctx.saved_tensors
        r, e, n, Gstar, ck, rho_t, eps_t = ctx.params
        grad, _, dr, de = api.smear_mcg_backward(api.to_links(U), r, e, n, Gstar, ck)
        g = float(gL)
        gU = api.from_links(grad, U.dtype) * g if ctx.needs_input_grad[0] else None
        grho = torch.tensor(dr * g, dtype=torch.float64, device=U.device) if rho_t else None
        geps = torch.tensor(de * g, dtype=torch.float64, device=U.device) if eps_t else None
        return gU, grho, geps, None, None, None


def stout_mcg_loss(U, rho, eps, n, Gstar, ckpt_every=5):
    return StoutMCGLoss.apply(U, rho, eps, n, Gstar, ckpt_every)
