"""torch.autograd.Function for the Hubbard energy E_U(psi, R).

Forward: project -> occupations -> U_eff (ACBN0, or a given U_eff) -> E_U
(Eq. E_Dudarev), all in the library's kernels.  Backward, with U_eff held
fixed as the ACBN0 potential prescribes (Sec. III, last paragraph before the
tables):
* dE/dpsi* = g_s dV w_k f_n (V_U psi) (Eq. minimization), returned in
  PyTorch's convention grad = 2 dE/dpsi*, computed by the apply kernel with
  per-state weights;
* dE/dR = -F, the Hubbard forces of Sec. IV through <grad phi|psi> with
  frozen sphere membership and normalization.
g_s = 2 for unpolarized contexts (their stored channel counts twice).
``R`` only carries the gradient: it must hold the context's site positions.
"""

import torch


class HubbardEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, R, hub, f, ueff=None):
        c = hub.project(psi)
        n, pbar, _ = hub.occupations(c, f, with_pbar=ueff is None, nbar=ueff is None)
        if ueff is None:
            _, _, ueff_t, _ = hub.acbn0(n, pbar)
        else:
            ueff_t = ueff.detach().to(torch.float64).contiguous()
        EU = hub.energy(ueff_t, n)
        ctx.hub = hub
        ctx.save_for_backward(psi, c, n, ueff_t, f)
        return EU.sum()

    @staticmethod
    def backward(ctx, grad_out):
        psi, c, n, ueff, f = ctx.saved_tensors
        hub = ctx.hub
        g = float(grad_out)
        gs = 2.0 if hub.spin == "unpolarized" else 1.0
        grad_psi = grad_R = None
        if ctx.needs_input_grad[0]:
            w = torch.tensor(hub.kweights, dtype=torch.float64, device=f.device)
            per_set = 1 if hub.spin == "spinor" else (2 if hub.spin == "collinear" else 1)
            colscale = (w.repeat_interleave(per_set)[:, None] * f).contiguous()
            grad_psi = torch.zeros_like(psi)
            hub.apply(ueff, n, c, grad_psi, alpha=2.0 * gs * hub.dV * g, colscale=colscale)
        if ctx.needs_input_grad[1]:
            grad_R = -g * hub.forces(psi, c, f, ueff, n)
        return grad_psi, grad_R, None, None, None
