"""torch.autograd.Function for the Hubbard energy E_U(psi, R) at a given U_eff.

Forward: project -> occupations -> E_U (Eq. E_Dudarev; App. A for spinors)
in the library's kernels.  U_eff is an input held fixed: the ACBN0 potential
is the ordinary DFT+U potential, with U-bar and J-bar not differentiated
(Sec. III, last paragraph before the tables).  A caller running ACBN0 takes
U_eff from Hubbard.acbn0 first and passes it here; with U_eff a function of
psi the returned gradient would not be the derivative of the forward, so
None is refused.
Backward: hub_energy_gradient gives both gradients, with the occupation
weights, the spin degeneracy, the volume element and the incoming gradient
applied inside the library: d/dpsi* (Eq. minimization) in PyTorch's
convention, and dE/dR (minus the Hubbard forces of Sec. IV through
<grad phi|psi>, sphere membership and normalization frozen).
``R`` only carries the gradient: it must hold the context's site positions.
"""

import torch


class HubbardEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, R, hub, f, ueff):
        if ueff is None:
            raise ValueError("HubbardEnergy needs U_eff (per site); take it from Hubbard.acbn0 for ACBN0")
        c = hub.project(psi)
        n, _, _ = hub.occupations(c, f, with_pbar=False, nbar=False)
        ueff_t = ueff.detach().to(torch.float64).contiguous()
        EU = hub.energy(ueff_t, n)
        ctx.hub = hub
        ctx.save_for_backward(psi, c, n, ueff_t, f)
        return EU.sum()

    @staticmethod
    def backward(ctx, grad_out):
        psi, c, n, ueff, f = ctx.saved_tensors
        grad_psi, grad_R = ctx.hub.energy_gradient(psi, c, f, ueff, n, scale=float(grad_out),
                                                   want_psi=ctx.needs_input_grad[0],
                                                   want_R=ctx.needs_input_grad[1])
        return grad_psi, grad_R, None, None, None
