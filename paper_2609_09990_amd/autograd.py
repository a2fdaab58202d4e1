"""DMRG energy as a differentiable node (the sweep as one node of the energy
graph, Sec. II.C): forward runs two-site sweeps on the GPU and returns the MPS
energies; backward seeds the state weights with the incoming cotangent and
calls dmrg_grad, which contracts the state's densities with the integral
derivatives without forming them.  The MPS is held fixed (Hellmann-Feynman):
exact for converged full-bond states; at truncated bond the result is the
gradient of <Psi|H|Psi>/<Psi|Psi> of the final MPS (Sec. II.E).  Entries of h
and B are independent variables (a symmetric parameterisation sums the (p,q)
and (q,p) entries).
"""
import numpy as np
import torch

from ._lib import Problem, Solver


class DMRGEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, B, n_alpha, n_beta, e_core, opts):
        opts = dict(opts)
        n_sweeps = opts.pop("n_sweeps", 4)
        prob = Problem(h.detach().cpu().numpy(), B.detach().cpu().numpy(), n_alpha, n_beta, e_core)
        sol = Solver(prob, **opts)
        sol.sweep(n_sweeps)
        e = sol.energy()
        ctx.solver = sol
        ctx.meta = (h.dtype, h.device, B.dtype, B.device)
        return torch.as_tensor(e, dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, grad_e):
        sol = ctx.solver
        w = grad_e.detach().to("cpu", torch.float64).numpy()
        dh, dB, _ = sol.grad(np.ascontiguousarray(w))
        hdt, hdev, bdt, bdev = ctx.meta
        return (torch.as_tensor(dh, dtype=hdt, device=hdev), torch.as_tensor(dB, dtype=bdt, device=bdev),
                None, None, None, None)


def dmrg_energy(h, B, n_alpha, n_beta, e_core=0.0, *, n_sweeps=4, **solver_options):
    """Energies (n_states,) of the MPS after `n_sweeps` sweeps; differentiable in h and B.

    solver_options are those of Solver (M, n_states, weights, tol, max_iter, ...)."""
    opts = dict(solver_options)
    opts["n_sweeps"] = n_sweeps
    return DMRGEnergy.apply(h, B, int(n_alpha), int(n_beta), float(e_core), opts)
