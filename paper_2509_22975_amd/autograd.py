"""Differentiable ground-state energy (Hellmann-Feynman through the C ABI).

``ground_energy(model, keys, t, U, eps)`` returns E0 of H~(t, U, eps) on the
basis ``keys`` as a torch scalar whose gradient with respect to the bond
amplitudes t [n_bonds], on-site U [n_orb] and orbital energies eps [n_orb]
is <Omega| dH~/dtheta |Omega> (Hellmann-Feynman), evaluated by
``mcd_hamiltonian_contract`` on the GPU.  Parameters can be functions of other
tensors (for example the 33 impurity parameters eps_b, V_ib, U); autograd
composes the chain rule.
"""
from __future__ import annotations

import numpy as np

from . import Operator, lanczos_ground


def _torch():
    import torch
    return torch


class _GroundEnergy:
    pass


def _make_function():
    torch = _torch()

    class GroundEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t, U, eps, model, keys, storage, lanczos_kw):
            m = model.with_params(
                bonds=[(b[0], b[1], float(v)) for b, v in zip(model.bonds, t.detach().cpu().numpy())],
                U=U.detach().cpu().numpy(), eps=eps.detach().cpu().numpy())
            op = Operator(m, keys, storage=storage)
            e0, psi, _, _, info = lanczos_ground(op, **lanczos_kw)
            dt, dU, de = op.contract(psi)
            op.close()
            ctx.save_for_backward(torch.as_tensor(dt, dtype=t.dtype, device=t.device),
                                  torch.as_tensor(dU, dtype=U.dtype, device=U.device),
                                  torch.as_tensor(de, dtype=eps.dtype, device=eps.device))
            return torch.tensor(e0, dtype=torch.float64, device=t.device)

        @staticmethod
        def backward(ctx, g):
            dt, dU, de = ctx.saved_tensors
            return g * dt, g * dU, g * de, None, None, None, None

    return GroundEnergy


_FN = None


def ground_energy(model, keys, t, U, eps, storage="csr", **lanczos_kw):
    """E0(t, U, eps) as a differentiable torch scalar (see module docstring)."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    kw = dict(max_iter=600, tol=1e-12, seed=11)
    kw.update(lanczos_kw)
    return _FN.apply(t, U, eps, model, keys, storage, kw)


def impurity_parameters(model):
    """theta = (eps_b [8], V_ib [24], U) of the impurity + bath model and a
    function mapping theta (torch) to (t, U, eps) tensors."""
    torch = _torch()
    n = model.n_orb
    imp = [i for i in range(n) if model.U[i] != 0.0]
    baths = [i for i in range(n) if model.U[i] == 0.0]
    hyb = [q for q, b in enumerate(model.bonds) if (b[0] in imp) != (b[1] in imp)]
    theta0 = np.concatenate([model.eps[baths], [model.bonds[q][2] for q in hyb],
                             [model.U[imp[0]]]])

    def expand(theta):
        t = torch.tensor([b[2] for b in model.bonds], dtype=torch.float64, device=theta.device)
        t = t.index_put((torch.tensor(hyb, device=theta.device),), theta[len(baths):len(baths) + len(hyb)])
        U = torch.zeros(n, dtype=torch.float64, device=theta.device)
        U = U.index_put((torch.tensor(imp, device=theta.device),), theta[-1].expand(len(imp)))
        eps = torch.tensor(model.eps, dtype=torch.float64, device=theta.device)
        eps = eps.index_put((torch.tensor(baths, device=theta.device),), theta[:len(baths)])
        # impurity orbital energies are -U/2 (mu = U/2 on the impurity)
        eps = eps.index_put((torch.tensor(imp, device=theta.device),), (-0.5 * theta[-1]).expand(len(imp)))
        return t, U, eps

    return theta0, expand
