"""Differentiable ground-state energy and Green function through the C ABI.

``ground_energy(model, keys, t, U, eps)`` returns E0 of H~(t, U, eps) on the
basis ``keys`` as a torch scalar whose gradient with respect to the bond
amplitudes t [n_bonds], on-site U [n_orb] and orbital energies eps [n_orb]
is <Omega| dH~/dtheta |Omega> (Hellmann-Feynman), evaluated by
``mcd_hamiltonian_contract`` on the GPU.  Parameters can be functions of other
tensors (for example the 33 impurity parameters eps_b, V_ib, U); autograd
composes the chain rule.

``green_function(...)`` returns (E0, G) with G the band-Lanczos Green
function [n_freq, n_sel, n_sel] (complex128); when a derivative is needed
the forward keeps its two sector runs (``mcd_band_lanczos_green_keep``) and
the backward is one call of ``mcd_band_green_vjp_keep`` (resolvent
contraction over the kept Krylov blocks, Hellmann-Feynman dE0, and one
conjugate-gradient solve for the ground-state response), so a loss of G and
E0 gets its gradient with respect to every bond amplitude, U_i and eps_i in
one backward pass.
"""
from __future__ import annotations

import numpy as np

from . import Operator, band_green_vjp, band_lanczos_green, lanczos_ground


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
            _require_converged(info, "ground state")
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
_GFN = None


class NotConvergedError(RuntimeError):
    """A solve behind a differentiable quantity stopped at its iteration cap:
    the value (and Hellmann-Feynman or response gradients built on it) would
    not belong to the converged state."""


def _require_converged(info, what):
    if not info.converged:
        raise NotConvergedError(
            f"{what} did not converge (iterations {info.iters}, residual {info.residual:.3e}); "
            "raise max_iter / cg_max_iter or loosen the tolerance")


def _make_green_function():
    torch = _torch()

    class GreenFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t, U, eps, model, keys, orbitals, spins, omega, band_kw, lanczos_kw,
                    storage):
            m = model.with_params(
                bonds=[(b[0], b[1], float(v)) for b, v in zip(model.bonds, t.detach().cpu().numpy())],
                U=U.detach().cpu().numpy(), eps=eps.detach().cpu().numpy())
            op = Operator(m, keys, storage=storage)
            e0, psi, _, _, info = lanczos_ground(op, **lanczos_kw)
            op.close()
            _require_converged(info, "ground state")
            # with a derivative ahead, keep the sector runs for it (no recomputation)
            ctx.keep = None
            if any(ctx.needs_input_grad[:3]) and not band_kw.get("per_column", False):
                G, _, ctx.keep = band_lanczos_green(m, keys, psi, e0, orbitals, spins, omega,
                                                    keep=True, **band_kw)
            else:
                G, _ = band_lanczos_green(m, keys, psi, e0, orbitals, spins, omega, **band_kw)
            ctx.m, ctx.keys, ctx.psi, ctx.e0 = m, keys, psi, e0
            ctx.sel = (orbitals, spins, omega)
            ctx.band_kw = band_kw
            ctx.shapes = (t, U, eps)
            return (torch.tensor(e0, dtype=torch.float64, device=t.device),
                    torch.as_tensor(G, device=t.device))

        @staticmethod
        def backward(ctx, e0_bar, G_bar):
            orbitals, spins, omega = ctx.sel
            nf, ns = len(omega), len(orbitals)
            gb = (np.zeros((nf, ns, ns), dtype=np.complex128) if G_bar is None
                  else G_bar.detach().cpu().numpy().astype(np.complex128))
            eb = 0.0 if e0_bar is None else float(e0_bar.item())
            kw = {k: v for k, v in ctx.band_kw.items() if k not in ("w_t", "per_column")}
            # the kept runs serve the first backward and are then released (a
            # second backward recomputes them: same result)
            kept, ctx.keep = ctx.keep, None
            try:
                dt, dU, de, vinfo = band_green_vjp(ctx.m, ctx.keys, ctx.psi, ctx.e0, orbitals,
                                                   spins, omega, gb, e0_bar=eb, keep=kept, **kw)
            finally:
                if kept is not None:
                    kept.close()
            _require_converged(vinfo, "response solve of the Green-function derivative")
            t, U, eps = ctx.shapes
            as_t = lambda a, ref: torch.as_tensor(a, dtype=ref.dtype, device=ref.device)
            return (as_t(dt, t), as_t(dU, U), as_t(de, eps), None, None, None, None, None, None,
                    None, None)

    return GreenFunction


def green_function(model, keys, t, U, eps, orbitals, spins, omega, storage="csr",
                   lanczos_kw=None, **band_kw):
    """(E0, G) as differentiable torch tensors; G = G+ + G- [n_freq, n_sel, n_sel]
    complex128 from ``band_lanczos_green`` with ``band_kw`` (w_t must stay 1)."""
    global _GFN
    if _GFN is None:
        _GFN = _make_green_function()
    if band_kw.get("w_t", 1.0) != 1.0:
        raise ValueError("the derivative of G needs w_t = 1")
    kw = dict(max_iter=600, tol=1e-12, seed=11)
    kw.update(lanczos_kw or {})
    return _GFN.apply(t, U, eps, model, keys, list(orbitals), list(spins),
                      np.asarray(omega, dtype=np.float64), dict(band_kw), kw, storage)


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
