"""torch.autograd binding of the hand-written adjoint (qmc_grad).

``Wavefunction`` holds the variational parameters theta = [primitive
exponents | MO coefficients (n_ao x n_mo, row-major) | Pade b | e-n
parameters per nucleus | e-e-n parameters per term (when the system has
them)] and the nuclear positions R as leaf tensors.  ``psi_eloc(wf, X)`` returns
(log|Psi|, sign, E_L) per walker from the HIP evaluation kernel; its backward
pass calls qmc_grad once and applies the per-walker Jacobians to the incoming
gradients, so any scalar built from log|Psi| and E_L differentiates to theta
and R without a tape through the kernels.

With these two outputs the estimators of the Methods section are plain torch
expressions over walkers:
  eq. nabla_loss  dE/dtheta = 2 <(E_L - E) d log|Psi|/dtheta>
                  (the surrogate  mean(E_L) + 2 mean((E_L - E).detach() * log|Psi|)
                   has this gradient plus <dE_L/dtheta>, whose expectation is 0)
  eq. force       F_alpha = -<dE_L/dR_alpha + (E_L - E) 2 d log|Psi|/dR_alpha>
                  (the same surrogate, differentiated to R, gives -F)

The handle is rebuilt from the tensors whenever their values change (after an
optimiser step), so the kernels always see the parameters autograd
differentiates.  Walker positions are inputs, not parameters: no gradient
flows to X.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qmc


def _jastrow_blocks(sysd: dict):
    """The many-body Jastrow arrays the system carries, in the qmc_grad order."""
    out = []
    if sysd.get("jas_en") is not None:
        out.append(("jas_en", np.asarray(sysd["jas_en"], dtype=np.float64).shape))
    een = sysd.get("jas_een")
    if een is not None and len(een) > 0:
        out.append(("jas_een", np.asarray(een, dtype=np.float64).shape))
    return out


def pack_theta(sysd: dict) -> np.ndarray:
    """theta in the qmc_grad layout."""
    parts = [np.asarray(sysd["prim_exp"], dtype=np.float64).ravel(),
             np.asarray(sysd["mo_coef"], dtype=np.float64).ravel(),
             [float(sysd.get("jas_b", 1.0))]]
    for key, _ in _jastrow_blocks(sysd):
        parts.append(np.asarray(sysd[key], dtype=np.float64).ravel())
    return np.concatenate(parts)


def unpack_theta(sysd: dict, theta, R) -> dict:
    """A copy of the system dict with theta and R substituted."""
    theta = np.asarray(theta, dtype=np.float64)
    n_prim = int(np.asarray(sysd["prim_exp"]).size)
    shape = np.asarray(sysd["mo_coef"]).shape
    n_mo_coef = shape[0] * shape[1]
    blocks = _jastrow_blocks(sysd)
    n = n_prim + n_mo_coef + 1 + sum(int(np.prod(sh)) for _, sh in blocks)
    if theta.shape != (n,):
        raise ValueError(f"theta has shape {theta.shape}, expected ({n},)")
    d = dict(sysd)
    d["prim_exp"] = theta[:n_prim].copy()
    d["mo_coef"] = np.ascontiguousarray(theta[n_prim:n_prim + n_mo_coef].reshape(shape))
    q = n_prim + n_mo_coef
    d["jas_b"] = float(theta[q])
    q += 1
    for key, sh in blocks:
        k = int(np.prod(sh))
        d[key] = np.ascontiguousarray(theta[q:q + k].reshape(sh))
        q += k
    d["R"] = np.asarray(R, dtype=np.float64).reshape(-1, 3).copy()
    return d


class Wavefunction:
    """Slater-Jastrow parameters as differentiable tensors on the host
    (a few hundred doubles; the kernels read a device copy made at create)."""

    def __init__(self, sysd: dict, device: int = 0):
        self.base = sysd
        self.device = device
        self.theta = torch.tensor(pack_theta(sysd), dtype=torch.float64, requires_grad=True)
        self.R = torch.tensor(np.asarray(sysd["R"], dtype=np.float64).reshape(-1, 3),
                              requires_grad=True)
        self._system = None
        self._built_from = None

    def system(self) -> qmc.System:
        """The device system for the current parameter values."""
        cur = (self.theta.detach().clone(), self.R.detach().clone())
        if (self._system is None or not torch.equal(cur[0], self._built_from[0])
                or not torch.equal(cur[1], self._built_from[1])):
            sysd = unpack_theta(self.base, cur[0].numpy(), cur[1].numpy())
            # the previous handle stays alive while a pending backward holds it
            self._system, self._built_from = qmc.System(sysd, self.device), cur
        return self._system

    def close(self):
        if self._system is not None:
            self._system.close()
            self._system = None


class _PsiEloc(torch.autograd.Function):
    @staticmethod
    def forward(ctx, wf: Wavefunction, X, theta, R):
        system = wf.system()
        lp, sg, el = system.eval(X)
        ctx.system = system
        ctx.save_for_backward(X)
        ctx.mark_non_differentiable(sg)
        return lp, sg, el

    @staticmethod
    def backward(ctx, g_lp, g_sg, g_el):
        (X,) = ctx.saved_tensors
        need_theta, need_R = ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        if not (need_theta or need_R):
            return None, None, None, None
        dl, de, dlR, deR = ctx.system.grad(X)
        W = X.shape[0]
        g_lp = torch.zeros(W, dtype=torch.float64, device=X.device) if g_lp is None else g_lp
        g_el = torch.zeros(W, dtype=torch.float64, device=X.device) if g_el is None else g_el

        def vjp(g, J):
            # walkers that receive no gradient contribute nothing, even where
            # their Jacobian row is not finite (a singular walker)
            return g @ torch.where((g != 0)[:, None], J.reshape(W, -1), 0.0)

        g_theta = g_R = None
        if need_theta:
            g_theta = (vjp(g_lp, dl) + vjp(g_el, de)).cpu()
        if need_R:
            g_R = (vjp(g_lp, dlR) + vjp(g_el, deR)).reshape(-1, 3).cpu()
        return None, None, g_theta, g_R


def psi_eloc(wf: Wavefunction, X: torch.Tensor):
    """(log|Psi|, sign, E_L) of walkers X [W, N_e, 3] (float64, on the
    system's device), differentiable with respect to wf.theta and wf.R."""
    return _PsiEloc.apply(wf, X, wf.theta, wf.R)
