"""Differentiable unrolled sequential RL deconvolution.

Two torch.autograd.Functions around the library's hand-written adjoint
passes:
  * MVDLoss: forward runs n iterations from psi0 with the given PSFs and
    returns L = sum_v |psi_n (x) P_v - phi_v|^2; its gradients with respect
    to the PSF values and psi0 come from the same library call;
  * MVDDeconvolve: forward returns psi_n itself, so any loss written in torch
    can follow it; the forward records its checkpoints in the handle
    (mvd_forward_recorded) and backward is the library's vector-Jacobian
    product over that record (mvd_backward_recorded), or, if the handle has
    run something else in between, over a recomputed run (mvd_backward).
n_iter is the number of iterations, or a pair (n, variant) for runs with a
compound back-projection kernel ("eff", "opt1", "opt2"; the default is RL),
whose gradients also flow through the kernels' construction.
psf_from_theta builds the anisotropic Gaussian PSF of a view from
(sigma_xy, sigma_z) in torch, so gradients reach the PSF parameters through
autograd.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import mvd


def _run(n_iter):
    return (int(n_iter[0]), n_iter[1]) if isinstance(n_iter, (tuple, list)) else (int(n_iter), "rl")


class MVDLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, handle, n_iter, psi0, *psfs):
        handle.set_psfs([p.detach().to("cpu", torch.float32).numpy() for p in psfs])
        want_p = any(ctx.needs_input_grad[3:])
        want_psi = ctx.needs_input_grad[2]
        n, variant = _run(n_iter)
        loss, gp, gpsi = handle.loss_grad(n, psi0, grad_psf=want_p, grad_psi0=want_psi, variant=variant)
        # gradients come back on the device and in the dtype of each input
        ctx.gp = None if gp is None else [torch.from_numpy(g).to(dtype=p.dtype, device=p.device)
                                          for g, p in zip(gp, psfs)]
        ctx.gpsi = None if gpsi is None else gpsi.to(dtype=psi0.dtype, device=psi0.device)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        gpsi = None if ctx.gpsi is None else ctx.gpsi * gout.to(ctx.gpsi.device)
        n_psf = len(ctx.needs_input_grad) - 3
        gps = (None,) * n_psf if ctx.gp is None else tuple(g * gout.to(g.device) for g in ctx.gp)
        return (None, None, gpsi) + gps


class MVDDeconvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, handle, n_iter, psi0, *psfs):
        host = [p.detach().to("cpu", torch.float32).numpy() for p in psfs]
        handle.set_psfs(host)
        n, variant = _run(n_iter)
        out, token = handle.forward_recorded(n, psi0.detach(), variant=variant)
        ctx.handle, ctx.n_iter, ctx.variant, ctx.host, ctx.token = handle, n, variant, host, token
        ctx.psi0 = psi0.detach()
        ctx.meta = [(p.dtype, p.device) for p in psfs]
        ctx.psi_meta = (psi0.dtype, psi0.device)
        return out.to(dtype=psi0.dtype, device=psi0.device)

    @staticmethod
    def backward(ctx, gout):
        want_p = any(ctx.needs_input_grad[3:])
        want_psi = ctx.needs_input_grad[2]
        h = ctx.handle
        try:
            gp, gpsi = h.backward_recorded(ctx.token, gout, grad_psf=want_p, grad_psi0=want_psi)
        except mvd.MVDError as e:
            if e.code != mvd.MVD_ESTATE:
                raise
            # the handle ran other work since the forward pass: recompute
            h.set_psfs(ctx.host)
            gp, gpsi = h.backward(ctx.n_iter, ctx.psi0, gout, grad_psf=want_p, grad_psi0=want_psi,
                                  variant=ctx.variant)
        gps = (None,) * len(ctx.meta) if gp is None else \
            tuple(torch.from_numpy(g).to(dtype=dt, device=dev) for g, (dt, dev) in zip(gp, ctx.meta))
        if gpsi is not None:
            gpsi = gpsi.to(dtype=ctx.psi_meta[0], device=ctx.psi_meta[1])
        return (None, None, gpsi) + gps


def psf_from_theta(sigma_xy, sigma_z, theta_deg, extent_xyz):
    """Unnormalised anisotropic Gaussian exp(-d^T C^-1 d / 2) with C =
    R_y(theta) diag(sxy^2, sxy^2, sz^2) R_y(theta)^T on an odd box, as a torch
    float64 tensor (kz, ky, kx) differentiable in (sigma_xy, sigma_z)."""
    kx, ky, kz = extent_xyz
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    z, y, x = torch.meshgrid(torch.arange(kz, dtype=torch.float64) - (kz - 1) / 2,
                             torch.arange(ky, dtype=torch.float64) - (ky - 1) / 2,
                             torch.arange(kx, dtype=torch.float64) - (kx - 1) / 2, indexing="ij")
    # coordinates in the PSF's own frame: R^T d
    u = c * x - s * z
    w = s * x + c * z
    q = (u * u + y * y) / (sigma_xy * sigma_xy) + (w * w) / (sigma_z * sigma_z)
    return torch.exp(-0.5 * q)


def loss_and_theta_grad(handle, n_iter, psi0, theta, angles, extent_xyz):
    """Loss and d loss / d theta for theta = [[sigma_xy, sigma_z] per view]."""
    th = torch.as_tensor(np.asarray(theta, np.float64)).clone().requires_grad_(True)
    psfs = [psf_from_theta(th[v, 0], th[v, 1], angles[v], extent_xyz) for v in range(len(angles))]
    L = MVDLoss.apply(handle, n_iter, psi0, *psfs)
    L.backward()
    return float(L.detach()), th.grad.numpy().copy()
