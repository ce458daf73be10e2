"""PSF refinement driven by the differentiated deconvolution.

The paper measures its PSFs from beads; it shows the deconvolution tolerates
moderately wrong PSFs and remarks that a PSF measured inside the sample would
improve it further (the section on PSF robustness).  With the differentiated
form the PSF parameters can instead be fitted to the views themselves: with
several views a wrong PSF leaves them mutually inconsistent, so the data
misfit after n RL iterations,

    L(theta) = sum_v |psi_n(theta) (x) P_v(theta) - phi_v|^2,

identifies the PSFs.  P_v(theta) is the rotated anisotropic Gaussian of each
view with parameters (sigma_xy, sigma_z); the gradient comes from the
library's adjoint passes (through the normalisation of each PSF) and torch
autograd through the Gaussian model.  The descent works on log(theta), so the
widths stay positive, with a fixed relative step length that halves until the
loss decreases (backtracking).
"""
from __future__ import annotations

import numpy as np

from . import mvd
from .autograd import loss_and_theta_grad, psf_from_theta


def refine(views, angles, extent_xyz, theta0, n_iter=4, steps=15, step=0.05, min_step=1e-3, psi0=None):
    """Fit theta ([sigma_xy, sigma_z] per view) to the views.  Returns the
    final theta and the history of (loss, theta) after every accepted step
    (the first entry is the start)."""
    th = np.log(np.asarray(theta0, np.float64))
    psfs = [psf_from_theta(*np.exp(th[v]), angles[v], extent_xyz).numpy().astype(np.float32)
            for v in range(len(angles))]
    with mvd.Deconvolver(views, psfs) as d:
        if psi0 is None:
            psi0 = np.full(views[0].shape, d.stats()["scale"], np.float32)
        L, g = loss_and_theta_grad(d, n_iter, psi0, np.exp(th), angles, extent_xyz)
        hist = [(L, np.exp(th))]
        for _ in range(steps):
            glog = g * np.exp(th)  # d L / d log(theta)
            n = float(np.linalg.norm(glog))
            if n == 0.0:
                break
            s = step
            while s >= min_step:
                cand = th - s * glog / n
                Lc, gc = loss_and_theta_grad(d, n_iter, psi0, np.exp(cand), angles, extent_xyz)
                if Lc < L:
                    th, L, g = cand, Lc, gc
                    hist.append((L, np.exp(th)))
                    break
                s *= 0.5
            else:
                break
    return np.exp(th), hist
