"""Simulated multi-view SPIM acquisitions (the paper's section on the
simulation of SPIM data), for experiments on data with the degradations of a
real light-sheet microscope rather than the periodic blob volumes of synth.py.

Object: a sphere made of many small spheres with random centres, radii and
intensities, drawn at twice the final resolution and averaged down 2x2x2.
Ground truth: the object rotated by 15 degrees about the x axis, so that the
ground truth and the views all carry one interpolating rotation.  View n (at
angle a_n): the object rotated by a_n + 15 degrees about x (the microscope's
frame), then
  * attenuation along the light sheet: photons entering from the -y side are
    absorbed at rate delta times the density they cross (Beer-Lambert,
    delta = 0.01 per voxel of unit density, density = intensity / maximum),
  * convolution with the view's PSF (detection axis z),
  * axial sampling of every third z plane, Poisson counts with the convolved
    intensity as mean,
  * registration: linear rescaling to the isotropic grid along z, rotation
    back by -a_n about x (linear interpolation throughout).
The PSFs for deconvolution are the acquisition PSFs rotated into the ground
truth frame (exactly, for the analytic Gaussian model).

This is a data generator (numpy/scipy on the host); it holds none of the
deconvolution's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage, signal


@dataclass
class Acquisition:
    dims: tuple                 # (nx, ny, nz) of the reconstruction grid
    truth: np.ndarray           # (nz, ny, nx) float32, ground truth frame
    views: list                 # registered views (nz, ny, nx) float32
    psfs: list                  # PSFs in the ground truth frame (kz, ky, kx) float32
    angles: list
    meta: dict = field(default_factory=dict)


def sphere_object(dims, n_spheres, seed, radius_frac=0.36, r_range=(0.6, 2.2), i_range=(50.0, 250.0)):
    """A big sphere filled with small spheres of random centre, radius and
    intensity, drawn at twice the resolution and averaged down 2x2x2."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    hx, hy, hz = 2 * nx, 2 * ny, 2 * nz
    vol = np.zeros((hz, hy, hx), np.float32)
    R = radius_frac * 2 * min(nx, ny, nz)
    c0 = np.array([hz, hy, hx]) / 2.0
    for _ in range(n_spheres):
        # uniform point in the big sphere
        while True:
            p = rng.uniform(-1, 1, 3)
            if p @ p <= 1:
                break
        c = c0 + p * R
        r = 2 * rng.uniform(*r_range)
        a = rng.uniform(*i_range)
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, [hz, hy, hx])
        z, y, x = np.ogrid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        inside = (z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2 <= r * r
        np.maximum(vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]], a * inside, out=vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]])
    return vol.reshape(nz, 2, ny, 2, nx, 2).mean(axis=(1, 3, 5))


def rotate_x(vol, deg, order=1):
    """Rotate a (z, y, x) volume about the x axis through its centre (linear
    interpolation, zero outside)."""
    return ndimage.rotate(vol, deg, axes=(0, 1), reshape=False, order=order, mode="constant", cval=0.0)


def attenuate(vol, delta=0.01):
    """Light sheet entering from the -y side: the fraction of photons left at
    a voxel is exp(-delta * the density summed over the voxels before it),
    the density being the intensity relative to its maximum."""
    m = float(vol.max())
    if m <= 0:
        return vol.copy()
    before = np.cumsum(vol / m, axis=1) - vol / m
    return vol * np.exp(-delta * before)


def gaussian_psf_x(extent_xyz, sigma_xy, sigma_z, theta_deg):
    """Normalised anisotropic Gaussian (sigma_xy lateral, sigma_z along the
    detection axis z) rotated by theta about the x axis, sampled on an odd
    box (kz, ky, kx)."""
    kx, ky, kz = extent_xyz
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    z, y, x = np.meshgrid(np.arange(kz) - (kz - 1) / 2, np.arange(ky) - (ky - 1) / 2, np.arange(kx) - (kx - 1) / 2,
                          indexing="ij")
    # coordinates in the PSF's own frame (rotation about x mixes y and z, in
    # the sense of rotate_x: gaussian_psf_x(theta) = rotate_x(gaussian_psf_x(0), theta))
    v = c * y - s * z
    w = s * y + c * z
    g = np.exp(-0.5 * ((x * x + v * v) / sigma_xy ** 2 + w * w / sigma_z ** 2))
    return (g / g.sum()).astype(np.float32)


def acquire(obj, angle, psf_acq, rng, delta=0.01, axial_step=3, photons=1.0):
    """One view of the object at `angle`: rotate by angle + 15, attenuate,
    convolve, sample every axial_step-th plane with Poisson counts, rescale
    to the isotropic grid and rotate back by -angle."""
    v = rotate_x(obj, angle + 15.0)
    v = attenuate(v, delta)
    v = signal.fftconvolve(v, psf_acq, mode="same")
    v = np.maximum(v, 0.0)
    sampled = v[::axial_step]
    counts = rng.poisson(sampled * photons).astype(np.float32) / photons
    nz = obj.shape[0]
    zq = np.arange(nz) / axial_step
    iso = ndimage.map_coordinates(counts, np.meshgrid(zq, np.arange(obj.shape[1]), np.arange(obj.shape[2]),
                                                      indexing="ij"), order=1, mode="nearest")
    return np.maximum(rotate_x(iso, -angle), 0.0).astype(np.float32)


def simulate(dims=(96, 96, 96), angles=(0.0, 90.0, 180.0, 270.0), n_spheres=400, psf_extent=(13, 13, 25),
             sigma_xy=1.0, sigma_z=3.0, delta=0.01, photons=1.0, seed=1308):
    """A seeded multi-view acquisition of one sphere object."""
    ss = np.random.SeedSequence(seed)
    k_obj, k_noise = ss.spawn(2)
    obj = sphere_object(dims, n_spheres, k_obj)
    truth = rotate_x(obj, 15.0).astype(np.float32)
    rngs = [np.random.default_rng(q) for q in k_noise.spawn(len(angles))]
    acq_psf = gaussian_psf_x(psf_extent, sigma_xy, sigma_z, 0.0)
    views = [acquire(obj, a, acq_psf, r, delta, 3, photons) for a, r in zip(angles, rngs)]
    # the acquisition PSF seen in the ground truth frame: rotated by -angle
    psfs = [gaussian_psf_x(psf_extent, sigma_xy, sigma_z, -a) for a in angles]
    return Acquisition(dims=tuple(dims), truth=truth, views=views, psfs=psfs, angles=list(angles),
                       meta=dict(delta=delta, axial_step=3, photons=photons, seed=seed, n_spheres=n_spheres,
                                 sigma_xy=sigma_xy, sigma_z=sigma_z))


def correlation(a, b):
    """Pearson correlation of two volumes (the paper's quality measure)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    a = a - a.mean()
    b = b - b.mean()
    return float(a @ b / math.sqrt((a @ a) * (b @ b)))


def psf_robustness(acq, errors=(0.0, 5.0, 10.0, 20.0), variant="opt1", n_iter=20):
    """Deconvolve a simulated acquisition (sequential updates on the GPU)
    with each view's PSF rotated by a wrong angle, and report the best
    correlation to the ground truth and the iteration reaching it, per
    error (the paper's study of imperfect PSFs)."""
    import torch

    from . import mvd
    sx, sz = acq.meta.get("sigma_xy", 1.0), acq.meta.get("sigma_z", 3.0)
    ext = tuple(reversed(acq.psfs[0].shape))
    truth = torch.as_tensor(acq.truth).cuda()
    out = []
    for e in errors:
        psfs = [gaussian_psf_x(ext, sx, sz, -a + e) for a in acq.angles]
        best, at = -1.0, 0
        with mvd.Deconvolver(acq.views, psfs) as d:
            for it in range(n_iter):
                d.iterate(1, variant)
                psi = d.estimate()
                a = psi - psi.mean()
                b = truth - truth.mean()
                r = float((a * b).sum() / torch.sqrt((a * a).sum() * (b * b).sum()))
                if r > best:
                    best, at = r, it + 1
        out.append({"psf_error_deg": e, "best_correlation": round(best, 4), "at_iteration": at})
    return {"views_correlation": round(float(np.mean([correlation(v, acq.truth) for v in acq.views])), 4),
            "results": out}
