"""Seeded synthetic inputs: ground truth, PSFs, views and weights.

This module is the one place both sides of the parity tests draw their inputs
from.  It holds none of the deconvolution arithmetic: views are rendered
analytically (a Gaussian blob seen through a Gaussian PSF is again a Gaussian,
with the covariances added), never by convolving arrays, so no blur, ratio or
update step lives here.

Conventions: volumes of dims (nx, ny, nz) are C-ordered numpy arrays of shape
(nz, ny, nx); PSF boxes of extents (kx, ky, kz) have shape (kz, ky, kx).
View angles rotate the detection axis (z at 0 deg) about y.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 13080730


def rot_y(theta_deg):
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def psf_cov(sigma_xy, sigma_z, theta_deg):
    """Covariance (in x, y, z) of the anisotropic PSF of a view rotated about y."""
    R = rot_y(theta_deg)
    return R @ np.diag([sigma_xy ** 2, sigma_xy ** 2, sigma_z ** 2]) @ R.T


def gaussian_psf(extent_xyz, sigma_xy, sigma_z, theta_deg, dtype=np.float32):
    """Rotated anisotropic Gaussian sampled at integer offsets of an odd box
    centred at (k-1)/2, normalised to sum one."""
    kx, ky, kz = extent_xyz
    C = psf_cov(sigma_xy, sigma_z, theta_deg)
    Ci = np.linalg.inv(C)
    dz, dy, dx = np.meshgrid(np.arange(kz) - (kz - 1) / 2.0, np.arange(ky) - (ky - 1) / 2.0,
                             np.arange(kx) - (kx - 1) / 2.0, indexing="ij")
    d = np.stack([dx, dy, dz], axis=-1)
    q = np.einsum("...i,ij,...j->...", d, Ci, d)
    g = np.exp(-0.5 * q)
    return (g / g.sum()).astype(dtype)


def _window(center, cov, shape_zyx):
    """Evaluate exp(-1/2 d^T C^-1 d) on a periodic window around `center`.

    The covariance must keep y decoupled from x and z (rotations about y), so
    the window is the outer product of a y profile and an (x, z) profile."""
    assert abs(cov[0, 1]) < 1e-12 and abs(cov[1, 2]) < 1e-12
    nz, ny, nx = shape_zyx
    r = [int(math.ceil(4.0 * math.sqrt(cov[i, i]))) for i in range(3)]
    r = [min(r[0], (nx - 1) // 2), min(r[1], (ny - 1) // 2), min(r[2], (nz - 1) // 2)]
    base = [int(round(center[i])) for i in range(3)]
    off = [np.arange(-r[i], r[i] + 1) for i in range(3)]
    d = [base[i] + off[i] - center[i] for i in range(3)]
    gy = np.exp(-0.5 * d[1] ** 2 / cov[1, 1])
    M = np.linalg.inv(np.array([[cov[0, 0], cov[0, 2]], [cov[2, 0], cov[2, 2]]]))
    DX, DZ = np.meshgrid(d[0], d[2], indexing="xy")  # (nzw, nxw)
    gxz = np.exp(-0.5 * (M[0, 0] * DX * DX + 2.0 * M[0, 1] * DX * DZ + M[1, 1] * DZ * DZ))
    block = gxz[:, None, :] * gy[None, :, None]
    idx = ((base[2] + off[2]) % nz, (base[1] + off[1]) % ny, (base[0] + off[0]) % nx)
    return idx, block


def render(shape_zyx, centers, amps, covs, background):
    """Sum of Gaussian blobs A exp(-1/2 d^T C^-1 d) on a periodic grid."""
    vol = np.full(shape_zyx, background, dtype=np.float64)
    for c, a, C in zip(centers, amps, covs):
        idx, block = _window(c, C, shape_zyx)
        vol[np.ix_(*idx)] += a * block
    return vol


@dataclass
class Synthetic:
    dims: tuple                 # (nx, ny, nz)
    truth: np.ndarray           # (nz, ny, nx) float32
    views: list                 # N x (nz, ny, nx) float32
    psfs: list                  # N x (kz, ky, kx) float32
    weights: list | None        # N x (nz, ny, nx) float32 or None
    angles: list
    lam: float = 0.0
    variant: int = 1
    n_iter: int = 1
    meta: dict = field(default_factory=dict)


def blob_params(rng, n, dims, shell=None):
    """Blob centres (x, y, z), sigmas U[1.5, 3] and amplitudes U[200, 1000]."""
    nx, ny, nz = dims
    if shell is None:
        centers = rng.uniform(0.0, 1.0, size=(n, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    else:
        u = rng.normal(size=(n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        rad = rng.uniform(shell[0], shell[1], size=(n, 1))
        semi = 0.4 * np.array([nx, ny, nz], dtype=np.float64)
        centers = np.array([nx, ny, nz], dtype=np.float64) / 2.0 + u * rad * semi
    sig = rng.uniform(1.5, 3.0, size=n)
    amp = rng.uniform(200.0, 1000.0, size=n)
    return centers, sig, amp


def make_views(dims, centers, sig, amp, angles, sigma_xy, sigma_z, background):
    """Noise-free views: each blob seen through view v's PSF is a Gaussian with
    covariance sigma^2 I + Sigma_v and the same mass."""
    shape = (dims[2], dims[1], dims[0])

    def one(th):
        Cp = psf_cov(sigma_xy, sigma_z, th)
        covs, amps = [], []
        for s, a in zip(sig, amp):
            C = s * s * np.eye(3) + Cp
            covs.append(C)
            amps.append(a * s ** 3 / math.sqrt(np.linalg.det(C)))
        return render(shape, centers, amps, covs, background)

    with ThreadPoolExecutor(max(1, min(len(angles), os.cpu_count() or 1))) as ex:
        return list(ex.map(one, angles))


def make_truth(dims, centers, sig, amp, background):
    shape = (dims[2], dims[1], dims[0])
    covs = [s * s * np.eye(3) for s in sig]
    return render(shape, centers, amp, covs, background)


def overlap_weights(dims, angles, band=32.0, ramp=16.0):
    """Per-view weights for partially overlapping views.

    A view sees the half-space on its detection side (detection axis
    R_y(theta) e_z) plus a band of `band` voxels; below that the weight falls
    to zero along a cosine ramp of `ramp` voxels.  Then the per-voxel sum over
    views is limited to the minimal overlap m (the smallest per-voxel sum):
    w_v <- w_v min(1, m / sum_v w_v), so no weight ever exceeds one.
    """
    nx, ny, nz = dims
    z, x = np.meshgrid(np.arange(nz) - (nz - 1) / 2.0, np.arange(nx) - (nx - 1) / 2.0, indexing="ij")
    ws = []
    for th in angles:
        t = math.radians(th)
        s = x * math.sin(t) + z * math.cos(t)
        w = np.ones_like(s)
        lo = -band - ramp
        mid = (s < -band) & (s > lo)
        w[s <= lo] = 0.0
        w[mid] = 0.5 * (1.0 + np.cos(math.pi * (-band - s[mid]) / ramp))
        ws.append(w)
    S = np.sum(ws, axis=0)
    m = float(S[S > 0].min())
    f = np.minimum(1.0, m / np.maximum(S, 1e-30))
    out = []
    for w in ws:
        w2 = np.clip(w * f, 0.0, 1.0).astype(np.float32)
        out.append(np.ascontiguousarray(np.broadcast_to(w2[:, None, :], (nz, ny, nx))))
    return out


def _noisy(seq, vol, scale=1.0, chunks=16):
    """Poisson counts of vol * scale; z-slabs draw from their own child seeds
    (so the result does not depend on the thread count)."""
    kids = seq.spawn(chunks)
    edges = np.linspace(0, vol.shape[0], chunks + 1).astype(int)
    out = np.empty(vol.shape, np.float32)

    def slab(i):
        a, b = edges[i], edges[i + 1]
        out[a:b] = np.random.default_rng(kids[i]).poisson(vol[a:b] * scale)

    with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        list(ex.map(slab, range(chunks)))
    return out


def make_problem(dims, n_blobs, angles, psf_extent, sigma_xy, sigma_z, seed,
                 background=5.0, noise="photons", weights=False, lam=0.0,
                 variant=1, n_iter=1, shell=None):
    """Generic seeded problem.  noise: 'none', 'photons' (Poisson of the
    noise-free view in photon units) or 'peak1000' (one global scale so the
    brightest noise-free voxel over all views is 1000 photons)."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(4)
    rng_blobs = np.random.default_rng(kids[0])
    noise_seqs = kids[1].spawn(len(angles))
    centers, sig, amp = blob_params(rng_blobs, n_blobs, dims, shell)
    truth = make_truth(dims, centers, sig, amp, background)
    clean = make_views(dims, centers, sig, amp, angles, sigma_xy, sigma_z, background)
    if noise == "none":
        views = [v.astype(np.float32) for v in clean]
    elif noise == "photons":
        views = [_noisy(q, v) for q, v in zip(noise_seqs, clean)]
    elif noise == "peak1000":
        sc = 1000.0 / max(float(v.max()) for v in clean)
        views = [_noisy(q, v, sc) for q, v in zip(noise_seqs, clean)]
        truth = truth * sc
    else:
        raise ValueError(noise)
    psfs = [gaussian_psf(psf_extent, sigma_xy, sigma_z, th) for th in angles]
    w = overlap_weights(dims, angles) if weights else None
    return Synthetic(dims=tuple(dims), truth=truth.astype(np.float32), views=views, psfs=psfs,
                     weights=w, angles=list(angles), lam=lam, variant=variant, n_iter=n_iter,
                     meta=dict(n_blobs=n_blobs, sigma_xy=sigma_xy, sigma_z=sigma_z, seed=seed))


# ------------------------------------------------------- the five workloads --

def config1(scale=1):
    """64^3, 40 blobs, views 0/90 deg, 17^3 PSFs (sigma_xy 1.0, sigma_z 3.5),
    Poisson in photon units, efficient update, 5 iterations."""
    return make_problem((64, 64, 64), 40, [0.0, 90.0], (17, 17, 17), 1.0, 3.5,
                        SEED_BASE + 0, variant=1, n_iter=5)


def config2(variant=1):
    """128^3, 150 blobs, views 0/45/90/135 deg, 25^3 PSFs (1.2, 4.0), Poisson
    at peak 1000 photons, 20 iterations (RL and efficient)."""
    return make_problem((128, 128, 128), 150, [0.0, 45.0, 90.0, 135.0], (25, 25, 25), 1.2, 4.0,
                        SEED_BASE + 1, noise="peak1000", variant=variant, n_iter=20)


def config3(dims=(512, 512, 256), n_blobs=3000, psf_extent=(31, 31, 41)):
    """Embryo scale: 512x512x256, 3000 blobs on an ellipsoidal shell, six
    views at 60 deg steps, 31x31x41 PSFs (1.2, 4.0), overlap weights,
    lambda 0.0006, Optimization I, 10 iterations."""
    return make_problem(dims, n_blobs, [0.0, 60.0, 120.0, 180.0, 240.0, 300.0], psf_extent,
                        1.2, 4.0, SEED_BASE + 2, weights=True, lam=0.0006, variant=2,
                        n_iter=10, shell=(0.9, 1.0))


def smooth5_even(lo, hi):
    out = []
    for n in range(lo, hi + 1):
        if n % 2:
            continue
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def config4_dims(n_blocks=48, seed=SEED_BASE + 3):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    xy = smooth5_even(96, 256)
    zz = smooth5_even(96, 160)
    dims = []
    for _ in range(n_blocks):
        dims.append((int(rng.choice(xy)), int(rng.choice(xy)), int(rng.choice(zz))))
    jit = rng.uniform(0.85, 1.15, size=(n_blocks, 2))
    return dims, jit


def config4(n_blocks=48, dims_override=None):
    """48 independent blocks of seeded even 5-smooth sizes (x, y in [96, 256],
    z in [96, 160]), blob density 40 per 64^3, 17^3 PSFs with widths jittered
    by U[0.85, 1.15], views 0/45/90/135 deg, efficient update, 10 iterations."""
    dims, jit = config4_dims(n_blocks)
    if dims_override is not None:
        dims = dims_override
    blocks = []
    for i, d in enumerate(dims):
        nb = max(1, int(round(40.0 * d[0] * d[1] * d[2] / 64 ** 3)))
        blocks.append(make_problem(d, nb, [0.0, 45.0, 90.0, 135.0], (17, 17, 17),
                                   1.0 * jit[i % len(jit), 0], 3.5 * jit[i % len(jit), 1],
                                   SEED_BASE + 1000 + i, variant=1, n_iter=10))
    return blocks


def larva(dims=(1640, 1070, 345), n_blobs=6000, n_views=4):
    """Block-wise workload at the size of the paper's largest four-view
    dataset (an L1 larva, 1640x1070x345, four views, Optimization II,
    lambda 0): blobs filling an ellipsoidal body (radius U[0, 1] of the
    semi-axes 0.4 dims), views at 90 deg steps about y, 21x21x31 PSFs
    (sigma_xy 1.0, sigma_z 3.5), Poisson in photon units.  The extents are
    not 5-smooth and y is beyond one transform: the volume is processed in
    blocks."""
    return make_problem(dims, n_blobs, [0.0, 90.0, 180.0, 270.0][:n_views], (21, 21, 31), 1.0, 3.5,
                        SEED_BASE + 5, variant=3, n_iter=10, shell=(0.0, 1.0))


def config5_theta(seed=SEED_BASE + 4):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    true = np.tile(np.array([1.2, 4.0]), (4, 1))
    start = true * rng.uniform(0.8, 1.2, size=true.shape)
    return true, start


def config5():
    """128^3, four views, 25^3 PSFs; the data use sigma (1.2, 4.0); the
    differentiated run starts from PSF widths perturbed by U[0.8, 1.2]."""
    return make_problem((128, 128, 128), 150, [0.0, 45.0, 90.0, 135.0], (25, 25, 25), 1.2, 4.0,
                        SEED_BASE + 4, variant=0, n_iter=8)
