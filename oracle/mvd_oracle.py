"""FP64 CPU oracle for the sequential multi-view deconvolution update.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct reference
that the GPU library is checked against.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the HIP library: no kernels, no headers, no
tables, no pre- or post-processing.

Paper: Preibisch et al., "Efficient Bayesian-based Multi-View Deconvolution"
(arXiv 1308.0730).  Every function below names the passage it follows.

Conventions (the paper is silent on them; each is a documented reading):
  * Arrays are C-ordered [z][y][x]; a volume of dims (nx, ny, nz) has numpy
    shape (nz, ny, nx).  A kernel of extents (kx, ky, kz) has shape (kz, ky, kx).
  * Kernels are centred at c = (k - 1) / 2 per axis; even extents get one
    trailing zero plane first so that every extent is odd.
  * "convolution" in the update is circular over the volume (the views are
    registered onto one periodic grid):  (f * K)[x] = sum_d K[c + d] f[x - d].
  * P* is P mirrored through its centre: P*[c + d] = P[c - d]
    (section "Integrating xi and x", which explains why the second
    convolution of eq. 15 uses the inverted kernel).
  * Scale s = mean of all views; psi^0 = s everywhere (eq. 15 text: a
    constant guess at the average intensity); eps = 1e-6 s guards the ratio;
    lambda' = lambda / s makes the Tikhonov weight dimensionless.
  * Tikhonov: the update solves lambda' t^2 + t = u, evaluated as
    t = 2u / (1 + sqrt(1 + 4 lambda' u)) (no cancellation).
  * Weights blend the step: psi <- psi + w (t - psi)  (section on partially
    overlapping data: w is the fraction of one RL step that is applied).

Parity status: every function here is pinned by tests that do not retype
it: tests/test_oracle_pins.py (brute-force direct convolution, explicit-matrix
EM/OSEM, fixed point, flux, non-negativity, closed forms, delta-kernel special
cases), tests/test_oracle_combined.py (combined updates: explicit EM, fixed
point, single-view and identical-view reductions), tests/test_oracle_weights.py
(normalisation modes and the contributing-view image on hand-counted cases),
tests/test_oracle_linear.py (linear boundary: the restricted-matrix EM step
weighted by the sensitivity with explicit matrices, fixed point, flux
identity, delta kernels), tests/test_oracle_blocked.py (block-wise form:
equal to the whole-volume update and to direct summation with a halo of
twice the kernel radius, different with a thinner one) and
tests/test_oracle_grad.py (adjoint identities,
central finite differences of the loss and of <gbar, psi_n>).  No function is
"parity unpinned".
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
from scipy import signal

RL, EFF, OPT1, OPT2 = 0, 1, 2, 3
VARIANT_NAMES = {RL: "rl", EFF: "eff", OPT1: "opt1", OPT2: "opt2"}

EPS_SCALE = 1e-6


# ---------------------------------------------------------------- kernels --

def normalize(P):
    """Probability constraint of eq. 3: a PSF integrates to one."""
    P = np.asarray(P, dtype=np.float64)
    s = P.sum()
    if not s > 0:
        raise ValueError("kernel sum must be positive")
    return P / s


def pad_odd(P):
    """Append one zero plane to every even extent (centre convention)."""
    P = np.asarray(P, dtype=np.float64)
    pads = [(0, 1 - (n % 2)) for n in P.shape]
    return np.pad(P, pads)


def mirror(P):
    """P*: the kernel inverted through its centre (eq. 51, mirrored kernels)."""
    return np.ascontiguousarray(P[::-1, ::-1, ::-1])


def prepare_psf(P):
    """Normalise (eq. 3) and make every extent odd."""
    return pad_odd(normalize(P))


def conv_full(a, b):
    """Full linear convolution of two small kernels (FP64 FFT; pinned against
    direct summation in the tests).

    Centre bookkeeping: if a is centred at ca and b at cb, the result is
    centred at ca + cb.
    """
    return signal.fftconvolve(a, b, mode="full")


def conv_full_direct(a, b):
    """Full linear convolution of two small kernels by direct summation."""
    return signal.convolve(a, b, mode="full", method="direct")


def crop_center(K, shape):
    """Window of `shape` (odd extents) around the centre of K (odd extents)."""
    sl = []
    for n, m in zip(K.shape, shape):
        c = (n - 1) // 2
        h = (m - 1) // 2
        if m > n:
            raise ValueError("crop larger than kernel")
        sl.append(slice(c - h, c + h + 1))
    return K[tuple(sl)]


def compound_kernel(psfs, v, variant):
    """Back-projection kernel of view v for each variant.

    RL   : P_v*                                  (eq. 51, sequential form of section 7)
    EFF  : P_v* . prod_{w != v} (P_v* * P_w * P_w*)   (eq. 220 / 222)
    OPT1 : P_v* . prod_{w != v} (P_v* * P_w)          (eq. 230, Optimization I)
    OPT2 : prod of N factors P_v*  = (P_v*)^N         (eq. 240, Optimization II)
    '*' is convolution, '.' the pointwise product.  Each factor is cropped to
    the window of P_v (exact: the product with P_v* vanishes outside it) and
    the result is normalised to sum one, as every kernel is a probability
    distribution (eq. 3).  With one view every variant reduces to P_v*.
    """
    P = [prepare_psf(p) for p in psfs]
    Pv_m = mirror(P[v])
    n = len(P)
    if variant == RL:
        return Pv_m.copy()
    if variant == OPT2:
        return normalize(Pv_m ** n)
    K = Pv_m.copy()
    for w in range(n):
        if w == v:
            continue
        f = conv_full(Pv_m, P[w])
        if variant == EFF:
            f = conv_full(f, mirror(P[w]))
        elif variant != OPT1:
            raise ValueError("unknown variant")
        K = K * crop_center(f, Pv_m.shape)
    return normalize(K)


# ------------------------------------------------------------ convolution --

def embed(K, shape):
    """Wrap-embed a centred odd kernel into a periodic grid: h[d mod n] = K[c + d]."""
    h = np.zeros(shape, dtype=np.float64)
    kz, ky, kx = K.shape
    cz, cy, cx = (kz - 1) // 2, (ky - 1) // 2, (kx - 1) // 2
    iz = (np.arange(kz) - cz) % shape[0]
    iy = (np.arange(ky) - cy) % shape[1]
    ix = (np.arange(kx) - cx) % shape[2]
    np.add.at(h, np.ix_(iz, iy, ix), K)
    return h


def circ_conv(f, K):
    """Circular convolution with a centred kernel via the FP64 FFT."""
    f = np.asarray(f, dtype=np.float64)
    H = sfft.rfftn(embed(K, f.shape), workers=-1)
    return sfft.irfftn(sfft.rfftn(f, workers=-1) * H, s=f.shape, workers=-1)


def circ_conv_direct(f, K):
    """Circular convolution by brute-force summation over the kernel support."""
    f = np.asarray(f, dtype=np.float64)
    kz, ky, kx = K.shape
    cz, cy, cx = (kz - 1) // 2, (ky - 1) // 2, (kx - 1) // 2
    out = np.zeros_like(f)
    for a in range(kz):
        for b in range(ky):
            for c in range(kx):
                k = K[a, b, c]
                if k != 0.0:
                    out += k * np.roll(f, shift=(a - cz, b - cy, c - cx), axis=(0, 1, 2))
    return out


# ----------------------------------------------------------------- update --

def tikhonov(u, lam_p):
    """MAP step for the Tikhonov prior: the t >= 0 solving lam' t^2 + t = u.

    The paper offers Tikhonov regularisation without printing its form
    (section on noise and regularisation); this is the reading documented in
    the module header, evaluated in the rationalised form.
    """
    if lam_p == 0.0:
        return u
    return 2.0 * u / (1.0 + np.sqrt(1.0 + 4.0 * lam_p * u))


def scale_of(views):
    """Mean intensity over all voxels of all views (psi^0 of eq. 15)."""
    return float(np.mean([np.mean(np.asarray(v, dtype=np.float64)) for v in views]))


def view_update(psi, phi, P, K, w=None, lam_p=0.0, eps=0.0, conv=circ_conv, stats=None):
    """One view's update of psi (section 7, one line of the sequential scheme).

    b = psi * P_v (expected view, eq. 1); q = phi / max(b, eps);
    c = q * K_v; u = psi . max(c, 0); t = T_lambda(u); psi <- psi + w (t - psi).
    """
    b = conv(psi, P)
    q = phi / np.maximum(b, eps)
    c = conv(q, K)
    u = psi * np.maximum(c, 0.0)
    t = tikhonov(u, lam_p)
    if stats is not None:
        stats["ratio_clamps"] = stats.get("ratio_clamps", 0) + int(np.count_nonzero(b < eps))
        stats["neg_clamps"] = stats.get("neg_clamps", 0) + int(np.count_nonzero(c < 0))
    if w is None:
        return t
    return psi + w * (t - psi)


OVERLAP_ONE, OVERLAP_MIN, OVERLAP_AVG, OVERLAP_USER = 0, 1, 2, 3


def contributing_views(weights):
    """Number of views with a non-zero weight at every voxel (the image the
    section on partially overlapping data offers for choosing the overlap)."""
    return np.sum([np.asarray(w, dtype=np.float64) > 0 for w in weights], axis=0).astype(np.float64)


def normalize_weights(weights, mode=OVERLAP_MIN, value=1.0):
    """Limit the summed weight of every voxel to an overlap number m
    (section on partially overlapping data): m = 1 (the safe choice), the
    minimal or the average number of contributing views over the voxels that
    any view covers, or a user value.  Where the sum s exceeds m every view's
    weight is scaled by m / s; weights are never increased."""
    w = [np.asarray(x, dtype=np.float64) for x in weights]
    count = contributing_views(w)
    covered = count > 0
    if mode == OVERLAP_ONE:
        m = 1.0
    elif mode == OVERLAP_MIN:
        m = float(count[covered].min()) if covered.any() else 1.0
    elif mode == OVERLAP_AVG:
        m = float(count[covered].mean()) if covered.any() else 1.0
    else:
        m = float(value)
    s = np.sum(w, axis=0)
    f = np.ones_like(s)
    over = s > m
    f[over] = m / s[over]
    return [x * f for x in w], m


GEOMETRIC, ARITHMETIC = 0, 1


def combined_update(psi, views, P, K, mean=GEOMETRIC, lam_p=0.0, eps=0.0, conv=circ_conv, stats=None):
    """One combined update of psi from all views at once (eq. 51).

    Every view's back-projected ratio c_v = (phi_v / max(psi * P_v, eps)) * K_v
    is taken from the same psi.  Eq. 51 multiplies them; the convergence
    proof (section on the proof for multiple views) normalises that product
    by the number of views with the |V|-th root, i.e. the geometric mean.
    The additive ML-EM derivation uses the arithmetic mean of the same
    factors instead.  Then u = psi . mean(max(c_v, 0)) and t = T_lambda(u).
    """
    n = len(views)
    acc = None
    for v in range(n):
        b = conv(psi, P[v])
        q = views[v] / np.maximum(b, eps)
        c = conv(q, K[v])
        if stats is not None:
            stats["ratio_clamps"] = stats.get("ratio_clamps", 0) + int(np.count_nonzero(b < eps))
            stats["neg_clamps"] = stats.get("neg_clamps", 0) + int(np.count_nonzero(c < 0))
        c = np.maximum(c, 0.0)
        if acc is None:
            acc = c.copy()
        elif mean == GEOMETRIC:
            acc = acc * c
        else:
            acc = acc + c
    g = acc ** (1.0 / n) if mean == GEOMETRIC else acc / n
    return tikhonov(psi * g, lam_p)


class Problem:
    """Inputs of one deconvolution: views, PSFs, optional weights, lambda."""

    def __init__(self, views, psfs, weights=None, lam=0.0):
        self.views = [np.asarray(v, dtype=np.float64) for v in views]
        self.psfs = [np.asarray(p, dtype=np.float64) for p in psfs]
        self.weights = None if weights is None else [np.asarray(w, dtype=np.float64) for w in weights]
        self.lam = float(lam)
        self.n = len(self.views)
        self.shape = self.views[0].shape
        self.s = scale_of(self.views)
        self.eps = EPS_SCALE * self.s
        self.lam_p = self.lam / self.s
        self.P = [prepare_psf(p) for p in self.psfs]
        self._K = {}

    def kernels(self, variant):
        if variant not in self._K:
            self._K[variant] = [compound_kernel(self.psfs, v, variant) for v in range(self.n)]
        return self._K[variant]

    def psi0(self):
        return np.full(self.shape, self.s, dtype=np.float64)

    def iterate(self, psi, n_iter, variant, conv=circ_conv, flux=None, stats=None):
        """n_iter iterations; one iteration applies every view once, in index
        order (section 7; an iteration is complete when all views have
        contributed once)."""
        K = self.kernels(variant)
        psi = np.array(psi, dtype=np.float64)
        for _ in range(n_iter):
            for v in range(self.n):
                w = None if self.weights is None else self.weights[v]
                psi = view_update(psi, self.views[v], self.P[v], K[v], w, self.lam_p,
                                  self.eps, conv=conv, stats=stats)
                if flux is not None:
                    flux.append(float(psi.sum()))
        return psi


    def iterate_combined(self, psi, n_iter, variant, mean=GEOMETRIC, conv=circ_conv, flux=None, stats=None):
        """n_iter combined updates (eq. 51): all views contribute to one
        update of psi per iteration.  Weights are a device of the sequential
        scheme (a fraction of each view's step) and are not used here."""
        if self.weights is not None:
            raise ValueError("combined updates take no weights")
        K = self.kernels(variant)
        psi = np.array(psi, dtype=np.float64)
        for _ in range(n_iter):
            psi = combined_update(psi, self.views, self.P, K, mean, self.lam_p, self.eps, conv=conv, stats=stats)
            if flux is not None:
                flux.append(float(psi.sum()))
        return psi


# ------------------------------------------------------ linear boundary --
#
# The views are known on the volume only; light from sources up to one PSF
# radius p outside it reaches it.  psi lives on the extended domain
# (n + 2p per axis, the volume at offset p); b = psi * P is evaluated on the
# volume (linear convolution).  Where a view has no data (outside the volume)
# its ratio is neutral, q = 1, and the back-projection c = q * K is taken over
# that extended ratio, so the update is the same as the circular one on the
# extended domain.  Written with the view's sensitivity N = 1_volume * K (the
# part of K's light a voxel sends into the volume) this step is
#     psi (c) = psi (1 - N + K^T q)  =  psi + N (psi K^T q / N - psi):
# the restricted-matrix EM step psi K^T q / N taken as the fraction N of a
# full step, the same device the paper uses for partially overlapping views
# (a weight is the fraction of one RL step applied at a voxel).  It has no
# constant of its own and never divides by N.  Weights apply on the volume
# and are 1 in the margin.


def margins(psfs):
    """Per-axis radius (z, y, x) of the largest prepared PSF."""
    shapes = [prepare_psf(p).shape for p in psfs]
    return tuple(max(k[a] for k in shapes) // 2 for a in range(3))


def pad_kernel(K, p):
    """Centre an odd kernel in a (2p+1)^3 box."""
    K = np.asarray(K, dtype=np.float64)
    pads = [((2 * p[a] + 1 - K.shape[a]) // 2,) * 2 for a in range(3)]
    return np.pad(K, pads)


def lin_blur(psi_e, P, p):
    """b on the volume: (psi * P)(x) = sum_d P[c + d] psi(x - d), psi given on
    the extended domain."""
    return signal.fftconvolve(psi_e, pad_kernel(P, p), mode="valid")


def lin_back(q, K, p):
    """Back-projection of a ratio given on the volume (zero elsewhere) onto
    the extended domain: sum_x K[c + (xi - x)] q(x)."""
    return signal.fftconvolve(q, pad_kernel(K, p), mode="full")


def sensitivity(n, K, p):
    """N = 1_volume * K on the extended domain: the part of K's light that a
    voxel sends into the volume."""
    return lin_back(np.ones(n), K, p)


def view_update_linear(psi_e, phi, P, K, p, w_e=None, lam_p=0.0, eps=0.0, stats=None):
    """One view-update with the linear boundary (see the block comment):
    b on the volume, q = phi / max(b, eps) there and 1 on a band of 2p around
    it (every ratio the extended domain's back-projection reaches), c = q * K
    on the extended domain, then the steps of the circular update."""
    b = lin_blur(psi_e, P, p)
    q = phi / np.maximum(b, eps)
    q_ext = np.pad(q, [(2 * a, 2 * a) for a in p], constant_values=1.0)
    c = signal.fftconvolve(q_ext, pad_kernel(K, p), mode="valid")
    if stats is not None:
        stats["ratio_clamps"] = stats.get("ratio_clamps", 0) + int(np.count_nonzero(b < eps))
        stats["neg_clamps"] = stats.get("neg_clamps", 0) + int(np.count_nonzero(c < 0))
    u = psi_e * np.maximum(c, 0.0)
    t = tikhonov(u, lam_p)
    if w_e is None:
        return t
    return psi_e + w_e * (t - psi_e)


class ProblemLinear(Problem):
    """A Problem deconvolved with the linear boundary."""

    def __init__(self, views, psfs, weights=None, lam=0.0):
        super().__init__(views, psfs, weights, lam)
        self.p = margins(self.psfs)
        n = self.shape
        self.shape_e = tuple(n[a] + 2 * self.p[a] for a in range(3))
        self.weights_e = None
        if self.weights is not None:
            self.weights_e = [np.pad(w, [(q, q) for q in self.p], constant_values=1.0) for w in self.weights]

    def psi0(self):
        return np.full(self.shape_e, self.s, dtype=np.float64)

    def interior(self, psi_e):
        pz, py, px = self.p
        n = self.shape
        return psi_e[pz:pz + n[0], py:py + n[1], px:px + n[2]]

    def iterate(self, psi_e, n_iter, variant, flux=None, stats=None):
        K = self.kernels(variant)
        psi = np.array(psi_e, dtype=np.float64)
        for _ in range(n_iter):
            for v in range(self.n):
                w = None if self.weights_e is None else self.weights_e[v]
                psi = view_update_linear(psi, self.views[v], self.P[v], K[v], self.p, w, self.lam_p, self.eps,
                                         stats=stats)
                if flux is not None:
                    flux.append(float(psi.sum()))
        return psi


# ------------------------------------------------------- block-wise form --
#
# The paper processes a volume "in blocks to reduce the memory requirements"
# (main text; implementation section: copying and pasting blocks).  Here the
# volume (any extents, circular boundary: one period of a periodic grid) is
# cut into near-equal blocks; for each view-update every block takes psi,
# phi_v and w_v on its own computation grid, the block plus a halo wrapped
# periodically from the volume, runs the circular update on that grid and
# pastes its own voxels back.  Every block of one view-update reads the same
# psi.  A halo of at least twice the kernel radius on each side leaves the
# pasted voxels equal to the whole-volume update (the blur needs psi within
# one radius of a ratio voxel, the back-projection the ratio within one
# radius of an updated voxel); a thinner halo lets the grid's wrap-around
# reach them.

def block_layout(n, tiles):
    """(origin, extent) of `tiles` near-equal blocks along an axis of n voxels."""
    o = [(k * n) // tiles for k in range(tiles + 1)]
    return [(o[k], o[k + 1] - o[k]) for k in range(tiles)]


def wrap_window(f, start, shape):
    """f on the box start + [0, shape) per axis, read periodically."""
    idx = [np.arange(a, a + m) % n for a, m, n in zip(start, shape, f.shape)]
    return f[np.ix_(*idx)]


def view_update_blocked(psi, phi, P, K, tiles, halo, grid, w=None, lam_p=0.0, eps=0.0, conv=circ_conv):
    """One view-update computed block by block (see the block comment).
    tiles: blocks per axis (z, y, x); halo: voxels of the grid before a
    block's first voxel, per axis; grid: extents of every block's
    computation grid, at least the largest block plus twice the halo."""
    psi = np.asarray(psi, dtype=np.float64)
    out = np.empty_like(psi)
    lay = [block_layout(psi.shape[a], tiles[a]) for a in range(3)]
    for oz, ez in lay[0]:
        for oy, ey in lay[1]:
            for ox, ex in lay[2]:
                if ez + 2 * halo[0] > grid[0] or ey + 2 * halo[1] > grid[1] or ex + 2 * halo[2] > grid[2]:
                    raise ValueError("the grid must hold a block and its halo on both sides")
                start = (oz - halo[0], oy - halo[1], ox - halo[2])
                g_w = None if w is None else wrap_window(w, start, grid)
                g_new = view_update(wrap_window(psi, start, grid), wrap_window(phi, start, grid), P, K, g_w,
                                    lam_p, eps, conv=conv)
                out[oz:oz + ez, oy:oy + ey, ox:ox + ex] = g_new[halo[0]:halo[0] + ez, halo[1]:halo[1] + ey,
                                                                halo[2]:halo[2] + ex]
    return out


def iterate_blocked(pb, psi, n_iter, variant, tiles, halo, grid):
    """n_iter sequential iterations of Problem pb computed block by block."""
    K = pb.kernels(variant)
    psi = np.array(psi, dtype=np.float64)
    for _ in range(n_iter):
        for v in range(pb.n):
            w = None if pb.weights is None else pb.weights[v]
            psi = view_update_blocked(psi, pb.views[v], pb.P[v], K[v], tiles, halo, grid, w, pb.lam_p, pb.eps)
    return psi


def run(views, psfs, n_iter, variant, weights=None, lam=0.0, psi0=None, trajectory=False):
    """Deconvolve from psi0 (default: flat at the mean); optionally return
    the estimate after every iteration."""
    pb = Problem(views, psfs, weights, lam)
    psi = pb.psi0() if psi0 is None else np.asarray(psi0, dtype=np.float64)
    traj = []
    for _ in range(n_iter):
        psi = pb.iterate(psi, 1, variant)
        if trajectory:
            traj.append(psi.copy())
    return (psi, traj) if trajectory else psi


# ---------------------------------------------------------------- metrics --

def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------ differentiated form --
#
# Loss of the unrolled run: L = sum_v sum_x (psi^T (x) P_v - phi_v)^2, with
# psi^T after n_iter sequential iterations of the RL update from psi^0.
# Gradients with respect to psi^0 and to the raw PSF inputs (through the
# normalisation of eq. 3) by reverse-mode differentiation of every step; the
# clamps max(b, eps) and max(c, 0) contribute zero derivative where active.
# Pinned by central finite differences and adjoint dot-product tests.

def circ_corr_window(f, g, shape):
    """r[c + d] = sum_x f(x) g(x - d) for d in the centred window `shape`
    (odd extents): the adjoint of f = g (x) K with respect to K."""
    F = sfft.rfftn(np.asarray(f, dtype=np.float64), workers=-1)
    G = sfft.rfftn(np.asarray(g, dtype=np.float64), workers=-1)
    r = sfft.irfftn(F * np.conj(G), s=f.shape, workers=-1)
    kz, ky, kx = shape
    iz = (np.arange(kz) - (kz - 1) // 2) % f.shape[0]
    iy = (np.arange(ky) - (ky - 1) // 2) % f.shape[1]
    ix = (np.arange(kx) - (kx - 1) // 2) % f.shape[2]
    return r[np.ix_(iz, iy, ix)]


def compound_kernel_vjp(P, v, variant, Kbar):
    """Adjoint of the compound kernel construction (see compound_kernel):
    given Kbar = dL/dK_v on K_v's window, returns dL/dP_w for every
    prepared (normalised, odd) PSF P_w.  The steps of the construction are
    taken backwards: the normalisation K = U / sum U, the pointwise product
    U = P_v* . prod_w A_w, each factor A_w = crop(P_v* * P_w * P_w*) (EFF) or
    crop(P_v* * P_w) (OPT1), the full linear convolutions (adjoint: 'valid'
    correlations with the other operand) and the mirror."""
    n = len(P)
    Kbar = np.asarray(Kbar, dtype=np.float64)
    gP = [np.zeros_like(p) for p in P]
    Pv_m = mirror(P[v])
    if variant == RL or n == 1:
        gP[v] += mirror(Kbar)
        return gP
    if variant == OPT2:
        U = Pv_m ** n
        Ubar = (Kbar - np.sum(Kbar * U) / U.sum()) / U.sum()
        gP[v] += mirror(Ubar * n * Pv_m ** (n - 1))
        return gP
    # forward, keeping the pieces
    g1, full, A = {}, {}, {}
    for w in range(n):
        if w == v:
            continue
        g1[w] = conv_full(Pv_m, P[w])
        full[w] = conv_full(g1[w], mirror(P[w])) if variant == EFF else g1[w]
        A[w] = crop_center(full[w], Pv_m.shape)
    U = Pv_m.copy()
    for w in A:
        U = U * A[w]
    S = U.sum()
    K = U / S
    # K = U / S
    Ubar = (Kbar - np.sum(Kbar * K)) / S
    # U = Pv_m . prod A_w
    Pv_m_bar = Ubar * np.prod([A[w] for w in A], axis=0)
    for w in A:
        others = np.prod([A[u] for u in A if u != w], axis=0) if len(A) > 1 else 1.0
        Abar = Ubar * Pv_m * others
        # A = crop(full): the adjoint pads into the full support
        fbar = np.zeros_like(full[w])
        pads = [((nf - na) // 2) for nf, na in zip(full[w].shape, Abar.shape)]
        fbar[pads[0]:pads[0] + Abar.shape[0], pads[1]:pads[1] + Abar.shape[1],
             pads[2]:pads[2] + Abar.shape[2]] = Abar
        if variant == EFF:
            # full = g1 * mirror(P_w)
            g1bar = signal.correlate(fbar, mirror(P[w]), mode="valid", method="fft")
            gP[w] += mirror(signal.correlate(fbar, g1[w], mode="valid", method="fft"))
        else:
            g1bar = fbar
        # g1 = Pv_m * P_w
        Pv_m_bar = Pv_m_bar + signal.correlate(g1bar, P[w], mode="valid", method="fft")
        gP[w] += signal.correlate(g1bar, Pv_m, mode="valid", method="fft")
    gP[v] += mirror(Pv_m_bar)
    return gP


def loss_value(psi, views, P):
    return float(sum(np.sum((circ_conv(psi, p) - np.asarray(phi, np.float64)) ** 2) for p, phi in zip(P, views)))


def _taped_run(pb, n_iter, psi0, variant=RL):
    """The sequential run (back-projection kernels K_v of the variant)
    keeping every view-update's intermediates for the reverse sweep."""
    P = pb.P
    K = pb.kernels(variant)
    psi = np.asarray(psi0, dtype=np.float64).copy()
    tape = []
    for _ in range(n_iter):
        for v in range(pb.n):
            w = None if pb.weights is None else pb.weights[v]
            b = circ_conv(psi, P[v])
            q = pb.views[v] / np.maximum(b, pb.eps)
            c = circ_conv(q, K[v])
            u = psi * np.maximum(c, 0.0)
            t = tikhonov(u, pb.lam_p)
            new = t if w is None else psi + w * (t - psi)
            tape.append((v, psi, b, q, c, u, w))
            psi = new
    return psi, tape


def loss_and_grad(views, psfs, n_iter, psi0, weights=None, lam=0.0, variant=RL):
    """Loss and its gradients for the sequential update with the variant's
    back-projection kernels (RL: K_v = P_v*; the compound kernels depend on
    every PSF).

    Returns (L, dL/dpsi0, [dL/dpsf_v]) with each PSF gradient on the raw
    input extents of psfs[v]."""
    pb = Problem(views, psfs, weights, lam)
    P = pb.P
    N = pb.n
    psi, tape = _taped_run(pb, n_iter, psi0, variant)
    L = 0.0
    gpsi = np.zeros_like(psi)
    gP = [np.zeros_like(p) for p in P]
    for v in range(N):
        r = circ_conv(psi, P[v]) - pb.views[v]
        L += float(np.sum(r * r))
        gpsi += circ_conv(2.0 * r, mirror(P[v]))
        gP[v] += circ_corr_window(2.0 * r, psi, P[v].shape)
    gpsi, out = _reverse(pb, psfs, tape, gpsi, gP, variant)
    return L, gpsi, out


def vjp(views, psfs, n_iter, psi0, gbar, weights=None, lam=0.0, variant=RL):
    """Vector-Jacobian product of the unrolled run: for a given gbar (the
    gradient of some scalar with respect to psi_n), the gradients of
    <gbar, psi_n> with respect to psi0 and to the raw PSF values.

    Returns (psi_n, d/dpsi0, [d/dpsf_v])."""
    pb = Problem(views, psfs, weights, lam)
    psi, tape = _taped_run(pb, n_iter, psi0, variant)
    gP = [np.zeros_like(p) for p in pb.P]
    gpsi, out = _reverse(pb, psfs, tape, np.asarray(gbar, dtype=np.float64).copy(), gP, variant)
    return psi, gpsi, out


def _reverse(pb, psfs, tape, gpsi, gP, variant=RL):
    """Reverse sweep over the taped view-updates from the seed gpsi = d/dpsi_n
    (and PSF gradients gP accumulated so far, on the padded odd boxes); the
    gradients of the back-projection kernels go through the compound kernel
    construction (compound_kernel_vjp), then everything through the
    normalisation of eq. 3 onto the raw PSF extents."""
    P = pb.P
    N = pb.n
    K = pb.kernels(variant)
    gK = [np.zeros_like(k) for k in K]
    for (v, psi_in, b, q, c, u, w) in reversed(tape):
        g = gpsi
        tbar = g if w is None else w * g
        dT = 1.0 if pb.lam_p == 0.0 else 1.0 / np.sqrt(1.0 + 4.0 * pb.lam_p * u)
        ubar = tbar * dT
        gdirect = ubar * np.maximum(c, 0.0) + (0.0 if w is None else (1.0 - w) * g)
        cbar = ubar * psi_in * (c > 0)
        # c = q (x) K_v: the adjoint in q is a convolution with K_v*, in the
        # kernel K_v[c + j] gets sum_x cbar(x) q(x - j)
        qbar = circ_conv(cbar, mirror(K[v]))
        gK[v] += circ_corr_window(cbar, q, K[v].shape)
        bbar = np.where(b > pb.eps, -qbar * q / b, 0.0)
        gP[v] += circ_corr_window(bbar, psi_in, P[v].shape)
        gpsi = gdirect + circ_conv(bbar, mirror(P[v]))
    # the back-projection kernels are functions of the PSFs
    for v in range(N):
        for w, g in enumerate(compound_kernel_vjp(P, v, variant, gK[v])):
            gP[w] += g
    # through the normalisation P = G / sum(G) and the odd padding
    out = []
    for v in range(N):
        G = np.asarray(psfs[v], dtype=np.float64)
        S = G.sum()
        gpad = gP[v]
        gn = (gpad - np.sum(gpad * P[v])) / S
        out.append(gn[:G.shape[0], :G.shape[1], :G.shape[2]])
    return gpsi, out


def loss_of(views, psfs, n_iter, psi0, weights=None, lam=0.0, variant=RL):
    """The loss alone (forward), for finite differences."""
    pb = Problem(views, psfs, weights, lam)
    psi = pb.iterate(np.asarray(psi0, dtype=np.float64), n_iter, variant)
    return loss_value(psi, pb.views, pb.P)


# ------------------------------------------------- sampled view-update --------

def _periodic_box(f, center, half):
    """f on the box center +- half (per axis, periodic)."""
    idx = [(np.arange(c - h, c + h + 1)) % n for c, h, n in zip(center, half, f.shape)]
    return f[np.ix_(*idx)]


def view_update_at(psi, phi, P, K, points, w=None, lam_p=0.0, eps=0.0):
    """The result of view_update at the given voxels (z, y, x), each computed
    on its own from the windows it depends on: c at x needs q on K's window
    around x, which needs b = psi (x) P on that window, which needs psi on a
    box of both windows.  Same arithmetic as view_update, evaluated locally
    (for volumes too large for the whole-volume oracle)."""
    hk = [(n - 1) // 2 for n in K.shape]
    hp = [(n - 1) // 2 for n in P.shape]
    out = []
    for pt in points:
        # windows are taken first and converted to FP64 (the inputs may be
        # large float32 volumes)
        box = _periodic_box(psi, pt, [a + b for a, b in zip(hk, hp)]).astype(np.float64)
        # b on K's window around pt: valid convolution of the box with P
        b = signal.fftconvolve(box, P, mode="valid")
        q = _periodic_box(phi, pt, hk).astype(np.float64) / np.maximum(b, eps)
        # c(pt) = sum_d K[c + d] q(pt - d): q's window is indexed pt + e, so K flips
        c = float(np.sum(K[::-1, ::-1, ::-1] * q))
        p0 = float(psi[tuple(pt)])
        u = p0 * max(c, 0.0)
        t = float(tikhonov(np.array(u), lam_p))
        out.append(t if w is None else p0 + float(w[tuple(pt)]) * (t - p0))
    return np.array(out)
