"""Python binding of libmvd (ctypes over include/mvd.h).

Argument marshalling only: every step of the deconvolution runs in the HIP
library.  PyTorch provides device memory (the library allocates through
torch's caching allocator) and the stream the work is ordered on.  Importing
this module raises if the built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime the library shares

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmvd.so")

MVD_OK, MVD_EINVAL, MVD_ENOMEM, MVD_EDEVICE, MVD_ENONFINITE, MVD_ESTATE = 0, -1, -2, -3, -4, -5
RL, EFF, OPT1, OPT2 = 0, 1, 2, 3
MEM_HOST, MEM_DEVICE = 0, 1
MAX_VIEWS = 64
VARIANTS = {"rl": RL, "eff": EFF, "opt1": OPT1, "opt2": OPT2}


class Problem(C.Structure):
    _fields_ = [("n_views", C.c_int), ("dims", C.c_int * 3), ("views", C.POINTER(C.c_void_p)),
                ("psfs", C.POINTER(C.c_void_p)), ("psf_dims", C.POINTER(C.c_int)),
                ("weights", C.POINTER(C.c_void_p)), ("mem_kind", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("lam", C.c_double), ("eps_scale", C.c_double), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("use_graphs", C.c_int), ("tile_config", C.c_int), ("boundary", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("n_views", C.c_int), ("n_blocks", C.c_int),
                ("scale", C.c_double), ("flux", C.c_double * MAX_VIEWS), ("ratio_clamps", C.c_int64),
                ("neg_clamps", C.c_int64), ("nonfinite", C.c_int)]


class MVDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mvd error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmvd.so (built in-tree by paper_1308_0730_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python paper_1308_0730_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.mvd_create.argtypes = [C.POINTER(H), C.POINTER(Problem), C.POINTER(Options)]
    L.mvd_create_batch.argtypes = [C.POINTER(H), C.c_int, C.POINTER(Problem), C.POINTER(Options)]
    L.mvd_iterate.argtypes = [H, C.c_int, C.c_int]
    L.mvd_iterate_combined.argtypes = [H, C.c_int, C.c_int, C.c_int]
    L.mvd_grid_dims.argtypes = [H, C.c_int, C.POINTER(C.c_int)]
    L.mvd_normalize_weights.argtypes = [H, C.c_int, C.c_double, C.POINTER(C.c_double)]
    L.mvd_contributing_views.argtypes = [H, C.c_void_p, C.c_int, C.c_int]
    L.mvd_get_estimate.argtypes = [H, C.c_void_p, C.c_int, C.c_int]
    L.mvd_set_estimate.argtypes = [H, C.c_void_p, C.c_int, C.c_int]
    L.mvd_stats.argtypes = [H, C.POINTER(Stats)]
    L.mvd_view_update.argtypes = [H, C.c_int, C.c_int]
    L.mvd_loss_grad.argtypes = [H, C.c_int, C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                C.POINTER(C.c_void_p), C.c_void_p, C.c_int]
    L.mvd_backward.argtypes = [H, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                               C.POINTER(C.c_void_p), C.c_void_p, C.c_int]
    L.mvd_set_psfs.argtypes = [H, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.c_int]
    L.mvd_set_tiles.argtypes = [H, C.c_int, C.c_int, C.c_int]
    L.mvd_get_tiles.argtypes = [H, C.POINTER(C.c_int)]
    L.mvd_tile_candidates.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int]
    L.mvd_tile_shape.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)]
    L.mvd_profile.argtypes = [H, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.mvd_synchronize.argtypes = [H]
    L.mvd_destroy.argtypes = [H]
    L.mvd_last_error.argtypes = [H]
    L.mvd_last_error.restype = C.c_char_p
    L.mvd_compound_kernel.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.c_int, C.c_int,
                                      C.c_void_p, C.POINTER(C.c_int)]
    L.mvd_compound_kernel_vjp.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.c_int, C.c_int,
                                          C.c_void_p, C.POINTER(C.c_void_p)]
    L.mvd_kernel_spectrum.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_void_p, C.c_void_p]
    L.mvd_create_blocked.argtypes = [C.POINTER(H), C.POINTER(Problem), C.POINTER(Options), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]
    L.mvd_forward_recorded.argtypes = [H, C.c_int, C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_int64)]
    L.mvd_backward_recorded.argtypes = [H, C.c_int64, C.c_void_p, C.c_int, C.POINTER(C.c_void_p), C.c_void_p,
                                        C.c_int]
    L.mvd_set_schedule.argtypes = [H, C.c_int]
    L.mvd_get_schedule.argtypes = [H]
    L.mvd_blocking.argtypes = [H, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.mvd_iterate_noalloc.argtypes = [C.POINTER(Problem), C.POINTER(Options), C.c_void_p, C.c_int, C.c_int,
                                      C.c_void_p]
    L.mvd_version.restype = C.c_char_p
    for name in ("mvd_create", "mvd_create_batch", "mvd_iterate", "mvd_iterate_combined", "mvd_grid_dims",
                 "mvd_normalize_weights",
                 "mvd_contributing_views", "mvd_get_estimate",
                 "mvd_set_estimate",
                 "mvd_stats", "mvd_synchronize", "mvd_destroy", "mvd_compound_kernel", "mvd_kernel_spectrum",
                 "mvd_view_update", "mvd_profile", "mvd_set_tiles", "mvd_get_tiles", "mvd_tile_candidates",
                 "mvd_tile_shape", "mvd_loss_grad", "mvd_backward", "mvd_set_psfs", "mvd_iterate_noalloc",
                 "mvd_create_blocked", "mvd_blocking", "mvd_set_schedule", "mvd_get_schedule",
                 "mvd_forward_recorded", "mvd_backward_recorded", "mvd_compound_kernel_vjp"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc, h=None):
    if rc != MVD_OK:
        raise MVDError(rc, lib().mvd_last_error(h).decode())


def _variant(v):
    return VARIANTS[v.lower()] if isinstance(v, str) else int(v)


MEANS = {"geometric": 0, "arithmetic": 1}
OVERLAPS = {"one": 0, "min": 1, "avg": 2, "user": 3}


def _mean(m):
    return MEANS[m.lower()] if isinstance(m, str) else int(m)


def _ptr(x):
    return x.data_ptr() if isinstance(x, torch.Tensor) else x.ctypes.data


class _Marshalled:
    """Keeps the arrays of one problem alive while the library copies them."""

    def __init__(self, views, psfs, weights, device, on_device):
        def conv(a):
            if on_device:
                t = a if isinstance(a, torch.Tensor) else torch.from_numpy(
                    np.ascontiguousarray(np.asarray(a, np.float32)))
                return t.detach().to(device=device, dtype=torch.float32).contiguous()
            if isinstance(a, torch.Tensor):
                a = a.detach().cpu().numpy()
            return np.ascontiguousarray(np.asarray(a, dtype=np.float32))

        self.views = [conv(v) for v in views]
        self.psfs = [conv(p) for p in psfs]
        self.weights = None if weights is None else [conv(w) for w in weights]
        n = len(self.views)
        if len(self.psfs) != n or (self.weights is not None and len(self.weights) != n):
            raise ValueError("views, psfs and weights need one entry per view")
        shape = tuple(self.views[0].shape)
        if len(shape) != 3:
            raise ValueError("views are 3-D arrays (nz, ny, nx)")
        self.dims = (shape[2], shape[1], shape[0])
        for v in self.views:
            if tuple(v.shape) != shape:
                raise ValueError("every view has the volume's shape")
        for p in self.psfs:
            if len(p.shape) != 3:
                raise ValueError("PSFs are 3-D arrays (kz, ky, kx)")
        if self.weights is not None:
            for w in self.weights:
                if tuple(w.shape) != shape:
                    raise ValueError("weights have the volume's shape")
        self._v = (C.c_void_p * n)(*[_ptr(v) for v in self.views])
        self._p = (C.c_void_p * n)(*[_ptr(p) for p in self.psfs])
        self._k = (C.c_int * (3 * n))(*sum([[p.shape[2], p.shape[1], p.shape[0]] for p in self.psfs], []))
        self._w = None if self.weights is None else (C.c_void_p * n)(*[_ptr(w) for w in self.weights])
        self.problem = Problem(n, (C.c_int * 3)(*self.dims), C.cast(self._v, C.POINTER(C.c_void_p)),
                               C.cast(self._p, C.POINTER(C.c_void_p)), C.cast(self._k, C.POINTER(C.c_int)),
                               None if self._w is None else C.cast(self._w, C.POINTER(C.c_void_p)),
                               MEM_DEVICE if on_device else MEM_HOST)


NOALLOC_SCRATCH_BYTES = 64 << 20


def iterate_noalloc(views, psfs, n, variant="eff", weights=None, lam=0.0, eps_scale=0.0, psi0=None, out=None,
                    boundary="circular", tile_config=0, device=None):
    """n iterations on one volume through mvd_iterate_noalloc: the library
    allocates nothing (its buffers live in a static array of
    NOALLOC_SCRATCH_BYTES per GPU).  Inputs as for Deconvolver; psi0 (None:
    flat start) and out are CUDA tensors of the volume's shape (out is created
    when None: that allocation is the caller's).  Returns out."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    on_device = any(isinstance(v, torch.Tensor) and v.is_cuda for v in views)
    stream = torch.cuda.current_stream(dev)
    opts = Options(float(lam), float(eps_scale), C.c_void_p(stream.cuda_stream), ALLOC_FN(), FREE_FN(), None, 0,
                   int(tile_config), {"circular": 0, "linear": 1}[boundary] if isinstance(boundary, str)
                   else int(boundary))
    with torch.cuda.device(dev):
        m = _Marshalled(views, psfs, weights, dev, on_device)
        nx, ny, nz = m.dims
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
        for name, t in (("out", out), ("psi0", psi0)):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
                                  or tuple(t.shape) != (nz, ny, nx) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {(nz, ny, nx)}")
        rc = lib().mvd_iterate_noalloc(C.byref(m.problem), C.byref(opts),
                                       None if psi0 is None else C.c_void_p(psi0.data_ptr()), int(n),
                                       _variant(variant), C.c_void_p(out.data_ptr()))
    _check(rc)
    return out


class Deconvolver:
    """Sequential multi-view deconvolution of one volume or a batch of blocks.

    Deconvolver(views, psfs, weights=None, lam=0.0)              plain form
    Deconvolver.batch([(views, psfs, weights), ...], lam=0.0)    batched form
    Deconvolver.blocked(views, psfs, weights, tiles, halo)       block-wise form

    Volumes are (nz, ny, nx) float32; PSFs (kz, ky, kx).  Inputs may be numpy
    arrays (copied from host memory) or CUDA tensors (device memory).
    """

    def __init__(self, views=None, psfs=None, weights=None, lam=0.0, eps_scale=0.0, use_graphs=True,
                 tile_config=0, device=None, boundary="circular", _blocks=None, _blocking=None):
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        self._bufs = {}
        dev = self.device

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
            except RuntimeError:
                return None
            self._bufs[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self._bufs.pop(ptr, None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.stream = torch.cuda.current_stream(dev)
        opts = Options(float(lam), float(eps_scale), C.c_void_p(self.stream.cuda_stream), self._alloc_cb,
                       self._free_cb, None, 1 if use_graphs else 0, int(tile_config),
                       {"circular": 0, "linear": 1}[boundary] if isinstance(boundary, str) else int(boundary))
        blocks = _blocks if _blocks is not None else [(views, psfs, weights)]
        on_device = any(isinstance(v, torch.Tensor) and v.is_cuda for b in blocks for v in b[0])
        with torch.cuda.device(dev):
            ms = [_Marshalled(v, p, w, dev, on_device) for (v, p, w) in blocks]
            arr = (Problem * len(ms))(*[m.problem for m in ms])
            h = C.c_void_p()
            if _blocking is None:
                rc = lib().mvd_create_batch(C.byref(h), len(ms), arr, C.byref(opts))
            else:
                tiles, halo = _blocking
                t = None if tiles is None else (C.c_int * 3)(*tiles)
                hl = None if halo is None else (C.c_int * 3)(*halo)
                rc = lib().mvd_create_blocked(C.byref(h), arr, C.byref(opts), t, hl)
        if rc != MVD_OK:
            self._h = None
            raise MVDError(rc, lib().mvd_last_error(None).decode())
        self._h = h
        self._psf_shapes = [tuple(p.shape) for p in ms[0].psfs]
        self.dims = [m.dims for m in ms]
        self.n_views = len(ms[0].views)
        self.n_blocks = len(ms)

    @classmethod
    def batch(cls, blocks, **kw):
        return cls(_blocks=[(b[0], b[1], b[2] if len(b) > 2 else None) for b in blocks], **kw)

    @classmethod
    def blocked(cls, views, psfs, weights=None, tiles=None, halo=None, **kw):
        """Block-wise form: the volume (any extents) in blocks per axis
        (x, y, z) (None or 0 on an axis: as few as the transform lengths
        allow), each with `halo` voxels per side (None: twice the largest PSF
        radius, the exact choice)."""
        return cls(views, psfs, weights, _blocking=(tiles, halo), **kw)

    def blocking(self):
        """(tiles, halo, volume dims), each (x, y, z)."""
        t, h, d = (C.c_int * 3)(), (C.c_int * 3)(), (C.c_int * 3)()
        _check(lib().mvd_blocking(self._h, t, h, d), self._h)
        return tuple(t), tuple(h), tuple(d)

    def iterate(self, n, variant="eff"):
        _check(lib().mvd_iterate(self._h, int(n), _variant(variant)), self._h)
        return self

    def iterate_combined(self, n, variant="rl", mean="geometric"):
        """n combined updates (eq. 51): every view's factor from the same psi,
        merged by the geometric or the arithmetic mean."""
        _check(lib().mvd_iterate_combined(self._h, int(n), _variant(variant), _mean(mean)), self._h)
        return self

    def normalize_weights(self, mode="min", value=0.0):
        """Limit every voxel's summed weight to the overlap number (1, the
        minimal or average number of contributing views, or `value`); returns
        the number used per block."""
        m = (C.c_double * self.n_blocks)()
        mode = OVERLAPS[mode] if isinstance(mode, str) else int(mode)
        _check(lib().mvd_normalize_weights(self._h, mode, float(value), m), self._h)
        return list(m)

    def contributing_views(self, block=0):
        """Number of views with a non-zero weight at every voxel (CUDA tensor)."""
        nx, ny, nz = self.dims[block]
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device)
        _check(lib().mvd_contributing_views(self._h, C.c_void_p(out.data_ptr()), MEM_DEVICE, block), self._h)
        return out

    def view_update(self, view, variant="eff"):
        """One view-update (one line of the sequential scheme)."""
        _check(lib().mvd_view_update(self._h, int(view), _variant(variant)), self._h)
        return self

    PASS_NAMES = ("y_forward", "y_inverse", "z_product", "x_ratio", "x_update")

    def profile(self, n, variant="eff"):
        """Run n iterations with per-launch HIP-event timing; returns
        {pass: (mean ms, launches)}."""
        ms = (C.c_double * 5)()
        calls = (C.c_int * 5)()
        _check(lib().mvd_profile(self._h, int(n), _variant(variant), ms, calls), self._h)
        return {k: (ms[i], calls[i]) for i, k in enumerate(self.PASS_NAMES)}

    def set_psfs(self, psfs):
        """Replace the PSFs (host arrays); their spectra are recomputed."""
        ps = [np.ascontiguousarray(np.asarray(p.detach().cpu() if isinstance(p, torch.Tensor) else p,
                                              np.float32)) for p in psfs]
        ptrs = (C.c_void_p * len(ps))(*[p.ctypes.data for p in ps])
        dims = (C.c_int * (3 * len(ps)))(*sum([[p.shape[2], p.shape[1], p.shape[0]] for p in ps], []))
        _check(lib().mvd_set_psfs(self._h, C.cast(ptrs, C.POINTER(C.c_void_p)), dims, MEM_HOST), self._h)
        self._psf_shapes = [p.shape for p in ps]
        return self

    def loss_grad(self, n, psi0=None, grad_psf=True, grad_psi0=True, psf_shapes=None, variant="rl"):
        """Loss sum_v |psi_n (x) P_v - phi_v|^2 after n RL iterations from psi0
        (None: flat start) and, optionally, its gradients: a list of float64
        arrays shaped like the PSFs, and a CUDA tensor shaped like the volume.
        Returns (loss, grad_psfs or None, grad_psi0 or None)."""
        src, gps, gp_ptrs, gpsi = self._grad_buffers(psi0, grad_psf, grad_psi0, psf_shapes)
        loss = C.c_double()
        rc = lib().mvd_loss_grad(self._h, int(n), _variant(variant), None if src is None else C.c_void_p(src.data_ptr()), MEM_DEVICE,
                                 C.byref(loss), _ptr_array(gp_ptrs),
                                 None if gpsi is None else C.c_void_p(gpsi.data_ptr()), MEM_DEVICE)
        _check(rc, self._h)
        return loss.value, gps, gpsi

    def backward(self, n, psi0, grad_psi_n, grad_psf=True, grad_psi0=True, psf_shapes=None, variant="rl"):
        """Vector-Jacobian product of n RL iterations from psi0 (None: flat
        start): for grad_psi_n = dL/dpsi_n of any scalar L, returns
        (dL/dpsf list of float64 arrays or None, dL/dpsi0 CUDA tensor or None).
        Leaves the estimate at psi_n."""
        nx, ny, nz = self.dims[0]
        src, gps, gp_ptrs, gpsi = self._grad_buffers(psi0, grad_psf, grad_psi0, psf_shapes)
        g = grad_psi_n.detach().to(self.device, torch.float32).contiguous() if isinstance(grad_psi_n, torch.Tensor) \
            else torch.from_numpy(np.ascontiguousarray(np.asarray(grad_psi_n, np.float32))).to(self.device)
        if tuple(g.shape) != (nz, ny, nx):
            raise ValueError(f"grad_psi_n has shape {tuple(g.shape)}, expected {(nz, ny, nx)}")
        rc = lib().mvd_backward(self._h, int(n), _variant(variant), None if src is None else C.c_void_p(src.data_ptr()), MEM_DEVICE,
                                C.c_void_p(g.data_ptr()), MEM_DEVICE, _ptr_array(gp_ptrs),
                                None if gpsi is None else C.c_void_p(gpsi.data_ptr()), MEM_DEVICE)
        _check(rc, self._h)
        return gps, gpsi

    def forward_recorded(self, n, psi0=None, variant="rl"):
        """n RL iterations from psi0 (None: flat start) with one checkpoint
        per iteration; returns (psi_n as a CUDA tensor, token of the
        recorded run for backward_recorded)."""
        src, _, _, _ = self._grad_buffers(psi0, False, False, None)
        tok = C.c_int64()
        rc = lib().mvd_forward_recorded(self._h, int(n), _variant(variant), None if src is None else C.c_void_p(src.data_ptr()),
                                        MEM_DEVICE, C.byref(tok))
        _check(rc, self._h)
        return self.estimate(), tok.value

    def backward_recorded(self, token, grad_psi_n, grad_psf=True, grad_psi0=True, psf_shapes=None):
        """Vector-Jacobian product over the run recorded with `token`:
        (dL/dpsf list of float64 arrays or None, dL/dpsi0 CUDA tensor or
        None).  MVDError(MVD_ESTATE) if a later call changed the estimate,
        PSFs or weights."""
        nx, ny, nz = self.dims[0]
        _, gps, gp_ptrs, gpsi = self._grad_buffers(None, grad_psf, grad_psi0, psf_shapes)
        g = grad_psi_n.detach().to(self.device, torch.float32).contiguous() if isinstance(grad_psi_n, torch.Tensor) \
            else torch.from_numpy(np.ascontiguousarray(np.asarray(grad_psi_n, np.float32))).to(self.device)
        if tuple(g.shape) != (nz, ny, nx):
            raise ValueError(f"grad_psi_n has shape {tuple(g.shape)}, expected {(nz, ny, nx)}")
        rc = lib().mvd_backward_recorded(self._h, int(token), C.c_void_p(g.data_ptr()), MEM_DEVICE,
                                         _ptr_array(gp_ptrs), None if gpsi is None else C.c_void_p(gpsi.data_ptr()),
                                         MEM_DEVICE)
        _check(rc, self._h)
        return gps, gpsi

    def _grad_buffers(self, psi0, grad_psf, grad_psi0, psf_shapes):
        nx, ny, nz = self.dims[0]
        src = None
        if psi0 is not None:
            src = psi0.detach().to(self.device, torch.float32).contiguous() if isinstance(psi0, torch.Tensor) \
                else torch.from_numpy(np.ascontiguousarray(np.asarray(psi0, np.float32))).to(self.device)
        shapes = psf_shapes or getattr(self, "_psf_shapes", None)
        gps = None
        gp_ptrs = None
        if grad_psf:
            if shapes is None:
                raise ValueError("PSF shapes unknown: pass psf_shapes or call set_psfs first")
            gps = [np.zeros(sh, np.float64) for sh in shapes]
            gp_ptrs = (C.c_void_p * len(gps))(*[x.ctypes.data for x in gps])
        gpsi = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device) if grad_psi0 else None
        return src, gps, gp_ptrs, gpsi

    SCHEDULES = {"pass": 0, "block": 1, "run": 2}

    def set_schedule(self, schedule):
        """'pass' (each pass over every block of a lane), 'block' (a lane's
        blocks one at a time per iteration) or 'run' (a lane's blocks one at
        a time for the whole run); same results, different cache use."""
        sch = self.SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        _check(lib().mvd_set_schedule(self._h, sch), self._h)
        return self

    def schedule(self):
        return {v: k for k, v in self.SCHEDULES.items()}[lib().mvd_get_schedule(self._h)]

    def tiles(self):
        """Current launch-shape candidates (x, y, z)."""
        c = (C.c_int * 3)()
        _check(lib().mvd_get_tiles(self._h, c), self._h)
        return tuple(c)

    def set_tiles(self, cx, cy, cz):
        _check(lib().mvd_set_tiles(self._h, int(cx), int(cy), int(cz)), self._h)
        return self

    def grid_dims(self, block=0):
        """The computation grid (nx, ny, nz) of a block (larger than the
        volume with the linear boundary)."""
        d = (C.c_int * 3)()
        _check(lib().mvd_grid_dims(self._h, int(block), d), self._h)
        return tuple(d)

    def max_lengths(self):
        """Longest transform of each pass kind over the blocks' grids: (nx/2, ny, nz)."""
        g = [self.grid_dims(b) for b in range(self.n_blocks)]
        return (max(d[0] // 2 for d in g), max(d[1] for d in g), max(d[2] for d in g))

    def estimate(self, block=0, out=None):
        """The current estimate as a CUDA tensor (nz, ny, nx)."""
        nx, ny, nz = self.dims[block]
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device)
        rc = lib().mvd_get_estimate(self._h, C.c_void_p(out.data_ptr()), MEM_DEVICE, block)
        _check(rc, self._h)
        return out

    def set_estimate(self, psi, block=0):
        if isinstance(psi, torch.Tensor) and psi.is_cuda:
            t = psi.detach().to(torch.float32).contiguous()
            rc = lib().mvd_set_estimate(self._h, C.c_void_p(t.data_ptr()), MEM_DEVICE, block)
        else:
            a = np.ascontiguousarray(np.asarray(psi.cpu() if isinstance(psi, torch.Tensor) else psi, np.float32))
            rc = lib().mvd_set_estimate(self._h, C.c_void_p(a.ctypes.data), MEM_HOST, block)
        _check(rc, self._h)
        return self

    def stats(self):
        s = Stats()
        _check(lib().mvd_stats(self._h, C.byref(s)), self._h)
        return dict(iterations=s.iterations, n_views=s.n_views, n_blocks=s.n_blocks, scale=s.scale,
                    flux=list(s.flux[:s.n_views]), ratio_clamps=s.ratio_clamps, neg_clamps=s.neg_clamps,
                    nonfinite=bool(s.nonfinite))

    def synchronize(self):
        _check(lib().mvd_synchronize(self._h), self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().mvd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def create_raw(blocks, options=None):
    """mvd_create_batch on host-memory blocks [(views, psfs, weights), ...].

    Returns (return code, handle or None, message); used to exercise the
    argument checks, which run before any device call."""
    ms = [_Marshalled(v, p, w, None, False) for (v, p, w) in blocks]
    arr = (Problem * len(ms))(*[m.problem for m in ms])
    h = C.c_void_p()
    rc = lib().mvd_create_batch(C.byref(h), len(ms), arr, None if options is None else C.byref(options))
    msg = lib().mvd_last_error(None).decode()
    return rc, (h if h.value else None), msg


def _ptr_array(arr):
    return None if arr is None else C.cast(arr, C.POINTER(C.c_void_p))


def tile_candidates(kind, max_len):
    n = lib().mvd_tile_candidates(kind, max_len, None, 0)
    out = (C.c_int * max(n, 1))()
    lib().mvd_tile_candidates(kind, max_len, out, n)
    return list(out[:n])


def tile_shape(kind, cfg):
    t, p, m, e = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check(lib().mvd_tile_shape(kind, cfg, C.byref(t), C.byref(p), C.byref(m), C.byref(e)))
    return dict(threads=t.value, per_tile=p.value, max_len=m.value, exact_len=e.value)


def compound_kernel(psfs, v, variant):
    """K_v of the library's host code (FP64), shape (kz, ky, kx) odd."""
    ps = [np.ascontiguousarray(np.asarray(p, np.float32)) for p in psfs]
    n = len(ps)
    ptrs = (C.c_void_p * n)(*[p.ctypes.data for p in ps])
    dims = (C.c_int * (3 * n))(*sum([[p.shape[2], p.shape[1], p.shape[0]] for p in ps], []))
    k = ps[v].shape
    out = np.zeros((k[0] | 1, k[1] | 1, k[2] | 1), np.float64)
    od = (C.c_int * 3)()
    rc = lib().mvd_compound_kernel(n, C.cast(ptrs, C.POINTER(C.c_void_p)), C.cast(dims, C.POINTER(C.c_int)), v,
                                   _variant(variant), out.ctypes.data, od)
    _check(rc)
    return out


def compound_kernel_vjp(psfs, v, variant, kbar):
    """dL/dP_w (normalised, odd-padded PSFs) of every view from dL/dK_v, by
    the library's host code (FP64)."""
    ps = [np.ascontiguousarray(np.asarray(p, np.float32)) for p in psfs]
    n = len(ps)
    ptrs = (C.c_void_p * n)(*[p.ctypes.data for p in ps])
    dims = (C.c_int * (3 * n))(*sum([[p.shape[2], p.shape[1], p.shape[0]] for p in ps], []))
    kb = np.ascontiguousarray(np.asarray(kbar, np.float64))
    outs = [np.zeros((p.shape[0] | 1, p.shape[1] | 1, p.shape[2] | 1), np.float64) for p in ps]
    optrs = (C.c_void_p * n)(*[o.ctypes.data for o in outs])
    rc = lib().mvd_compound_kernel_vjp(n, C.cast(ptrs, C.POINTER(C.c_void_p)), C.cast(dims, C.POINTER(C.c_int)), v,
                                       _variant(variant), kb.ctypes.data, C.cast(optrs, C.POINTER(C.c_void_p)))
    _check(rc)
    return outs


def kernel_spectrum(K, dims):
    """(main, nyquist) spectrum of a centred odd kernel on a volume of dims (nx, ny, nz)."""
    K = np.ascontiguousarray(np.asarray(K, np.float64))
    nx, ny, nz = dims
    main = np.zeros((nz, ny, nx // 2), np.complex64)
    nyq = np.zeros((nz, ny), np.complex64)
    kd = (C.c_int * 3)(K.shape[2], K.shape[1], K.shape[0])
    dd = (C.c_int * 3)(nx, ny, nz)
    _check(lib().mvd_kernel_spectrum(K.ctypes.data, kd, dd, main.ctypes.data, nyq.ctypes.data))
    return main, nyq
