"""Failure paths of the C ABI on the GPU: a device allocator that runs out
(MVD_ENOMEM with *out left NULL and every buffer handed back), a lazy
allocation that fails inside a later call (the handle stays usable), and an
estimate that overflows FP32 (MVD_ENONFINITE at the next synchronising call,
cleared by setting a finite estimate)."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from tests.test_gpu_parity import problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


class CappedAllocator:
    """Device memory from torch, refused once `cap` bytes are live."""

    def __init__(self, mvd, cap):
        self.cap, self.live, self.bufs, self.refused = cap, 0, {}, 0

        def alloc(n, ctx):
            if self.live + n > self.cap:
                self.refused += 1
                return None
            t = torch.empty(int(n), dtype=torch.uint8, device="cuda")
            self.bufs[t.data_ptr()] = t
            self.live += n
            return t.data_ptr()

        def free(p, ctx):
            t = self.bufs.pop(p)
            self.live -= t.numel()

        self.alloc_cb, self.free_cb = mvd.ALLOC_FN(alloc), mvd.FREE_FN(free)

    def options(self, mvd):
        return mvd.Options(0.0, 0.0, C.c_void_p(torch.cuda.current_stream().cuda_stream), self.alloc_cb,
                           self.free_cb, None, 1, 0, 0)


def create(mvd, views, psfs, alloc):
    m = mvd._Marshalled(views, psfs, None, torch.device("cuda"), False)
    h = C.c_void_p()
    opts = alloc.options(mvd)
    rc = mvd.lib().mvd_create(C.byref(h), C.byref(m.problem), C.byref(opts))
    return rc, h


def test_create_fails_cleanly_when_the_allocator_runs_out(mvd):
    views, psfs, _ = problem((48, 40, 36), 3, 501)
    probe = CappedAllocator(mvd, 1 << 40)
    rc, h = create(mvd, views, psfs, probe)
    assert rc == mvd.MVD_OK
    need = probe.live  # what create holds
    mvd.lib().mvd_destroy(h)
    assert probe.live == 0 and not probe.bufs
    for cap in (0, need // 4, need // 2, need - 1):
        a = CappedAllocator(mvd, cap)
        rc, h = create(mvd, views, psfs, a)
        msg = mvd.lib().mvd_last_error(None).decode()
        print(f"cap {cap}: rc {rc} ({msg}); live after {a.live} bytes in {len(a.bufs)} buffers")
        assert rc == mvd.MVD_ENOMEM and not h.value
        assert a.refused >= 1 and a.live == 0 and not a.bufs


def test_lazy_allocation_failure_keeps_the_handle(mvd):
    """Enough memory for create and the RL run, not for the compound-kernel
    planes that the first OPT1 run builds: that call returns MVD_ENOMEM and
    the handle still runs RL, and OPT1 once memory is allowed."""
    views, psfs, _ = problem((48, 40, 36), 3, 502)
    probe = CappedAllocator(mvd, 1 << 40)
    rc, h = create(mvd, views, psfs, probe)
    assert rc == mvd.MVD_OK
    L = mvd.lib()
    assert L.mvd_iterate(h, 1, O.RL) == mvd.MVD_OK
    need = probe.live
    L.mvd_destroy(h)
    assert probe.live == 0
    a = CappedAllocator(mvd, need)
    rc, h = create(mvd, views, psfs, a)
    assert rc == mvd.MVD_OK
    try:
        assert L.mvd_iterate(h, 1, O.OPT1) == mvd.MVD_ENOMEM
        print("lazy failure:", L.mvd_last_error(h).decode())
        assert L.mvd_iterate(h, 2, O.RL) == mvd.MVD_OK
        out = torch.empty(views[0].shape, dtype=torch.float32, device="cuda")
        assert L.mvd_get_estimate(h, C.c_void_p(out.data_ptr()), mvd.MEM_DEVICE, 0) == mvd.MVD_OK
        pb = O.Problem(views, psfs)
        assert rel(out.cpu().numpy(), pb.iterate(pb.psi0(), 2, O.RL)) <= 1e-4
        a.cap = 1 << 40
        assert L.mvd_iterate(h, 1, O.OPT1) == mvd.MVD_OK
        assert L.mvd_synchronize(h) == mvd.MVD_OK
    finally:
        L.mvd_destroy(h)
    assert a.live == 0


def test_overflow_is_reported_as_nonfinite(mvd):
    """Views of 3e38 (finite) and an estimate of 1e20 with one voxel at 1e38:
    around that voxel the ratio is about 30, so the multiplicative step
    exceeds the FP32 range.  The next synchronising calls return
    MVD_ENONFINITE (the estimate is still copied out); setting a finite
    estimate clears the flag."""
    shape = (12, 16, 20)
    views = [np.full(shape, 3e38, np.float32) for _ in range(2)]
    _, psfs, _ = problem((20, 16, 12), 2, 503, psf_shape=(5, 5, 5))
    psi = np.full(shape, 1e20, np.float32)
    psi[6, 8, 10] = 1e38
    with mvd.Deconvolver(views, psfs) as d:
        d.set_estimate(psi)
        d.view_update(0, O.RL)
        with pytest.raises(mvd.MVDError) as e:
            d.synchronize()
        assert e.value.code == mvd.MVD_ENONFINITE
        with pytest.raises(mvd.MVDError) as e:
            d.estimate()
        assert e.value.code == mvd.MVD_ENONFINITE
        assert d.stats()["nonfinite"]
        d.set_estimate(np.full(shape, 1e20, np.float32))
        d.synchronize()
        assert not d.stats()["nonfinite"]
        d.iterate(1, O.RL)
        got = d.estimate().cpu().numpy()
    assert np.all(np.isfinite(got))
