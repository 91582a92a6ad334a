"""The device-pointer entry points: psara_set_data_dev and psara_get_image_dev.

Device buffers come from the HIP runtime the library itself runs on (hipMalloc through ctypes;
no torch in the process).  A solve whose data went in from device memory ends bit for bit where
the same solve with host data ends, and the image read into device memory equals the host
read-out; NULL, host memory and non-finite data are refused (the previous data kept).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from gpu_common import PREC, say
from oracle import problem
from paper_1801_02417_amd import psara as P
from paper_1801_02417_amd import workloads as wk

pytestmark = pytest.mark.gpu

STAGES = [6, 4, 4]


class DeviceBuffer:
    """hipMalloc'd memory of `nbytes`, with host copies in and out."""

    def __init__(self, nbytes: int):
        P.lib()                                  # the library loads the system HIP runtime first
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.hip.hipDeviceSynchronize.argtypes = []
        self.ptr = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(self.ptr), nbytes) == 0
        self.nbytes = nbytes

    def put(self, a: np.ndarray) -> None:
        a = np.ascontiguousarray(a)
        assert a.nbytes == self.nbytes
        assert self.hip.hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, 1) == 0     # host to device
        assert self.hip.hipDeviceSynchronize() == 0

    def get(self, shape, dtype=np.float64) -> np.ndarray:
        out = np.empty(shape, dtype=dtype)
        assert out.nbytes == self.nbytes
        assert self.hip.hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, 2) == 0  # device to host
        return out

    def free(self) -> None:
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = C.c_void_p()


def _solver(wl, b, prec, data):
    s = P.Solver(wl.n, wl.uv, taps=wl.taps, precision=PREC[prec])
    s.set_prior(wl.levels, b.gamma)
    data(s)
    s.opnorm(60, 1e-6)
    s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
    return s


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_device_data_and_image_equal_host_path(prec):
    wl = wk.blobs32()
    b = problem.build(wl, norm_rtol=1e-6, norm_max_iter=40)
    Y = np.ascontiguousarray(b.pb.Y, dtype=np.complex128)
    say(f"[dev] host-data solve {prec}")
    s_host = _solver(wl, b, prec, lambda s: s.set_data(Y, b.pb.eps))
    rep_h = s_host.reweighted_solve(P.PSARA_CONSTRAINED, STAGES)
    img_h = s_host.image()
    s_host.close()

    ybuf = DeviceBuffer(Y.nbytes)
    ybuf.put(Y.view(np.float64))
    sbuf = DeviceBuffer(wl.n * wl.n * 4 * 8)
    try:
        say(f"[dev] device-data solve {prec}")
        s_dev = _solver(wl, b, prec, lambda s: P.psara_set_data_dev(s.ctx, ybuf.ptr.value, b.pb.eps))
        rep_d = s_dev.reweighted_solve(P.PSARA_CONSTRAINED, STAGES)
        img_d = s_dev.image()
        P.psara_get_image_dev(s_dev.ctx, sbuf.ptr.value)
        img_dd = sbuf.get((wl.n * wl.n, 4))
        s_dev.close()
    finally:
        ybuf.free()
        sbuf.free()
    say(f"[dev] max |device - host| = {float(np.max(np.abs(img_d - img_h))):.3e}")
    assert np.array_equal(img_d, img_h)
    assert rep_d["residual"] == rep_h["residual"]
    assert np.array_equal(img_dd, img_h)


def test_device_entry_points_refuse_bad_buffers():
    wl = wk.tiny(n=16, M=150, taps=8, levels=2, seed=7)
    b = problem.build(wl, norm_rtol=1e-6, norm_max_iter=40)
    Y = np.ascontiguousarray(b.pb.Y, dtype=np.complex128)
    s = P.Solver(wl.n, wl.uv, taps=wl.taps, precision=P.PSARA_FP32_MIXED)
    s.set_prior(wl.levels, b.gamma)
    ybuf = DeviceBuffer(Y.nbytes)
    try:
        with pytest.raises(P.PsaraError) as e:
            P.psara_set_data_dev(s.ctx, 0, b.pb.eps)
        assert e.value.status == P.PSARA_EINVAL
        host = np.zeros(Y.size * 2)
        with pytest.raises(P.PsaraError) as e:
            P.psara_set_data_dev(s.ctx, host.ctypes.data, b.pb.eps)
        assert e.value.status == P.PSARA_EINVAL
        with pytest.raises(P.PsaraError) as e:
            P.psara_get_image_dev(s.ctx, host.ctypes.data)
        assert e.value.status == P.PSARA_EINVAL
        # good data, then data with a NaN: refused, and the good data kept
        ybuf.put(Y.view(np.float64))
        P.psara_set_data_dev(s.ctx, ybuf.ptr.value, b.pb.eps)
        bad = Y.copy()
        bad[len(bad) // 2, 1] = complex(np.nan, 0.0)
        ybuf.put(bad.view(np.float64))
        with pytest.raises(P.PsaraError) as e:
            P.psara_set_data_dev(s.ctx, ybuf.ptr.value, b.pb.eps)
        assert e.value.status == P.PSARA_ENAN
        # the refused upload changed nothing: ten iterations end where a solve with the host data ends
        ref = _solver(wl, b, "fp32", lambda r: r.set_data(Y, b.pb.eps))
        s.opnorm(60, 1e-6)
        s.set_steps(b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3)
        s.solve(P.PSARA_CONSTRAINED, 10, report=False)
        ref.solve(P.PSARA_CONSTRAINED, 10, report=False)
        assert np.array_equal(s.image(), ref.image())
        ref.close()
    finally:
        ybuf.free()
        s.close()
