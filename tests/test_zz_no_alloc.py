"""GPU test of the allocation-free merge-path SpMV (uc_spmv_merge_noalloc):
caller-owned device arrays, the library's static scratch, results equal to
the allocating entry point's bit for bit.

The device arrays are allocated through the HIP runtime the library itself
is linked against (looked up by its soname once the library is loaded), so
that one runtime serves the whole process."""

import ctypes
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2607_03627_amd import uclp
from paper_2607_03627_amd.instances import make_instance

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Hip:
    """hipMalloc / hipMemcpy / streams of the runtime libuclp uses."""

    def __init__(self):
        uclp.load()
        self.h = ctypes.CDLL("libamdhip64.so.7")
        self.h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.h.hipFree.argtypes = [ctypes.c_void_p]
        self.h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.h.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.h.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        self.live = []

    def ok(self, rc):
        assert rc == 0, f"HIP error {rc}"

    def upload(self, a):
        a = np.ascontiguousarray(a)
        p = ctypes.c_void_p()
        self.ok(self.h.hipMalloc(ctypes.byref(p), max(a.nbytes, 1)))
        self.live.append(p.value)
        if a.nbytes:
            self.ok(self.h.hipMemcpy(p.value, a.ctypes.data, a.nbytes, H2D))
        return p.value

    def download(self, p, n, dtype):
        out = np.empty(n, dtype)
        self.ok(self.h.hipMemcpy(out.ctypes.data, p, out.nbytes, D2H))
        return out

    def stream(self):
        s = ctypes.c_void_p()
        self.ok(self.h.hipStreamCreate(ctypes.byref(s)))
        return s.value

    def close(self):
        for p in self.live:
            self.h.hipFree(p)
        self.live = []


@pytest.fixture
def hip():
    h = Hip()
    yield h
    h.close()


def csr(lp):
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    A.sort_indices()
    return A


@pytest.mark.parametrize("prec", [uclp.UC_LP_FP64, uclp.UC_LP_FP32_MIXED])
def test_noalloc_spmv_equals_the_allocating_entry_point(hip, prec):
    # two calls in a row on the same scratch, the second with a smaller input
    # (fewer workgroups: the first call's coordinates and carries beyond the
    # second's range stay in the scratch and must not be read)
    rng = np.random.default_rng(5)
    nf = np.float64 if prec == uclp.UC_LP_FP64 else np.float32
    s = hip.stream()
    try:
        for A in (csr(make_instance("medium", 0)), csr(make_instance("tiny", 1))):
            say("case noalloc", prec, A.shape, A.nnz)
            m, n = A.shape
            x = rng.normal(size=n)
            rp, ci = hip.upload(A.indptr.astype(np.int32)), hip.upload(A.indices.astype(np.int32))
            v, xd = hip.upload(A.data.astype(nf)), hip.upload(x.astype(nf))
            y = hip.upload(np.full(m, np.nan, nf))
            uclp.uc_spmv_merge_noalloc(m, n, A.nnz, rp, ci, v, xd, y, prec, stream=s)
            hip.ok(hip.h.hipStreamSynchronize(s))
            got = hip.download(y, m, nf).astype(np.float64)
            ref = uclp.uc_spmv(m, n, A.indptr, A.indices, A.data, x, prec, uclp.UC_LP_SPMV_MERGEPATH)
            assert np.array_equal(got, ref)
    finally:
        hip.h.hipStreamDestroy(s)


def test_noalloc_spmv_rejects_what_it_cannot_take(hip):
    A = csr(make_instance("tiny", 0, n_periods=2))
    m, n = A.shape
    rp, ci = hip.upload(A.indptr.astype(np.int32)), hip.upload(A.indices.astype(np.int32))
    v, xd, y = hip.upload(A.data), hip.upload(np.ones(n)), hip.upload(np.zeros(m))
    # beyond the static scratch: refused before any launch
    rc = uclp.uc_spmv_merge_noalloc(2 ** 31 - 1, n, 2 ** 31 - 1, rp, ci, v, xd, y, uclp.UC_LP_FP64, raw=True)
    assert rc == uclp.UC_LP_ENOTSUP
    # a host array where a device array belongs
    hx = np.ones(n)
    rc = uclp.uc_spmv_merge_noalloc(m, n, A.nnz, rp, ci, v, hx.ctypes.data, y, uclp.UC_LP_FP64, raw=True)
    assert rc == uclp.UC_LP_EINVAL
    # and the valid call still works after both refusals
    uclp.uc_spmv_merge_noalloc(m, n, A.nnz, rp, ci, v, xd, y, uclp.UC_LP_FP64)
    hip.ok(hip.h.hipStreamSynchronize(None))
    got = hip.download(y, m, np.float64)
    assert np.allclose(got, A @ np.ones(n), rtol=1e-13, atol=1e-13)
