"""hif_inverse_error_noalloc, the allocation-free entry point for callers that cannot allocate
device memory, against hif_inverse_error (the same iteration and kernels on scratch allocated
for the call): equal bit for bit, on two calls in a row, the second with a smaller grid, and a
clear HIF_ERR_ARG (nothing launched) for a grid above its fixed scratch.  Called through the
C ABI directly."""
import ctypes

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _estimates(lib, h, x0, iters):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    a, b = ctypes.c_double(), ctypes.c_double()
    st1 = lib.hif_inverse_error(h._p(), ctypes.c_void_p(x0.data_ptr()), iters, ctypes.byref(a), s)
    st2 = lib.hif_inverse_error_noalloc(h._p(), ctypes.c_void_p(x0.data_ptr()), iters,
                                        ctypes.byref(b), s)
    return st1, a.value, st2, b.value


def test_noalloc_equals_allocating_entry_point(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    lib = hifcn.raw_library()
    for n, leaf, eps, iters in ((256, 8, 1e-6, 12), (96, 8, 1e-4, 20)):   # second call smaller
        print(f"[case] noalloc n={n}", flush=True)
        a = torch.tensor(gen.grf_coefficient(n, 2, 0.1, 600 + n), device="cuda")
        h = hifcn.factor(a, 1e-2, n, 2, eps, store="f64", leaf=leaf)
        x0 = torch.tensor(gen.normal_vector(n * n, 700 + n), device="cuda")
        st1, e1, st2, e2 = _estimates(lib, h, x0, iters)
        assert st1 == hifcn.HIF_OK and st2 == hifcn.HIF_OK, (st1, st2)
        assert e2 == e1 and e1 > 0, (e1, e2)
        # and again on the same handle: the shared scratch keeps nothing from the last call
        st3 = lib.hif_inverse_error_noalloc(h._p(), ctypes.c_void_p(x0.data_ptr()), iters,
                                            ctypes.byref(ctypes.c_double(0)),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st3 == hifcn.HIF_OK
        assert h.inverse_error_noalloc(x0, iters) == e1
        h.close()


def test_noalloc_rejects_grids_above_its_scratch(gpu_lib):
    import torch
    from paper_2004_05566_amd import hifcn
    lib = hifcn.raw_library()
    n = 520   # 270,400 DOFs > 262,144
    a = torch.tensor(gen.grf_coefficient(n, 2, 0.1, 5), device="cuda")
    h = hifcn.factor(a, 1e-2, n, 2, 1e-4, store="f32", leaf=8)
    x0 = torch.tensor(gen.normal_vector(n * n, 6), device="cuda")
    est = ctypes.c_double(-1.0)
    st = lib.hif_inverse_error_noalloc(h._p(), ctypes.c_void_p(x0.data_ptr()), 5,
                                       ctypes.byref(est),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == hifcn.HIF_ERR_ARG
    assert b"exceeds" in lib.hif_last_error()
    assert est.value == -1.0
    # the allocating entry point takes it
    assert h.inverse_error(x0, 5) > 0
    h.close()
