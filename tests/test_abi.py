"""The C-ABI library loads and exports every entry point declared in include/hifcn.h (no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hifcn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["hif_factor", "hif_import", "hif_apply", "hif_spmv", "cn_step", "cn_solve",
              "hif_factor_bytes", "hif_get_info", "hif_destroy", "hif_last_error"]:
        assert n in names, n


def test_library_exports_every_declared_symbol():
    from paper_2004_05566_amd import hifcn
    lib = ctypes.CDLL(hifcn.library_path())
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(hifcn.EXPORTS) == set(_declared())


def test_error_path_without_gpu_work():
    """Argument errors are reported through status codes and hif_last_error, no exception."""
    from paper_2004_05566_amd import hifcn
    lib = hifcn.raw_library()
    h = ctypes.c_void_p(123)
    g = hifcn._Grid()
    g.dim = 4
    st = lib.hif_factor(None, 0.1, ctypes.byref(g), 1e-3, 1, None, ctypes.byref(h))
    assert st == hifcn.HIF_ERR_ARG and not h.value
    assert b"NULL" in lib.hif_last_error() or b"dim" in lib.hif_last_error()
    assert lib.hif_factor_bytes(None) == 0
    lib.hif_destroy(None)


def test_factor_options_errors_without_gpu_work():
    from paper_2004_05566_amd import hifcn
    lib = hifcn.raw_library()
    h = ctypes.c_void_p(123)
    g = hifcn._Grid()
    g.dim = 2
    o = hifcn._FactorOpts()
    o.reserved[1] = 7
    st = lib.hif_factor_ex(None, 0.1, ctypes.byref(g), 1e-3, 1, ctypes.byref(o), None,
                           ctypes.byref(h))
    assert st == hifcn.HIF_ERR_ARG and not h.value
    assert b"reserved" in lib.hif_last_error()


def test_batch_step_argument_errors_without_gpu_work():
    from paper_2004_05566_amd import hifcn
    lib = hifcn.raw_library()
    assert lib.cn_batch_step(None, None, None, None, -1, None, None, None, None) == \
        hifcn.HIF_ERR_ARG
    assert lib.cn_batch_step(None, None, None, None, 0, None, None, None, None) == hifcn.HIF_OK
    assert lib.cn_batch_step(None, None, None, None, 2, None, None, None, None) == \
        hifcn.HIF_ERR_ARG
    assert b"NULL" in lib.hif_last_error()


def test_info_struct_layout():
    """hif_info_t: 2 x i32, 2 x i64, 2 x i32, 2 x i64, f64 (no padding surprises)."""
    import ctypes
    from paper_2004_05566_amd import hifcn
    assert ctypes.sizeof(hifcn._Info) == 72
    assert hifcn._Info.apply_bytes.offset == 56
    assert hifcn._Info.top_level.offset == 64
    assert hifcn._Info.device_bytes.offset == 32
    assert hifcn._Info.build_mfma_ms.offset == 48
