"""C-ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2312_02667_amd import ptebd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ptebd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ptebd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ptebd.lib()
    declared = _declared_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(ptebd.EXPORTED)


def test_version_string():
    assert ptebd.lib().ptebd_version().decode().startswith("ptebd")


def _create(n_states, n_sites, caps, d=2, precision=0):
    lib = ptebd.lib()
    ns = np.asarray(n_sites, np.int32)
    cs = np.asarray(caps, np.int32)
    h = ctypes.c_void_p()
    code = lib.ptebd_mps_create(n_states, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                cs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), d, precision,
                                None, ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("args", [
    (1, [10], [32], 3, 0),      # d must be 2
    (0, [10], [32], 2, 0),      # no states
    (1, [1], [32], 2, 0),       # N < 2
    (1, [10], [0], 2, 0),       # chi_cap < 1
    (1, [10], [1024], 2, 0),    # chi_cap > 512
    (1, [10], [32], 2, 7),      # unknown precision
    (1, [10], [32], 2, 2),      # PTEBD_BF16X3: declared, not built
])
def test_create_rejects_bad_arguments_before_device_work(args):
    code, h = _create(*args)
    assert code == ptebd.EINVAL
    assert not h.value
    assert ptebd.lib().ptebd_last_error().decode()


def test_null_handle_calls_are_rejected():
    lib = ptebd.lib()
    out = ctypes.c_double()
    assert lib.ptebd_norm(None, 0, ctypes.byref(out)) == ptebd.EINVAL
    assert lib.ptebd_apply_layer(None, 0, None, None, None, 4, 1e-12, 0, 0, None) == ptebd.EINVAL
    assert lib.ptebd_mps_destroy(None) == ptebd.OK


def test_svd_batched_rejects_bad_arguments():
    lib = ptebd.lib()
    a = np.zeros(8)
    s = np.zeros(2)
    p = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ps = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ptebd_svd_batched(0, 0, 2, 2, p, ps, None, None, None, 30, 4.0, None) == ptebd.EINVAL
    assert lib.ptebd_svd_batched(5, 1, 2, 2, p, ps, None, None, None, 30, 4.0, None) == ptebd.EINVAL
    assert lib.ptebd_svd_batched(ptebd.BF16X3, 1, 2, 2, p, ps, None, None, None, 30, 4.0,
                                 None) == ptebd.EINVAL
    assert "not built" in lib.ptebd_last_error().decode()
    a[0] = np.nan
    assert lib.ptebd_svd_batched(0, 1, 2, 2, p, ps, None, None, None, 30, 4.0, None) == ptebd.EINVAL


def test_header_constants_match_binding():
    """The binding's flag and precision constants are the header's."""
    src = open(os.path.join(ROOT, "include", "ptebd.h")).read()
    defs = dict(re.findall(r"#define (PTEBD_[A-Z0-9_]+)\s+\(?(-?[0-9.e+-]+)\)?", src))
    assert int(defs["PTEBD_FLAG_NO_STABILIZE"]) == ptebd.FLAG_NO_STABILIZE
    assert int(defs["PTEBD_FLAG_RELATIVE_EPS"]) == ptebd.FLAG_RELATIVE_EPS
    assert int(defs["PTEBD_FLAG_COMPLEMENT_EPS"]) == ptebd.FLAG_COMPLEMENT_EPS
    assert float(defs["PTEBD_FP32_CUTOFF_FLOOR"]) == ptebd.FP32_CUTOFF_FLOOR == 2.0 ** -19
    assert int(defs["PTEBD_FP64"]) == ptebd.FP64 and int(defs["PTEBD_FP32"]) == ptebd.FP32
    assert int(defs["PTEBD_BF16X3"]) == ptebd.BF16X3


def test_every_declaration_cites_or_documents():
    """Every entry point in the header carries a comment block of its own (the passage it
    follows, or what it is for), placed right above its declaration."""
    src = open(os.path.join(ROOT, "include", "ptebd.h")).read()
    for name in _declared_functions():
        idx = re.search(r"^[a-z][a-z_ *]*\b" + name + r"\(", src, flags=re.M).start()
        head = src[:idx]
        # the text between the previous declaration's end and this one holds a comment
        prev = max(head.rfind(";"), head.rfind("{"))
        assert "*/" in head[prev:], name


def test_svd_noalloc_rejects_oversized_batches_before_device_work():
    """The allocation-free SVD refuses a batch that does not fit its fixed scratch array
    (one 1024 x 1024 FP64 matrix needs well over 32 MiB) with EINVAL and a message, before it
    touches the device, so this runs without a GPU."""
    lib = ptebd.lib()
    a = np.zeros(8)
    s = np.zeros(2)
    p = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ps = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ptebd_svd_batched_noalloc(0, 1, 1024, 1024, p, ps, None, None, None, 30, 4.0,
                                         None) == ptebd.EINVAL
    assert "scratch" in lib.ptebd_last_error().decode()
    assert lib.ptebd_svd_batched_noalloc(0, 0, 2, 2, p, ps, None, None, None, 30, 4.0,
                                         None) == ptebd.EINVAL
    assert lib.ptebd_svd_batched_noalloc(ptebd.BF16X3, 1, 2, 2, p, ps, None, None, None, 30, 4.0,
                                         None) == ptebd.EINVAL
