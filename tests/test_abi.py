"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point that include/nfft.h declares, and validates arguments
before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2302_00414_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nfft.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nfft_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert set(_declared()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_strerror_texts():
    lib = _lib.load()
    for s in range(6):
        assert lib.nfft_strerror(s)
    assert b"unknown" in lib.nfft_strerror(99)


@pytest.mark.parametrize("args,status", [
    ((0, 32, 2.0, 4), _lib.NFFT_EINVAL),       # d out of range
    ((4, 32, 2.0, 4), _lib.NFFT_EINVAL),
    ((2, 31, 2.0, 4), _lib.NFFT_EINVAL),       # odd M
    ((2, 0, 2.0, 4), _lib.NFFT_EINVAL),
    ((2, 32, 0.5, 4), _lib.NFFT_EINVAL),       # sigma < 1
    ((2, 32, float("nan"), 4), _lib.NFFT_EINVAL),
    ((2, 32, 2.0, 0), _lib.NFFT_EINVAL),       # m < 1
    ((2, 4, 2.0, 4), _lib.NFFT_EINVAL),        # M_sigma = 8 < 2m + 2
    ((2, 32, 2.0, 9), _lib.NFFT_EUNSUPPORTED),  # m > 8
    ((2, 30, 2.0, 4), _lib.NFFT_EUNSUPPORTED),  # M_sigma = 60 not a power of two
    ((3, 64, 2.0, 8), _lib.NFFT_OK),           # float32 3-D, m = 8: two float32 planes fit in LDS
    ((3, 64, 2.0, 6), _lib.NFFT_OK),           # valid
])
def test_plan_validation_before_device(args, status):
    lib = _lib.load()
    x = np.zeros((4, args[0] if 1 <= args[0] <= 3 else 1))
    h = ctypes.c_void_p(123)
    st = lib.nfft_plan(ctypes.byref(h), *args, 4, x.ctypes.data, _lib.NFFT_F32, 1, None)
    if status == _lib.NFFT_OK:
        # validation passed; without a GPU the plan fails at the device
        assert st in (_lib.NFFT_OK, _lib.NFFT_EDEVICE)
        if st == _lib.NFFT_OK:
            lib.nfft_destroy(h)
    else:
        assert st == status
        assert h.value is None
        assert lib.nfft_last_error(None)


def test_f64_3d_large_m_unsupported():
    """The padded float64 accumulation tile of a 3-D plan with m = 8 does not fit in LDS."""
    lib = _lib.load()
    x = np.zeros((4, 3))
    h = ctypes.c_void_p()
    st = lib.nfft_plan(ctypes.byref(h), 3, 64, 2.0, 8, 4, x.ctypes.data, _lib.NFFT_F64, 1, None)
    assert st == _lib.NFFT_EUNSUPPORTED


@pytest.mark.parametrize("d,m,prec,tuning,status", [
    (2, 6, _lib.NFFT_F32, [12], _lib.NFFT_EINVAL),                # tile edge not a power of two
    (2, 6, _lib.NFFT_F32, [4], _lib.NFFT_EINVAL),                 # tile edge below 8
    (2, 6, _lib.NFFT_F32, [512], _lib.NFFT_EINVAL),               # tile edge above 256
    (2, 6, _lib.NFFT_F32, [0, 8], _lib.NFFT_EINVAL),              # work item below 16 nodes
    (2, 6, _lib.NFFT_F32, [0, 0, 96], _lib.NFFT_EINVAL),          # spread threads not 64/128/256
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 3], _lib.NFFT_EINVAL),        # rhs per group not 1/2/4/8
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 70000], _lib.NFFT_EINVAL),  # fft min work-groups
    (2, 6, _lib.NFFT_F32, [-1], _lib.NFFT_EINVAL),                # negative entry
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 3], _lib.NFFT_EINVAL),  # spread planes not 1/2
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 8], _lib.NFFT_EINVAL),  # spread mode not 1..7
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 7], _lib.NFFT_OK),   # padded tile on the matrix cores
    (2, 8, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 7], _lib.NFFT_OK),   # 2m + 1 > 16: resolved to mode 5
    (2, 6, _lib.NFFT_F32, [0, 0, 512, 0, 0, 0, 7], _lib.NFFT_OK),  # eight waves a work-group
    (2, 6, _lib.NFFT_F64, [0, 0, 0, 0, 0, 0, 7], _lib.NFFT_OK),   # float64 on the matrix cores
    (3, 4, _lib.NFFT_F32, [8, 0, 0, 0, 0, 0, 7], _lib.NFFT_OK),   # d = 3 on the matrix cores
    (3, 4, _lib.NFFT_F64, [8, 0, 0, 0, 0, 0, 7], _lib.NFFT_OK),   # d = 3 float64 on the matrix cores
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 6], _lib.NFFT_OK),   # grid-tile gather
    (2, 6, _lib.NFFT_F64, [0, 0, 0, 0, 0, 0, 6], _lib.NFFT_OK),   # float64: resolved to mode 4
    (2, 6, _lib.NFFT_F32, [8, 0, 0, 0, 0, 0, 6], _lib.NFFT_OK),   # tile edge 8: resolved to mode 4
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 5], _lib.NFFT_OK),   # padded tile in registers
    (2, 6, _lib.NFFT_F32, [0, 0, 512, 0, 0, 0, 5], _lib.NFFT_OK),  # eight waves a work-group
    (2, 6, _lib.NFFT_F32, [0, 0, 512], _lib.NFFT_OK),             # LDS kernel: resolved to 256
    (2, 6, _lib.NFFT_F64, [0, 0, 0, 0, 0, 0, 5], _lib.NFFT_OK),   # float64: resolved to mode 4
    (2, 6, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 4], _lib.NFFT_OK),   # window evaluated late
    (2, 6, _lib.NFFT_F64, [0, 0, 0, 0, 0, 0, 3], _lib.NFFT_OK),   # precomputed window factors
    (3, 4, _lib.NFFT_F32, [0, 0, 0, 0, 0, 0, 3], _lib.NFFT_OK),   # mode 3 resolves to 1 for d = 3
    (2, 8, _lib.NFFT_F32, [32, 0, 256, 0, 0, 2], _lib.NFFT_OK),   # 16 float32 48^2 planes fit
    (3, 4, _lib.NFFT_F32, [32], _lib.NFFT_EUNSUPPORTED),          # 40^3 padded tile exceeds LDS
    (2, 8, _lib.NFFT_F32, [64, 0, 256], _lib.NFFT_EUNSUPPORTED),  # 16 private 80^2 tiles exceed LDS
    (2, 8, _lib.NFFT_F64, [32, 0, 0, 8], _lib.NFFT_EUNSUPPORTED),  # 8 float64 48^2 tiles exceed LDS
    (2, 6, _lib.NFFT_F32, [32, 512, 64, 4, 128], _lib.NFFT_OK),
    (2, 6, _lib.NFFT_F32, None, _lib.NFFT_OK),
])
def test_tuning_validation_before_device(d, m, prec, tuning, status):
    lib = _lib.load()
    x = np.zeros((4, d))
    h = ctypes.c_void_p(123)
    arr = (ctypes.c_int32 * len(tuning))(*tuning) if tuning is not None else None
    st = lib.nfft_plan_tuned(ctypes.byref(h), d, 128, 2.0, m, 4, x.ctypes.data, prec, 4, arr,
                             len(tuning) if tuning else 0, None)
    if status == _lib.NFFT_OK:
        assert st in (_lib.NFFT_OK, _lib.NFFT_EDEVICE)
        if st == _lib.NFFT_OK:
            lib.nfft_destroy(h)
    else:
        assert st == status, lib.nfft_last_error(None)
        assert h.value is None
        assert lib.nfft_last_error(None)


def test_weights_argument_checks():
    lib = _lib.load()
    x = np.zeros((8, 2))
    info = (ctypes.c_double * 4)()
    buf = ctypes.c_void_p(1)
    assert lib.nfft_weights(2, 16, 2.0, 8, 8, x.ctypes.data, 1e-13, 100, None, info, None) == _lib.NFFT_EINVAL
    assert lib.nfft_weights(2, 16, 2.0, 8, 8, x.ctypes.data, 0.0, 100, buf, info, None) == _lib.NFFT_EINVAL
    assert lib.nfft_weights(2, 16, 2.0, 8, 8, x.ctypes.data, 1e-13, 0, buf, info, None) == _lib.NFFT_EINVAL
    assert lib.nfft_weights(2, 15, 2.0, 8, 8, x.ctypes.data, 1e-13, 10, buf, info, None) == _lib.NFFT_EINVAL
    assert lib.nfft_last_error(None)


def test_tuning_knobs_need_a_plan():
    lib = _lib.load()
    out = (ctypes.c_int32 * 7)()
    assert lib.nfft_get_tuning(None, out, 7) == _lib.NFFT_EINVAL
    assert lib.nfft_set_tuning(None, _lib.NFFT_TUNE_SPREAD_THREADS, 64) == _lib.NFFT_EINVAL


def test_bad_counts_and_pointers():
    lib = _lib.load()
    h = ctypes.c_void_p()
    x = np.zeros((4, 2))
    assert lib.nfft_plan(ctypes.byref(h), 2, 32, 2.0, 4, 0, x.ctypes.data, 0, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_plan(ctypes.byref(h), 2, 32, 2.0, 4, 4, None, 0, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_plan(ctypes.byref(h), 2, 32, 2.0, 4, 4, x.ctypes.data, 7, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_plan(ctypes.byref(h), 2, 32, 2.0, 4, 4, x.ctypes.data, 0, 0, None) == _lib.NFFT_EINVAL
    assert lib.nfft_plan(None, 2, 32, 2.0, 4, 4, x.ctypes.data, 0, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_adjoint(None, None, None, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_forward(None, None, None, 1, None) == _lib.NFFT_EINVAL
    assert lib.nfft_refine(None, None, None, 1, 2, None, None) == _lib.NFFT_EINVAL
    assert lib.nfft_set_weights(None, None, None) == _lib.NFFT_EINVAL
    assert lib.nfft_destroy(None) == _lib.NFFT_OK


def test_footprint_grows_with_inputs():
    lib = _lib.load()
    a = lib.nfft_footprint(2, 256, 2.0, 6, 262144, _lib.NFFT_F32, 1)
    b = lib.nfft_footprint(2, 256, 2.0, 6, 262144, _lib.NFFT_F64, 1)
    c = lib.nfft_footprint(2, 256, 2.0, 6, 262144, _lib.NFFT_F32, 32)
    assert 0 < a < b and c > 8 * a
    # the per-node part: window factor table (4 m reals) among the node arrays
    n2 = lib.nfft_footprint(2, 256, 2.0, 6, 2 * 262144, _lib.NFFT_F32, 1)
    assert n2 - a >= 262144 * 4 * 6 * 4
    assert lib.nfft_footprint(2, 31, 2.0, 6, 10, 0, 1) == -1
