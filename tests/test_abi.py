"""The C ABI library loads, exports every entry point include/adc.h declares,
and rejects bad input on the host before touching any device (runs on CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2511_21640_amd as adc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "adc.h")).read()
    return sorted(set(re.findall(r"\b(adc_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    assert _declared() == sorted(adc.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(adc.LIB_PATH):
        adc.build()
    return adc.load()


def test_exports(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def _problem(kind=0, o=2, v=3, N=4, k=1, eps=None, L=None, x=1.0):
    n = o + v
    eps = np.linspace(-1, 1, n) if eps is None else eps
    if L is None:
        rng = np.random.default_rng(0)
        G = rng.standard_normal((N, n, n)) + 1j * rng.standard_normal((N, n, n))
        L = 0.05 * (G + G.conj().transpose(0, 2, 1))
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.complex128)
    p = adc.AdcProblem(kind, o, v, N, k, eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), L.ctypes.data, 0, x)
    return p, (eps, L)


def _init(lib, p):
    h = ctypes.c_void_p()
    return lib.adc_init(ctypes.byref(p), 1, None, ctypes.byref(h)), h


def test_validation_errors(lib):
    assert lib.adc_init(None, 1, None, None) == -1
    p, keep = _problem(o=0)
    assert _init(lib, p)[0] == -1
    p, keep = _problem(kind=7)
    assert _init(lib, p)[0] == -1
    p, keep = _problem(v=1)
    assert _init(lib, p)[0] == -1
    eps = np.linspace(-1, 1, 5)
    eps[2] = np.nan
    p, keep = _problem(eps=eps)
    assert _init(lib, p)[0] == -2
    p, keep = _problem(x=float("inf"))
    assert _init(lib, p)[0] == -2
    rng = np.random.default_rng(1)
    L = 0.05 * (rng.standard_normal((4, 5, 5)) + 1j * rng.standard_normal((4, 5, 5)))
    p, keep = _problem(L=L)
    assert _init(lib, p)[0] == -3
    L = np.zeros((4, 5, 5), complex)
    L[1, 2, 2] = np.inf
    p, keep = _problem(L=L)
    assert _init(lib, p)[0] == -2
    # a batch of two instances whose second entry is invalid is rejected on
    # the host before any device work
    p0, keep0 = _problem()
    p1, keep1 = _problem(o=0)
    arr = (adc.AdcProblem * 2)(p0, p1)
    h = ctypes.c_void_p()
    assert lib.adc_init(arr, 2, None, ctypes.byref(h)) == -1
    assert not h.value
    # options out of range
    opts = adc.AdcOptions()
    opts.precision = 3
    assert lib.adc_init(arr, 1, ctypes.byref(opts), ctypes.byref(h)) == -1
    # the failed call leaves its detail for the calling thread
    assert isinstance(lib.adc_last_error(), bytes) and len(lib.adc_last_error()) > 0
    # every option out of its documented range is rejected before any device
    # work, and the detail names the option
    for field, value, word in [("precision", 3, b"precision"), ("n_streams", -1, b"n_streams"),
                               ("graphs", 3, b"graphs"), ("precond", 2, b"precond"),
                               ("conv_tol", -1e-6, b"conv_tol"), ("conv_tol", float("nan"), b"conv_tol"),
                               ("conv_tol", float("inf"), b"conv_tol"), ("max_iter", -1, b"max_iter"),
                               ("max_subspace", -4, b"max_subspace"), ("refine_fp64", 2, b"refine_fp64"),
                               ("refine_fp64", -2, b"refine_fp64")]:
        opts = adc.AdcOptions()
        setattr(opts, field, value)
        h = ctypes.c_void_p()
        assert lib.adc_init(arr, 1, ctypes.byref(opts), ctypes.byref(h)) == -1, field
        assert not h.value
        assert word in lib.adc_last_error(), (field, lib.adc_last_error())


def test_null_handle(lib):
    """Every entry point that takes a handle rejects NULL with INVALID_ARG
    before touching the device (the other arguments are NULL or 1)."""
    for name in ("adc_dims", "adc_sigma", "adc_sigma_term", "adc_sigma_noalloc", "adc_properties", "adc_fns",
                 "adc_davidson", "adc_sigma_backward"):
        f = getattr(lib, name)
        args = []
        for t in f.argtypes:
            if t in (ctypes.c_int, ctypes.c_longlong):
                args.append(1)
            elif t is ctypes.c_double:
                args.append(0.5)
            else:
                args.append(None)
        assert f(*args) == -1, name
        assert lib.adc_last_error().startswith(name.encode() + b":"), (name, lib.adc_last_error())


def test_strerror(lib):
    for c in (0, 1, -1, -2, -3, -4, -5, -6, 99):
        assert isinstance(lib.adc_strerror(c), bytes)
    lib.adc_free(None)
