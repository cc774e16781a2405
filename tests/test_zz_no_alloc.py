"""The allocation-free sigma entry point (adc_sigma_noalloc) against adc_sigma.

It runs the same build with every temporary in the library's fixed device
scratch, so its result must equal adc_sigma's on the same inputs: two calls
in a row on one handle, the second with fewer vectors (the scratch keeps the
first call's contents, nothing may depend on them), in FP64, FP32 and
split-bf16, for EE, IP and EA; a second handle afterwards; and a request that
cannot fit the scratch is refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

from adcgen import make_problem

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _rand(rng, k, dim):
    return torch.from_numpy(rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))).cuda()


def _noalloc(h, Y, prec):
    """adc_sigma_noalloc straight through the C ABI."""
    S = torch.full_like(Y, complex("nan"))
    rc = h._lib.adc_sigma_noalloc(h._h, 0, ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                  Y.shape[0], adc.PREC[prec])
    return rc, S


@pytest.mark.parametrize("kind,o,v,N", [("EE", 6, 24, 80), ("IP", 8, 40, 120), ("EA", 5, 36, 100)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16"])
def test_noalloc_equals_sigma(kind, o, v, N, prec):
    print(f"case noalloc {kind} o={o} v={v} N={N} {prec}", flush=True)
    P = make_problem(kind, o, v, N, seed=71, n_roots=3, x=0.5, scale=0.2)
    h = adc.Handle(kind, o, v, P.eps, P.L, 3, x=P.x)
    rng = np.random.default_rng(71)
    for k in (4, 2):
        Y = _rand(rng, k, h.dim)
        ref = h.sigma(Y, precision=prec)
        rc, S = _noalloc(h, Y, prec)
        torch.cuda.synchronize()
        assert rc == 0, adc.ERRORS.get(rc, rc)
        err = ((S - ref).abs().max() / ref.abs().max()).item()
        print(f"  k={k} max rel diff {err:.2e}", flush=True)
        # the same kernels on the same operands: bitwise equal up to the
        # choice of cached planes, which holds the same values
        assert err <= 1e-14
    h.close()


def test_noalloc_second_handle_and_too_large():
    print("case noalloc second handle + too large", flush=True)
    P = make_problem("EE", 4, 16, 50, seed=72, n_roots=2, x=1.0, scale=0.2)
    h = adc.Handle("EE", 4, 16, P.eps, P.L, 2, x=P.x, precision="split_bf16")
    rng = np.random.default_rng(72)
    Y = _rand(rng, 3, h.dim)
    rc, S = _noalloc(h, Y, "split_bf16")
    assert rc == 0
    assert ((S - h.sigma(Y)).abs().max() / S.abs().max()).item() <= 1e-14
    # an EE instance whose doubles accumulators alone exceed 128 MiB
    P2 = make_problem("EE", 20, 120, 40, seed=73, n_roots=1, x=0.5, scale=0.05)
    h2 = adc.Handle("EE", 20, 120, P2.eps, P2.L, 1, x=P2.x)
    Y2 = torch.zeros((1, h2.dim), dtype=torch.complex128, device="cuda")
    rc, S2 = _noalloc(h2, Y2, "fp64")
    assert rc == -7
    assert torch.isnan(S2).all().item()   # nothing was written
    assert b"scratch" in h._lib.adc_strerror(-7)
