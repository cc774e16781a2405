"""Parity at the full benchmark sizes, where the oracle cannot form the whole
matrix: on outputs it can compute, and through properties that hold at any
size.

* C2 (EE, the timed workload): the complete sigma build for one trial vector
  whose singles part is zero (only the M12 and M22 blocks of the oracle),
  and for a general vector (every block, M11 included, from the oracle's
  matrix-free sigma), FP64, FP32 and split-bf16, in the launch configuration
  bench.py times;
* C3-EA: sampled rows of the particle-particle ladder, each <ab||cd> row formed
  by the oracle from L on its own; Hermiticity of the whole sigma;
* C3-IP: Hermiticity of the whole sigma.
"""
import numpy as np
import pytest

from adcgen import config_problem
from oracle.adc_terms import Ints, dims, sigma, sigma_block

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _herm_check(h, rng):
    """FP64 <Z, M Y> - <M Z, Y>, relative to max|MY| sum|Z|."""
    Y = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    Z = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    SY, SZ = h.sigma(Y, precision="fp64"), h.sigma(Z, precision="fp64")
    a = (Z.conj() * SY).sum(1)
    b = (SZ.conj() * Y).sum(1)
    return ((a - b).abs().max() / (SY.abs().max() * Z.abs().sum())).item()


def test_c2_full_sigma_doubles_input():
    P = config_problem("C2")
    print("case C2 EE full sigma, zero-singles trial vector", flush=True)
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    n1, n2 = dims("EE", P.o, P.v)
    rng = np.random.default_rng(22)
    Y = np.zeros((1, n1 + n2), complex)
    Y[0, n1:] = rng.standard_normal(n2) + 1j * rng.standard_normal(n2)
    S64 = h.sigma(torch.from_numpy(Y).cuda(), precision="fp64").cpu().numpy()
    S32 = h.sigma(torch.from_numpy(Y).cuda(), precision="fp32").cpu().numpy()
    Sbf = h.sigma(torch.from_numpy(Y).cuda(), precision="split_bf16").cpu().numpy()
    ints = Ints(P.eps, P.L, P.o)
    Y2 = Y[:, n1:]
    ref1 = sigma_block(ints, "EE", "12", 1, Y2) + P.x * sigma_block(ints, "EE", "12", 2, Y2)
    ref2 = sigma_block(ints, "EE", "22", 0, Y2) + P.x * sigma_block(ints, "EE", "22", 1, Y2)
    ref = np.concatenate([ref1, ref2], axis=1)
    e64 = np.abs(S64 - ref).max() / np.abs(ref).max()
    e32 = np.abs(S32 - ref).max() / np.abs(ref).max()
    ebf = np.abs(Sbf - ref).max() / np.abs(ref).max()
    print("C2 rel err fp64", e64, "fp32", e32, "split-bf16", ebf)
    assert e64 < 1e-12
    assert e32 < 1e-6
    # split-bf16 (the arithmetic bench.py times): 16 significant bits per
    # operand, one split product per term (see the ladder test below for two)
    assert 1e-12 < ebf < 1e-5


def test_c2_full_sigma_general_vector():
    """Every block of M (eq. 11), singles included, at the benchmark size."""
    P = config_problem("C2")
    print("case C2 EE full sigma, general trial vector", flush=True)
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    rng = np.random.default_rng(23)
    Y = rng.standard_normal((1, h.dim)) + 1j * rng.standard_normal((1, h.dim))
    Yd = torch.from_numpy(Y).cuda()
    S64 = h.sigma(Yd, precision="fp64").cpu().numpy()
    S32 = h.sigma(Yd, precision="fp32").cpu().numpy()
    Sbf = h.sigma(Yd, precision="split_bf16").cpu().numpy()
    h.close()
    ref = sigma(Ints(P.eps, P.L, P.o), "EE", P.x, Y)
    e64 = np.abs(S64 - ref).max() / np.abs(ref).max()
    e32 = np.abs(S32 - ref).max() / np.abs(ref).max()
    ebf = np.abs(Sbf - ref).max() / np.abs(ref).max()
    print("C2 general vector rel err fp64", e64, "fp32", e32, "split-bf16", ebf)
    assert e64 < 1e-12
    assert e32 < 1e-6
    # the particle-particle ladder chains two split products (reading of the
    # tolerances: about 2 * 2^-16 of the output scale at most)
    assert 1e-12 < ebf < 3e-5


def test_c3_ea_ladder_rows_and_hermiticity():
    P = config_problem("C3-EA")
    print("case C3-EA ladder rows + hermiticity", flush=True)
    h = adc.Handle("EA", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, precision="fp32", mem_budget=32 << 30)
    rng = np.random.default_rng(32)
    Y = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    S = h.sigma_term("ladder", Y, precision="fp64").cpu().numpy()
    Sbf = h.sigma_term("ladder", Y, precision="split_bf16").cpu().numpy()
    Yh = Y.cpu().numpy()
    o, v = P.o, P.v
    Lvv = P.L[:, o:, o:]
    iu = np.triu_indices(v, 1)
    Pv = len(iu[0])
    worst = worst_bf = 0.0
    for (i, a, b) in [(0, 0, 1), (7, 3, 250), (59, 398, 399), (31, 100, 101), (12, 5, 377), (44, 250, 251)]:
        W = np.einsum("Qc,Qd->cd", Lvv[:, a, :], Lvv[:, b, :])
        g = (W - W.T)[iu]                       # <ab||cd>, c<d
        p = a * (2 * v - a - 1) // 2 + (b - a - 1)
        ref = P.x * (Yh[:, v + i * Pv: v + (i + 1) * Pv] @ g)
        got = S[:, v + i * Pv + p]
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
        worst_bf = max(worst_bf, np.abs(Sbf[:, v + i * Pv + p] - ref).max() / np.abs(ref).max())
    print("C3-EA ladder sampled rel err", worst, "split-bf16", worst_bf)
    assert worst < 1e-12
    # two split-bf16 products in a row (the <ab||cd> assembly over N = 2400,
    # then the contraction over P_v = 79,800): each operand split carries up
    # to 2^-16 relative error and the three-product form drops lo*lo'
    # (<= 2^-16), so each product term is off by ~2^-16 of its size at
    # random; the two chained products give ~2 * 2^-16 = 3e-5 relative to the
    # output scale
    assert worst_bf < 3e-5
    assert _herm_check(h, rng) < 1e-13


def test_c3_ip_hermiticity():
    P = config_problem("C3-IP")
    print("case C3-IP hermiticity", flush=True)
    h = adc.Handle("IP", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    assert _herm_check(h, np.random.default_rng(31)) < 1e-13
