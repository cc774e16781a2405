"""GPU parity of the EE sigma build and Davidson solver against the oracle.

Bar: FP64 sigma max|dS| / max|S| <= 1e-12 (accumulation order differs from
the oracle's); eigenvalues within 1e-8 Eh of the oracle's converged values.
"""
import numpy as np
import pytest

from adcgen import config_problem, make_problem
from oracle.adc_terms import Ints, diag0, dims
from oracle.adc_terms import sigma as osigma
from oracle.davidson import davidson as odavidson

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _handle(P, **kw):
    return adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, **kw)


def _rand(rng, k, dim):
    return rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))


@pytest.mark.parametrize("o,v,N,x,seed", [(3, 6, 20, 1.0, 1), (4, 7, 30, 0.5, 2), (2, 5, 10, 0.0, 3),
                                          (5, 9, 40, 1.0, 4), (1, 6, 10, 1.0, 5), (6, 13, 50, 0.7, 6)])
def test_ee_sigma_fp64_matches_oracle(o, v, N, x, seed):
    print(f"case EE o={o} v={v} N={N} x={x} seed={seed}", flush=True)
    P = make_problem("EE", o, v, N, seed=seed, x=x, scale=0.2)
    h = _handle(P)
    rng = np.random.default_rng(seed)
    Y = _rand(rng, 3, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, o), "EE", x, Y)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err
    h.close()


def test_ee_sigma_hermitian_and_affine_in_x():
    P = make_problem("EE", 8, 40, 120, seed=7, x=1.0)
    rng = np.random.default_rng(7)
    h1 = _handle(P)
    Y = torch.from_numpy(_rand(rng, 2, h1.dim)).cuda()
    Z = torch.from_numpy(_rand(rng, 2, h1.dim)).cuda()
    SY, SZ = h1.sigma(Y), h1.sigma(Z)
    a = (Z.conj() * SY).sum(1)
    b = (SZ.conj() * Y).sum(1)
    assert (a - b).abs().max().item() <= 1e-13 * SY.abs().max().item() * Z.abs().sum().item()
    P.x = 0.0
    h0 = _handle(P)
    P.x = 0.5
    hh = _handle(P)
    Sh = hh.sigma(Y)
    S0 = h0.sigma(Y)
    assert (Sh - 0.5 * (S0 + SY)).abs().max().item() <= 1e-12 * SY.abs().max().item()


def test_c1_sigma_and_davidson():
    P = config_problem("C1")
    h = _handle(P)
    rng = np.random.default_rng(11)
    ints = Ints(P.eps, P.L, P.o)
    Y = _rand(rng, 4, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(ints, "EE", P.x, Y)
    assert np.abs(S - ref).max() / np.abs(ref).max() < 1e-12
    out = h.davidson()
    n1 = dims("EE", P.o, P.v)[0]
    d = np.concatenate([diag0(ints, "EE", 1), diag0(ints, "EE", 2)])
    from oracle.adc_terms import m11_block
    M11 = sum(m11_block(ints, "EE", k) for k in range(3)) + P.x * m11_block(ints, "EE", 3)
    w, X, rn, it, conv = odavidson(lambda Z: osigma(ints, "EE", P.x, Z), d, np.diag(M11).real, 4, tol=1e-9)
    print("gpu", out["omega"], out["resnorm"], out["iters"], "oracle", w)
    assert out["converged"].all()
    assert np.abs(out["omega"] - w).max() < 1e-8


def test_one_electron_ee_is_exact():
    P = make_problem("EE", 1, 8, 12, seed=9, n_roots=3, scale=0.3)
    from oracle.isr import antisym_integrals
    g = antisym_integrals(P.L)
    exact = np.linalg.eigvalsh(np.diag(P.eps[1:]) - g[1:, 0, 1:, 0]) - P.eps[0]
    h = _handle(P, conv_tol=1e-10)
    out = h.davidson()
    assert np.abs(out["omega"] - exact[:3]).max() < 1e-9


def test_ee_sigma_fp32_and_mixed_davidson():
    """FP32 MFMA contractions (fp32 operands and accumulation): relative sigma
    error of a few fp32 ulps times sqrt(K); eigenvalues after the FP64
    refinement equal the FP64 path's."""
    P = config_problem("C1")
    rng = np.random.default_rng(12)
    h = _handle(P, precision="fp32")
    Y = _rand(rng, 4, h.dim)
    S32 = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, P.o), "EE", P.x, Y)
    err = np.abs(S32 - ref).max() / np.abs(ref).max()
    print("fp32 rel err", err)
    assert err < 1e-6
    assert err > 1e-12  # really ran in reduced precision
    out = h.davidson()
    h64 = _handle(P, precision="fp64")
    out64 = h64.davidson()
    assert out["converged"].all()
    assert np.abs(out["omega"] - out64["omega"]).max() < 1e-8


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_split_bf16_sigma_and_mixed_davidson(kind):
    """Split-bf16 contractions: x = hi + lo with hi, lo bf16 (16 mantissa bits
    together), three products per real MAC in fp32; relative sigma error of a
    few 2^-17 times sqrt(K).  After the FP64 refinement the eigenvalues equal
    the FP64 path's."""
    P = make_problem(kind, 6, 18, 80, seed=13, n_roots=4, x=1.0)
    rng = np.random.default_rng(13)
    h = _handle(P, precision="split_bf16")
    Y = _rand(rng, 3, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, P.o), kind, P.x, Y)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    print(kind, "split-bf16 rel err", err)
    assert 1e-12 < err < 1e-5
    out = h.davidson()
    out64 = _handle(P, precision="fp64").davidson()
    assert out["converged"].all()
    assert np.abs(out["omega"] - out64["omega"]).max() < 1e-8


@pytest.mark.parametrize("kind,v,budget", [("EE", 40, 0), ("EE", 40, 1 << 20), ("EA", 40, 1 << 20),
                                            ("EE", 37, 3 << 19), ("EA", 53, 1 << 21)])
def test_split_bf16_ladder_blocks(kind, v, budget):
    """The split-bf16 particle-particle ladder over several a-blocks: with the
    default workspace only the Hermitian upper part of <ab||cd> is assembled
    (grouped over exact-range blocks) and mirrored; a workspace of 1-2 MiB
    forces many row groups, each assembling its upper part, mirroring its
    diagonal block and contracting the conjugate transpose of its rows into
    the later columns.  All equal the FP64 ladder to split-bf16 accuracy."""
    P = make_problem(kind, 4, v, 120, seed=41, n_roots=2, x=1.0)
    print(f"case split-bf16 ladder {kind} v={v} budget={budget}", flush=True)
    h = _handle(P, precision="split_bf16", mem_budget=budget)
    rng = np.random.default_rng(41)
    Y = torch.from_numpy(_rand(rng, 3, h.dim)).cuda()
    S64 = h.sigma_term("ladder", Y, precision="fp64").cpu().numpy()
    Sbf = h.sigma_term("ladder", Y, precision="split_bf16").cpu().numpy()
    err = np.abs(Sbf - S64).max() / np.abs(S64).max()
    print("ladder split-bf16 rel err", err)
    # two split-bf16 products in a row (assembly, then contraction): about
    # 2 * 2^-16 relative to the output scale
    assert 1e-12 < err < 3e-5


@pytest.mark.parametrize("o,v,x", [(2, 20, 1.0), (3, 70, 1.0), (3, 67, 0.5), (2, 66, 0.0)])
def test_split_bf16_ee_pair_layouts(o, v, x):
    """Split-bf16 EE sigma over the shapes that pick different forms of the
    doubles' planes: few occupied pairs (P_o * v < 32: the unpacked copies are
    split), one or two 64-wide virtual tiles with odd and even v (planes of the
    pair-packed doubles and of the ring layout written straight from the
    packed vectors), and x = 0 (no ring term)."""
    print(f"case split-bf16 EE o={o} v={v} x={x}", flush=True)
    P = make_problem("EE", o, v, 60, seed=47, n_roots=2, x=x, scale=0.2)
    h = _handle(P, precision="split_bf16")
    rng = np.random.default_rng(47)
    Y = _rand(rng, 2, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, o), "EE", x, Y)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    print("split-bf16 rel err", err)
    assert 1e-12 < err < 1e-5
    h.close()
