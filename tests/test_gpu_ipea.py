"""GPU parity of the IP and EA sigma builds and solvers against the oracle
(FP64: max|dS| / max|S| <= 1e-12; eigenvalues within 1e-8 Eh)."""
import numpy as np
import pytest

from adcgen import make_problem
from oracle.adc_terms import Ints, diag0, m11_block
from oracle.adc_terms import sigma as osigma
from oracle.davidson import davidson as odavidson

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _handle(P, **kw):
    return adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, **kw)


def _rand(rng, k, dim):
    return rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))


CASES = [("IP", 3, 6, 20, 1.0, 1), ("IP", 4, 7, 30, 0.5, 2), ("IP", 2, 5, 10, 0.0, 3), ("IP", 6, 11, 40, 1.0, 4),
         ("EA", 3, 6, 20, 1.0, 5), ("EA", 4, 7, 30, 0.5, 6), ("EA", 2, 5, 10, 0.0, 7), ("EA", 5, 12, 40, 1.0, 8),
         ("EA", 1, 6, 10, 1.0, 9), ("IP", 1, 5, 8, 1.0, 10)]


@pytest.mark.parametrize("kind,o,v,N,x,seed", CASES)
def test_sigma_fp64_matches_oracle(kind, o, v, N, x, seed):
    print(f"case {kind} o={o} v={v} N={N} x={x} seed={seed}", flush=True)
    P = make_problem(kind, o, v, N, seed=seed, x=x, scale=0.2)
    h = _handle(P)
    rng = np.random.default_rng(seed)
    Y = _rand(rng, 3, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, o), kind, x, Y)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err
    h.close()


@pytest.mark.parametrize("kind", ["IP", "EA"])
def test_hermitian(kind):
    P = make_problem(kind, 10, 50, 150, seed=21)
    rng = np.random.default_rng(21)
    h = _handle(P)
    Y = torch.from_numpy(_rand(rng, 2, h.dim)).cuda()
    Z = torch.from_numpy(_rand(rng, 2, h.dim)).cuda()
    SY, SZ = h.sigma(Y), h.sigma(Z)
    a = (Z.conj() * SY).sum(1)
    b = (SZ.conj() * Y).sum(1)
    assert (a - b).abs().max().item() <= 1e-13 * SY.abs().max().item() * Z.abs().sum().item()


@pytest.mark.parametrize("kind,o,v,N", [("IP", 8, 30, 100), ("EA", 6, 24, 90)])
def test_davidson_matches_oracle(kind, o, v, N):
    P = make_problem(kind, o, v, N, seed=31, n_roots=4, x=1.0)
    ints = Ints(P.eps, P.L, o)
    d = np.concatenate([diag0(ints, kind, 1), diag0(ints, kind, 2)])
    M11 = sum(m11_block(ints, kind, q) for q in range(4))
    w, X, rn, it, conv = odavidson(lambda Z: osigma(ints, kind, 1.0, Z), d, np.diag(M11).real, 4, tol=1e-9)
    h = _handle(P)
    out = h.davidson()
    print("gpu", out["omega"], out["iters"], "oracle", w, it)
    assert out["converged"].all()
    assert np.abs(out["omega"] - w).max() < 1e-8


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_tiny_memory_budget_gives_same_sigma(kind):
    """A 64 KiB budget forces one-row ladder batches, one-index chunks of the
    v^4 intermediates and splitting of every contraction whose operand copy
    exceeds 4096 elements; the result must still match the oracle."""
    P = make_problem(kind, 4, 9, 25, seed=41, x=0.8, scale=0.2)
    h = _handle(P, mem_budget=1 << 16)
    rng = np.random.default_rng(41)
    Y = _rand(rng, 2, h.dim)
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(P.eps, P.L, P.o), kind, P.x, Y)
    assert np.abs(S - ref).max() / np.abs(ref).max() < 1e-12
