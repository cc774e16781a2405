"""Seeded synthetic inputs: determinism, structure, and the batched draw."""
import numpy as np

from adcgen import c4_draw, config_problem, make_problem, make_L


def test_L_is_hermitian_and_scaled():
    P = make_problem("EE", 3, 7, 40, seed=3)
    L = P.L
    assert np.abs(L - L.conj().transpose(0, 2, 1)).max() == 0.0
    # scale s_Q = 0.05 exp(-Q/30): the diagonal of L^Q is s_Q * sqrt(2) * N(0,1)
    s = 0.05 * np.exp(-np.arange(40) / 30.0)
    ratio = np.sqrt(np.mean(np.abs(L) ** 2, axis=(1, 2))) / s
    assert np.all((ratio > 0.6) & (ratio < 1.4))
    assert np.all(np.diff(P.eps[:3]) >= 0) and np.all(np.diff(P.eps[3:]) >= 0)
    assert P.eps[:3].max() < -0.3 + 1e-12 and P.eps[3:].min() > 0.1 - 1e-12


def test_chunked_draw_equals_whole_draw():
    rng = np.random.default_rng(5)
    L1 = make_L(rng, 50, 6, chunk=7)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 6, 6))
    Y = rng.standard_normal((50, 6, 6))
    G = (X + 1j * Y) / np.sqrt(2)
    s = 0.05 * np.exp(-np.arange(50) / 30.0)
    L2 = s[:, None, None] * (G + G.conj().transpose(0, 2, 1)) / np.sqrt(2)
    assert np.array_equal(L1, L2)


def test_config_determinism():
    a = config_problem("C1")
    b = config_problem("C1")
    assert np.array_equal(a.L, b.L) and np.array_equal(a.eps, b.eps)
    assert (a.kind, a.o, a.v, a.n_chol, a.n_roots, a.x) == ("EE", 6, 18, 80, 4, 1.0)


def test_c4_draw_statistics():
    d = c4_draw()
    kinds = [t[0] for t in d]
    assert (kinds.count("EE"), kinds.count("IP"), kinds.count("EA")) == (22, 21, 21)
    assert sum(t[4] for t in d) == 648
    assert d[0][:5] == ("EE", 29, 231, 1560, 14)
