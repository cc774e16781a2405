"""Pins of O1 (numerical ISR) against facts fixed outside it.

* E(2), E(3) of the RS series vs the closed-form spin-orbital MP2 and the
  three-term MP3 energies;
* first-order EE singles block == CIS matrix; IP/EA Koopmans (M11(1) = 0);
* one electron (o = 1): Phi_0 is exact, so the EE spectrum equals
  eigh(eps_a delta_ab - <a0||b0>) - eps_0 and the IP energy is -eps_0;
* order structure against FCI: the ADC(n) eigenvalue error vanishes as
  lam^(n+1), and at x = 1/2 the lam^3 error coefficient is half that of x = 0;
* the MP amplitudes used by O2 equal the coefficients of O1's ground state.
"""
import numpy as np
import pytest

from adcgen import make_problem
from oracle.adc_terms import Ints
from oracle.fci import FCI
from oracle.isr import ISR, antisym_integrals, manifold, pairs


def _tensors(eps, g, o):
    e = eps
    n = len(e)
    O, V = slice(0, o), slice(o, n)
    D = e[:o, None, None, None] + e[None, :o, None, None] - e[None, None, o:, None] - e[None, None, None, o:]
    return O, V, D


def _mp2(eps, g, o):
    O, V, D = _tensors(eps, g, o)
    return 0.25 * np.sum(np.abs(g[O, O, V, V]) ** 2 / D)


def _mp3(eps, g, o):
    # Textbook spin-orbital third-order energy: particle ladder, hole ladder
    # and ring, each <0|V R V R V|0>.
    O, V, D = _tensors(eps, g, o)
    a = np.einsum("ijab,abcd,cdij,ijab,ijcd->", g[O, O, V, V], g[V, V, V, V], g[V, V, O, O], 1 / D, 1 / D)
    b = np.einsum("ijab,klij,abkl,ijab,klab->", g[O, O, V, V], g[O, O, O, O], g[V, V, O, O], 1 / D, 1 / D)
    c = np.einsum("ijab,kbcj,acik,ijab,ikac->", g[O, O, V, V], g[O, V, V, O], g[V, V, O, O], 1 / D, 1 / D)
    return a / 8 + b / 8 + c


@pytest.mark.parametrize("kind,o,v,seed", [("EE", 2, 4, 1), ("IP", 3, 4, 2), ("EA", 3, 5, 3)])
def test_ground_state_energies(kind, o, v, seed):
    P = make_problem(kind, o, v, 20, seed=seed, scale=0.3)
    g = antisym_integrals(P.L)
    isr = ISR(kind, P.eps, g, o)
    assert abs(isr.E0[0] - P.eps[:o].sum()) < 1e-13
    assert abs(isr.E0[2] - _mp2(P.eps, g, o)) < 1e-13
    assert abs(isr.E0[3] - _mp3(P.eps, g, o)) < 1e-13


def test_integrals_antisymmetry_and_hermiticity():
    P = make_problem("EE", 3, 4, 15, seed=4)
    g = antisym_integrals(P.L)
    scale = np.abs(g).max()
    assert np.abs(g + g.transpose(1, 0, 2, 3)).max() <= 1e-15 * scale
    assert np.abs(g + g.transpose(0, 1, 3, 2)).max() <= 1e-15 * scale
    assert np.abs(g.conj() - g.transpose(2, 3, 0, 1)).max() <= 1e-15 * scale


def test_first_order_singles_blocks():
    o, v = 3, 5
    P = make_problem("EE", o, v, 15, seed=5, scale=0.3)
    g = antisym_integrals(P.L)
    isr = ISR("EE", P.eps, g, o)
    O, V = slice(0, o), slice(o, o + v)
    cis = np.einsum("ajib->iajb", g[V, O, O, V]).reshape(o * v, o * v)
    d = (P.eps[None, o:] - P.eps[:o, None]).reshape(-1)
    assert np.abs(isr.block("11", 0) - np.diag(d)).max() < 1e-14
    assert np.abs(isr.block("11", 1) - cis).max() < 1e-13
    for kind, diag in [("IP", -P.eps[:o]), ("EA", P.eps[o:])]:
        isr2 = ISR(kind, P.eps, g, o)
        assert np.abs(isr2.block("11", 0) - np.diag(diag)).max() < 1e-14
        assert np.abs(isr2.block("11", 1)).max() < 1e-13


def test_one_electron_closed_forms():
    o, v = 1, 6
    P = make_problem("EE", o, v, 15, seed=6, scale=0.4)
    g = antisym_integrals(P.L)
    hvv = np.diag(P.eps[1:]) - g[1:, 0, 1:, 0]
    exact = np.linalg.eigvalsh(hvv) - P.eps[0]
    isr = ISR("EE", P.eps, g, o)
    for x in (0.0, 0.5, 1.0):
        assert np.abs(np.linalg.eigvalsh(isr.matrix(x)) - exact).max() < 1e-13
    ints = Ints(P.eps, P.L, o)
    from oracle.adc_terms import dense_matrix
    assert np.abs(np.linalg.eigvalsh(dense_matrix(ints, "EE", 1.0)) - exact).max() < 1e-13
    isr_ip = ISR("IP", P.eps, g, o)
    assert abs(np.linalg.eigvalsh(isr_ip.matrix(1.0))[0] + P.eps[0]) < 1e-13


def _lowest_error(isr, fci, kind, x, lam):
    w = fci.omegas(kind, lam)
    e = np.linalg.eigvalsh(isr.matrix(x, lam))[0]
    return abs(w[np.argmin(np.abs(w - e))] - e)


@pytest.mark.parametrize("kind,o,v,seed", [("EE", 2, 4, 7), ("IP", 3, 4, 8), ("EA", 2, 5, 9)])
def test_order_structure_against_fci(kind, o, v, seed):
    P = make_problem(kind, o, v, 20, seed=seed, scale=0.3)
    g = antisym_integrals(P.L)
    isr = ISR(kind, P.eps, g, o)
    fci = FCI(P.eps, g, o)
    lams = [0.05, 0.025]
    e2 = [_lowest_error(isr, fci, kind, 0.0, l) for l in lams]
    e3 = [_lowest_error(isr, fci, kind, 1.0, l) for l in lams]
    eh = [_lowest_error(isr, fci, kind, 0.5, l) for l in lams]
    slope2 = np.log2(e2[0] / e2[1])
    slope3 = np.log2(e3[0] / e3[1])
    assert abs(slope2 - 3.0) < 0.2, slope2
    assert abs(slope3 - 4.0) < 0.3, slope3
    assert abs(eh[1] / e2[1] - 0.5) < 0.05


def test_amplitudes_are_the_ground_state_coefficients():
    o, v = 3, 5
    P = make_problem("EE", o, v, 20, seed=10, scale=0.3)
    g = antisym_integrals(P.L)
    isr = ISR("EE", P.eps, g, o)
    c1, c2, _ = manifold("EE", o, v)
    ints = Ints(P.eps, P.L, o)

    def coef(strings, vec):
        phi = np.zeros(len(isr.fs.sector(o)), complex)
        phi[isr.i0] = 1
        return np.array([np.vdot(isr.fs.apply_string(s, phi, o)[0], vec) for s in strings])

    def pack(t):
        return np.array([t[i, j, a, b] for (i, j) in pairs(o) for (a, b) in pairs(v)])

    assert np.abs(coef(c2, isr.psi_raw[1]) - pack(ints.amp("t"))).max() < 1e-14
    assert np.abs(coef(c2, isr.psi_raw[2]) - pack(ints.amp("t2"))).max() < 1e-14
    assert np.abs(coef(c1, isr.psi_raw[2]) - ints.amp("ts").reshape(-1)).max() < 1e-14
