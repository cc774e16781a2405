"""Pins of the frozen-natural-spinor oracle (Section 2.4, eqs. 25-32) against
what the mathematics fixes, independently of its formulas:

* eq. 25 is the virtual block of the second-order one-particle density,
  <psi1| a+_b a_a |psi1>, with psi1 the first-order wavefunction that O1
  builds in determinant space; its trace counts two electrons per doubly
  excited determinant;
* the ADC(2) state density (eq. 31, derived here) equals <Psi|a+_b a_a|Psi>
  for Psi made of O1's zeroth-order intermediate states, EE and EA;
* eqs. 26-30: B has orthonormal columns and makes the Fock block diagonal with
  ascending e~; the kept natural spinors are those at or above eta_crit;
* the Cholesky vectors of the truncated problem give the integrals that the
  rule for a change of spinor basis gives (bra indices conjugated);
* without truncation the ADC(3) spectrum is unchanged, and eq. 32 then adds
  nothing.
"""
import numpy as np
import pytest

from adcgen import make_problem
from oracle.adc_terms import Ints, dense_matrix, dims
from oracle.fns import corrected, mp2_vv_density, natural_spinors, state_vv_density, transform_problem, truncate
from oracle.isr import ISR, antisym_integrals


def _vv_expect(fs, psi, o, v, N):
    """<psi| a+_b a_a |psi> for a, b virtual, psi a vector of sector N."""
    D = np.zeros((v, v), dtype=np.complex128)
    for a in range(v):
        t = fs.op("a", o + a, N) @ psi
        for b in range(v):
            D[a, b] = np.vdot(psi, fs.op("c", o + b, N - 1) @ t)
    return D


@pytest.mark.parametrize("o,v,seed", [(2, 4, 1), (3, 5, 2), (4, 5, 3)])
def test_mp2_density_is_the_second_order_density(o, v, seed):
    P = make_problem("EE", o, v, 12, seed=seed, scale=0.3)
    isr = ISR("EE", P.eps, antisym_integrals(P.L), o)
    ints = Ints(P.eps, P.L, o)
    D = mp2_vv_density(P.eps, ints.g("vvoo"), o)
    psi1 = np.asarray(isr.psi_raw[1]).reshape(-1)
    ref = _vv_expect(isr.fs, psi1, o, v, o)
    assert np.abs(D - ref).max() < 1e-14
    assert np.abs(D - D.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(D).min() > -1e-15
    t = ints.amp("t")
    assert abs(np.trace(D).real - 0.5 * np.sum(np.abs(t) ** 2)) < 1e-14


@pytest.mark.parametrize("kind,o,v,seed", [("EE", 3, 4, 4), ("EE", 2, 5, 5), ("EA", 3, 4, 6), ("EA", 2, 5, 7)])
def test_state_density_from_zeroth_order_states(kind, o, v, seed):
    P = make_problem(kind, o, v, 12, seed=seed, scale=0.3)
    isr = ISR(kind, P.eps, antisym_integrals(P.L), o)
    n1, n2 = dims(kind, o, v)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(n1 + n2) + 1j * rng.standard_normal(n1 + n2)
    X /= np.linalg.norm(X)
    psi = isr.states[0] @ X                     # zeroth-order intermediate states
    Nt = o + (1 if kind == "EA" else 0)
    ref = _vv_expect(isr.fs, psi, o, v, Nt)
    D = state_vv_density(kind, o, v, X)
    assert np.abs(D - ref).max() < 1e-14
    # one electron more in the virtuals for EA, one for EE singles, two for EE doubles
    w1 = np.sum(np.abs(X[:n1]) ** 2)
    expect = (1.0 if kind == "EA" else w1) + (1.0 if kind == "EA" else 2.0) * np.sum(np.abs(X[n1:]) ** 2)
    assert abs(np.trace(D).real - expect) < 1e-14


def test_truncation_basis():
    P = make_problem("EE", 4, 14, 40, seed=8, scale=0.3)
    ints = Ints(P.eps, P.L, P.o)
    D = mp2_vv_density(P.eps, ints.g("vvoo"), P.o)
    eta, V = natural_spinors(D)
    assert (np.diff(eta) <= 0).all() and abs(eta.sum() - np.trace(D).real) < 1e-14
    eta_crit = 0.5 * (eta[8] + eta[9])
    B, et, eta2 = truncate(P.eps, P.o, D, eta_crit)
    assert B.shape == (14, 9)
    assert np.abs(B.conj().T @ B - np.eye(9)).max() < 1e-14
    F = B.conj().T @ np.diag(P.eps[P.o:]) @ B
    assert np.abs(F - np.diag(et)).max() < 1e-13 and (np.diff(et) > 0).all()
    # the kept space is the span of the 9 natural spinors of largest occupation
    Pk = V[:, :9] @ V[:, :9].conj().T
    assert np.abs(Pk @ B - B).max() < 1e-13


def test_cholesky_vectors_follow_the_spinors():
    """With any orthonormal B, <a'b'||c'd'> from the transformed vectors equals
    sum conj(B_aa') conj(B_bb') B_cc' B_dd' <ab||cd> (likewise for the blocks
    with occupied indices)."""
    P = make_problem("EE", 3, 6, 15, seed=9, scale=0.3)
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    B = Q[:, :4]
    e2, L2 = transform_problem(P.eps, P.L, 3, B, np.array([0.5, 1.0, 1.5, 2.0]))
    g = antisym_integrals(P.L)
    g2 = antisym_integrals(L2)
    # basis change of all spinors: identity on the occupied, B on the virtuals
    U = np.zeros((9, 7), dtype=np.complex128)
    U[:3, :3] = np.eye(3)
    U[3:, 3:] = B
    ref = np.einsum("pa,qb,rc,sd,pqrs->abcd", U.conj(), U.conj(), U, U, g)
    assert np.abs(g2 - ref).max() < 1e-13
    assert np.abs(L2 - L2.conj().transpose(0, 2, 1)).max() < 1e-15


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_no_truncation_keeps_the_spectrum(kind):
    P = make_problem(kind, 3, 6, 15, seed=10, scale=0.3)
    ints = Ints(P.eps, P.L, P.o)
    D = mp2_vv_density(P.eps, ints.g("vvoo"), P.o)
    B, et, _ = truncate(P.eps, P.o, D, 0.0)
    e2, L2 = transform_problem(P.eps, P.L, P.o, B, et)
    w = np.linalg.eigvalsh(dense_matrix(ints, kind, 1.0))
    w2 = np.linalg.eigvalsh(dense_matrix(Ints(e2, L2, P.o), kind, 1.0))
    assert np.abs(w - w2).max() < 1e-12
    w0 = np.linalg.eigvalsh(dense_matrix(ints, kind, 0.0))
    assert np.abs(corrected(w2[:3], w0[:3], w0[:3]) - w[:3]).max() < 1e-12
