"""Pins of the ISR property oracle (Section 2.2) to O1, which builds the
intermediate states and the MP ground state as series in determinant space:

* f^I_pq = <Psi~_I| c+_p c_q |Psi_0> at orders 0 and 1 equals the closed form
  of the transition density (for every unit vector Y = e_I);
* the zeroth-order state density equals <Psi|c+_p c_q|Psi> for Psi made of the
  zeroth-order intermediate states;
* the second-order ground-state density equals the lambda^2 coefficient of
  <Psi_0|c+_p c_q|Psi_0> for the normalised series Psi_0;
* sum rules: the state density has trace o and the correlation density
  trace 0.
"""
import numpy as np
import pytest

from adcgen import make_problem
from oracle.adc_terms import Ints, dims
from oracle.isr import ISR, antisym_integrals
from oracle.props import ground_state_density2, state_density, state_density0, transition_density


def _onebody(fs, p, q, vec, N):
    return fs.op("c", p, N - 1) @ (fs.op("a", q, N) @ vec)


def _series_expect(fs, bra, ket, n, N, orders):
    """sum_{m<=order} <bra^(m)| c+_p c_q |ket^(order-m)> for each order:
    bra, ket lists of [dimN x cols] arrays; returns [orders][cols_bra][cols_ket][n][n]."""
    out = []
    for od in orders:
        acc = None
        for m in range(od + 1):
            B, K = bra[m], ket[od - m]
            R = np.zeros((B.shape[1], K.shape[1], n, n), dtype=np.complex128)
            for p in range(n):
                for q in range(n):
                    R[:, :, p, q] = B.conj().T @ _onebody(fs, p, q, K, N)
            acc = R if acc is None else acc + R
        out.append(acc)
    return out


@pytest.mark.parametrize("o,v,seed", [(2, 4, 1), (3, 4, 2), (3, 5, 3)])
def test_transition_density_is_isr_f(o, v, seed):
    P = make_problem("EE", o, v, 12, seed=seed, scale=0.3)
    isr = ISR("EE", P.eps, antisym_integrals(P.L), o)
    n = o + v
    psi0 = [np.asarray(c).reshape(-1, 1) for c in isr.psi0]
    f0, f1 = _series_expect(isr.fs, isr.states, psi0, n, o, [0, 1])
    t = Ints(P.eps, P.L, o).amp("t")
    n1, n2 = dims("EE", o, v)
    for I in range(n1 + n2):
        e = np.zeros(n1 + n2)
        e[I] = 1.0
        # rho^{0->K} = Y^* f: for Y = e_I this is f^I itself
        ref = f0[I, 0] + f1[I, 0]
        assert np.abs(transition_density(o, v, t, e) - ref).max() < 1e-14, I


@pytest.mark.parametrize("o,v,seed", [(2, 4, 4), (3, 4, 5)])
def test_state_density_zeroth_order(o, v, seed):
    P = make_problem("EE", o, v, 12, seed=seed, scale=0.3)
    isr = ISR("EE", P.eps, antisym_integrals(P.L), o)
    n1, n2 = dims("EE", o, v)
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal(n1 + n2) + 1j * rng.standard_normal(n1 + n2)
    Y /= np.linalg.norm(Y)
    psi = isr.states[0] @ Y
    n = o + v
    ref = np.zeros((n, n), dtype=np.complex128)
    for p in range(n):
        for q in range(n):
            ref[p, q] = np.vdot(psi, _onebody(isr.fs, p, q, psi, o))
    R = state_density0(o, v, Y)
    assert np.abs(R - ref).max() < 1e-14
    assert abs(np.trace(R).real - o) < 1e-13


@pytest.mark.parametrize("o,v,seed", [(2, 4, 6), (3, 5, 7)])
def test_ground_state_density_second_order(o, v, seed):
    P = make_problem("EE", o, v, 12, seed=seed, scale=0.3)
    isr = ISR("EE", P.eps, antisym_integrals(P.L), o)
    psi0 = [np.asarray(c).reshape(-1, 1) for c in isr.psi0]
    n = o + v
    (g2,) = _series_expect(isr.fs, psi0, psi0, n, o, [2])
    ints = Ints(P.eps, P.L, o)
    R = ground_state_density2(o, v, ints.amp("t"), ints.amp("ts"))
    assert np.abs(R - g2[0, 0]).max() < 1e-14
    assert abs(np.trace(R)) < 1e-14
    Y = np.zeros(dims("EE", o, v)[0] + dims("EE", o, v)[1])
    Y[0] = 1.0
    assert abs(np.trace(state_density(o, v, ints.amp("t"), ints.amp("ts"), Y)).real - o) < 1e-13
