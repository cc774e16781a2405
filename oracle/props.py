"""ISR one-particle properties of EE states: transition density matrices and
excited-state density matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Section 2.2 (properties in the ISR formulation): with f^I_pq =
<Psi~_I| c+_p c_q |Psi_0> and g^IJ_pq = <Psi~_I| c+_p c_q |Psi~_J>, the
transition density of state K (eigenvector Y_K) is rho^{0->K}_pq = Y_K^* f_pq
and its density is rho^K_pq = Y_K^* g_pq Y_K; a one-particle operator d gives
T_{0->K} = sum_pq d_pq rho^{0->K}_pq and D_K = sum_pq d_pq rho^K_pq.  The
ground-state density enters at second order, rho = rho(0) + rho(2).

The paper prints neither f nor g, nor their orders.  Readings (stated here and
pinned to O1, which builds f and g as series in determinant space):
* f through first order (the zeroth-order term and the first-order term of
  the MP ground state and of the intermediate states);
* the excited-state density as the zeroth-order ISR density of Y_K (the order
  the paper uses for its state densities) with the ground-state correlation
  density rho(2) added: rho^K = Y_K^* g(0) Y_K + rho_GS(2) (the shifted form
  Y^* G Y + D_0 with D_0 through second order).

Closed forms (indices: i j k l occupied, a b c d virtual; Y singles Y_ia and
doubles Y_ijab, t first-order doubles, ts second-order singles; doubles
extended antisymmetrically in each pair):
  rho^{0->K}:  vo  (a,i) = conj(Y_ia)
               ov  (j,b) = sum_ia conj(Y_ia) t_ijab
               vv  (c,d) = 1/2 sum_ijb conj(Y_ijcb) t_ijdb
               oo  (k,l) = -1/2 sum_jab conj(Y_ljab) t_kjab
  rho^K(0):    vv  (c,d) = sum_i conj(Y_ic) Y_id + 1/2 sum_ije conj(Y_ijce) Y_ijde
               oo  (k,l) = delta_kl |Y|^2 - sum_a conj(Y_la) Y_ka - 1/2 sum_jab conj(Y_ljab) Y_kjab
               ov  (k,d) = sum_ia conj(Y_ia) Y_ikad,   vo = its conjugate transpose
  rho_GS(2):   vv  (c,d) = 1/2 sum_ijb conj(t_ijcb) t_ijdb
               oo  (k,l) = -1/2 sum_jab conj(t_ljab) t_kjab
               ov  (k,d) = ts_kd,   vo = its conjugate transpose
Matrices are [n][n] over all spinors, occupied first, element [p][q] for
c+_p c_q.
"""
from __future__ import annotations

import numpy as np

from oracle.adc_terms import dims, packed_index


def _split(o: int, v: int, Y: np.ndarray):
    """Packed EE vector -> singles [o][v] and antisymmetric doubles [o][o][v][v]."""
    n1, _ = dims("EE", o, v)
    S = np.asarray(Y[:n1], dtype=np.complex128).reshape(o, v)
    T = np.zeros((o, o, v, v), dtype=np.complex128)
    i, j, a, b = packed_index("EE", 2, o, v)
    X = np.asarray(Y[n1:], dtype=np.complex128)
    T[i, j, a, b] = X
    T[j, i, a, b] = -X
    T[i, j, b, a] = -X
    T[j, i, b, a] = X
    return S, T


def transition_density(o: int, v: int, t: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """rho^{0->K} through first order for the packed EE vector Y."""
    S, T = _split(o, v, Y)
    n = o + v
    R = np.zeros((n, n), dtype=np.complex128)
    R[o:, :o] = np.conj(S).T
    R[:o, o:] = np.einsum("ia,ijab->jb", np.conj(S), t)
    R[o:, o:] = 0.5 * np.einsum("ijcb,ijdb->cd", np.conj(T), t)
    R[:o, :o] = -0.5 * np.einsum("ljab,kjab->kl", np.conj(T), t)
    return R


def ground_state_density2(o: int, v: int, t: np.ndarray, ts: np.ndarray) -> np.ndarray:
    """rho_GS(2): the second-order part of the ground-state density."""
    n = o + v
    R = np.zeros((n, n), dtype=np.complex128)
    R[o:, o:] = 0.5 * np.einsum("ijcb,ijdb->cd", np.conj(t), t)
    R[:o, :o] = -0.5 * np.einsum("ljab,kjab->kl", np.conj(t), t)
    R[:o, o:] = ts
    R[o:, :o] = np.conj(ts).T
    return R


def state_density0(o: int, v: int, Y: np.ndarray) -> np.ndarray:
    """rho^K(0) = Y^* g(0) Y for the packed EE vector Y (not normalised)."""
    S, T = _split(o, v, Y)
    n = o + v
    nrm = np.vdot(Y, Y).real
    R = np.zeros((n, n), dtype=np.complex128)
    R[o:, o:] = np.einsum("ic,id->cd", np.conj(S), S) + 0.5 * np.einsum("ijce,ijde->cd", np.conj(T), T)
    R[:o, :o] = (nrm * np.eye(o) - np.einsum("la,ka->kl", np.conj(S), S)
                 - 0.5 * np.einsum("ljab,kjab->kl", np.conj(T), T))
    R[:o, o:] = np.einsum("ia,ikad->kd", np.conj(S), T)
    R[o:, :o] = np.conj(R[:o, o:]).T
    return R


def state_density(o: int, v: int, t: np.ndarray, ts: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """rho^K = rho^K(0) + rho_GS(2) for a normalised Y."""
    return state_density0(o, v, Y) + ground_state_density2(o, v, t, ts)
