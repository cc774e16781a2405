"""Frozen natural spinors: truncation of the virtual space and the transform
of the problem into the truncated basis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Section 2.4 (frozen natural spinors):

* eq. 25  MP2 virtual-virtual density
          D_ab = 1/2 sum_{c,i,j} <ac||ij> <ij||bc> / (e_ij^ac e_ij^bc),
          e_ij^ac = e_i + e_j - e_a - e_c;
* eq. 26  natural spinors: D V = V eta (eigenvectors V, occupations eta);
* eq. 27  keep the natural spinors with eta >= eta_crit (V~ = V T);
* eq. 28  Fock matrix of the virtual block in that basis, F~ = V~^H F V~
          (F = diag(e_vir): canonical reference);
* eq. 29  semicanonicalisation, F~ Z~ = Z~ e~;
* eq. 30  B = V~ Z~, the map from the canonical to the truncated virtuals:
          new virtual spinor a' = sum_a (spinor a) B_aa';
* eq. 31  state-specific density D^SS(k) = D^MP2 + D^state(k), the second
          term from the ADC(2) eigenvector of state k through the
          zeroth-order intermediate states (the expressions are not printed;
          this module derives them: see state_vv_density);
* eq. 32  correction omega(k) = omega_ADC(3)^FNS + omega_ADC(2)^canonical
          - omega_ADC(2)^FNS.

The Cholesky vectors follow the spinors (eq. 42 with the MO coefficients
C B): L'_a'b' = sum_ab conj(B_aa') L_ab B_bb', L'_ib' = sum_b L_ib B_bb',
L'_a'j = sum_a conj(B_aa') L_aj, L'_ij = L_ij.

Readings: the density convention is the one eq. 25 prints, D_ab =
<a+_b a_a> (the pins check this against the determinant-space expectation
value), so that the columns of V are the coefficients of the natural spinors
in the canonical virtuals; occupations are sorted in descending order and
the eigenvalues of F~ ascending.
"""
from __future__ import annotations

import numpy as np

from oracle.adc_terms import dims, packed_index


def mp2_vv_density(eps: np.ndarray, g_vvoo: np.ndarray, o: int) -> np.ndarray:
    """eq. 25 from <ac||ij> (g_vvoo[a,c,i,j]); <ij||bc> = conj(<bc||ij>)."""
    e_o, e_v = eps[:o], eps[o:]
    den = e_o[None, None, :, None] + e_o[None, None, None, :] - e_v[:, None, None, None] - e_v[None, :, None, None]
    t = g_vvoo / den                                   # <ac||ij> / e_ij^ac
    return 0.5 * np.einsum("acij,bcij->ab", t, np.conj(t))


def _antisym_doubles(kind: str, o: int, v: int, X2: np.ndarray) -> np.ndarray:
    """Packed doubles of one vector -> the tensor antisymmetric in each pair."""
    idx = packed_index(kind, 2, o, v)
    if kind == "EE":
        T = np.zeros((o, o, v, v), dtype=np.complex128)
        i, j, a, b = idx
        T[i, j, a, b] = X2
        T[j, i, a, b] = -X2
        T[i, j, b, a] = -X2
        T[j, i, b, a] = X2
    elif kind == "EA":
        T = np.zeros((o, v, v), dtype=np.complex128)
        j, a, b = idx
        T[j, a, b] = X2
        T[j, b, a] = -X2
    else:
        raise ValueError(kind)
    return T


def state_vv_density(kind: str, o: int, v: int, X: np.ndarray) -> np.ndarray:
    """Virtual-virtual density <Psi|a+_b a_a|Psi> of the state made of the
    zeroth-order intermediate states (the CES strings applied to the
    reference determinant) with the packed coefficients X (EE: singles (i,a),
    doubles (i<j, a<b); EA: singles a, doubles (j, a<b)).  At zeroth order
    the reference's virtual block is empty, so this is the state's
    contribution of eq. 31.  Derived from the strings:
      EE  D_ab = sum_i conj(X_ib) X_ia + 1/2 sum_{ijc} conj(X_ijbc) X_ijac
      EA  D_ab = conj(X_b) X_a + sum_{jc} conj(X_jbc) X_jac
    with the doubles extended antisymmetrically in each pair."""
    n1, n2 = dims(kind, o, v)
    X = np.asarray(X, dtype=np.complex128)
    X1, X2 = X[:n1], X[n1:]
    T = _antisym_doubles(kind, o, v, X2)
    if kind == "EE":
        S = X1.reshape(o, v)
        return np.einsum("ib,ia->ab", np.conj(S), S) + 0.5 * np.einsum("ijbc,ijac->ab", np.conj(T), T)
    return np.outer(X1, np.conj(X1)) + np.einsum("jbc,jac->ab", np.conj(T), T)


def natural_spinors(D: np.ndarray):
    """eq. 26: occupations eta (descending) and eigenvectors V (columns)."""
    w, V = np.linalg.eigh(D)
    order = np.argsort(-w, kind="stable")
    return w[order], V[:, order]


def truncate(eps: np.ndarray, o: int, D: np.ndarray, eta_crit: float):
    """eqs. 26-30.  Returns (B [v][v'], e~ [v'] ascending, eta [v])."""
    eta, V = natural_spinors(D)
    keep = eta >= eta_crit                               # eq. 27
    Vt = V[:, keep]
    Ft = np.conj(Vt).T @ np.diag(eps[o:]) @ Vt           # eq. 28
    et, Zt = np.linalg.eigh(0.5 * (Ft + np.conj(Ft).T))  # eq. 29 (ascending)
    return Vt @ Zt, et, eta                              # eq. 30


def transform_problem(eps: np.ndarray, L: np.ndarray, o: int, B: np.ndarray, et: np.ndarray):
    """Orbital energies and Cholesky vectors in the truncated basis
    (occupied spinors unchanged, virtuals a' = sum_a a B_aa')."""
    v2 = B.shape[1]
    n2 = o + v2
    Lt = np.empty((L.shape[0], n2, n2), dtype=np.complex128)
    Lt[:, :o, :o] = L[:, :o, :o]
    Lt[:, :o, o:] = L[:, :o, o:] @ B
    Lt[:, o:, :o] = np.conj(B).T @ L[:, o:, :o]
    Lt[:, o:, o:] = np.conj(B).T @ L[:, o:, o:] @ B
    return np.concatenate([eps[:o], et]), Lt


def corrected(omega3_fns: np.ndarray, omega2_can: np.ndarray, omega2_fns: np.ndarray) -> np.ndarray:
    """eq. 32."""
    return np.asarray(omega3_fns) + np.asarray(omega2_can) - np.asarray(omega2_fns)
