"""One-step pivoted Cholesky of the electron-repulsion matrix and the
transform of its vectors to the molecular spinor basis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Section 2.5.  The ERI matrix (mu nu|kappa lambda), read as a symmetric
positive semidefinite matrix V over composite indices, is factorised as
V ~ sum_P L^P (L^P)^T (eq. 41).  In the one-step procedure the vectors are
made one at a time: each new vector is the column of the remaining matrix at
its largest remaining diagonal element, scaled by one over the square root of
that element, and the procedure stops when that element falls below the
threshold tau.  The vectors are then carried to the molecular spinor basis,
L^P_pq = sum_{mu nu} conj(C_mu p) L^P_mu nu C_nu q (eq. 42).

Readings: among equal largest diagonal elements the lowest index is taken;
the procedure also stops after max_vec vectors or when no diagonal element is
positive.
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky(V: np.ndarray, tau: float, max_vec: int | None = None):
    """Returns (L [n_vec][m], pivots [n_vec]) with V ~ L^T L."""
    V = np.asarray(V, dtype=np.float64)
    m = V.shape[0]
    max_vec = m if max_vec is None else max_vec
    d = np.diag(V).copy()            # diagonal of the remaining matrix
    vecs, piv = [], []
    while len(vecs) < max_vec:
        p = int(np.argmax(d))
        if not d[p] > 0.0 or d[p] < tau:
            break
        col = V[:, p].copy()         # column p of the remaining matrix
        for l in vecs:
            col -= l[p] * l
        l = col / np.sqrt(d[p])
        vecs.append(l)
        piv.append(p)
        d = d - l * l
    L = np.array(vecs).reshape(len(vecs), m)
    return L, np.array(piv, dtype=np.int64)


def unpack_pairs(Lp: np.ndarray, n_ao: int) -> np.ndarray:
    """Vectors over packed pairs mu <= nu -> symmetric [P][n_ao][n_ao]."""
    iu = np.triu_indices(n_ao)
    out = np.zeros((Lp.shape[0], n_ao, n_ao))
    out[:, iu[0], iu[1]] = Lp
    out[:, iu[1], iu[0]] = Lp
    return out


def mo_transform(L_ao: np.ndarray, C: np.ndarray) -> np.ndarray:
    """eq. 42: L^P_pq = sum_{mu nu} conj(C_mu p) L^P_mu nu C_nu q."""
    return np.einsum("mp,Pmn,nq->Ppq", np.conj(C), L_ao, C)
