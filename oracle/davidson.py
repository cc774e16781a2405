"""CPU block Davidson and Rayleigh-quotient certificates (FP64).

TEST INFRASTRUCTURE ONLY.

Solves M X = X Omega (eq. 10) for the k algebraically lowest roots of the
Hermitian ADC matrix using only sigma products, as the paper's Davidson step
does (Section 2.4, root solve; the settings are not printed, the readings
below are this project's):

* guesses: unit vectors on the k smallest diagonal entries of M11 (ties to
  the lower index);
* preconditioner (omega - D)^-1 with |denominator| floored at 1e-4, D the
  zeroth-order diagonal;
* convergence: ||r_k|| <= tol and |d omega_k| <= 1e-10;
* subspace limit 6k, collapse to 2k; two-pass Gram-Schmidt.
"""
from __future__ import annotations

import numpy as np


def _orthonormalize(N: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Two passes of block Gram-Schmidt against V, then modified Gram-Schmidt
    within N; directions that lose more than half their norm are dropped."""
    keep = []
    for a in range(N.shape[0]):
        x = N[a].copy()
        n0 = np.linalg.norm(x)
        if n0 == 0:
            continue
        for _ in range(2):
            if V.shape[0]:
                x = x - V.T @ (V.conj() @ x)
            for y in keep:
                x = x - np.vdot(y, x) * y
        nx = np.linalg.norm(x)
        if nx > 1e-3 * n0 and nx > 1e-14:
            keep.append(x / nx)
    return np.array(keep) if keep else np.zeros((0, N.shape[1]), dtype=N.dtype)


def davidson(sigma_fn, diag: np.ndarray, guess_diag: np.ndarray, k: int, tol: float = 1e-7,
             max_iter: int = 200, max_sub: int | None = None):
    """Returns (omega, X, resnorm, iterations, converged)."""
    dim = len(diag)
    max_sub = max_sub or max(6 * k, 2 * k + 2)
    order = np.lexsort((np.arange(len(guess_diag)), guess_diag))[:k]
    V = np.zeros((k, dim), dtype=np.complex128)
    V[np.arange(k), order] = 1.0
    S = sigma_fn(V)
    omega_old = np.full(k, np.inf)
    for it in range(1, max_iter + 1):
        G = V.conj() @ S.T
        G = 0.5 * (G + G.conj().T)
        w_all, U_all = np.linalg.eigh(G)
        w, U = w_all[:k], U_all[:, :k]
        X = U.T @ V
        AX = U.T @ S
        R = AX - w[:, None] * X
        rn = np.linalg.norm(R, axis=1)
        conv = (rn <= tol) & (np.abs(w - omega_old) <= 1e-10)
        omega_old = w.copy()
        if np.all(conv):
            return w, X, rn, it, conv
        idx = np.nonzero(~conv)[0]
        den = w[idx, None] - diag[None, :]
        den = np.where(np.abs(den) < 1e-4, np.where(den < 0, -1e-4, 1e-4), den)
        N = R[idx] / den
        if V.shape[0] + N.shape[0] > max_sub:
            m = min(2 * k, U_all.shape[1])
            V = U_all[:, :m].T @ V
            S = U_all[:, :m].T @ S
        N = _orthonormalize(N, V)
        if N.shape[0] == 0:
            break
        V = np.concatenate([V, N])
        S = np.concatenate([S, sigma_fn(N)])
    return w, X, rn, it, conv


def rayleigh_certificate(sigma_fn, X: np.ndarray):
    """theta_r = x_r^H M x_r / x_r^H x_r and ||M x_r - theta_r x_r|| for given
    vectors; |theta - omega_exact| <= ||r||^2 / gap."""
    X = np.atleast_2d(X)
    nrm = np.einsum("ki,ki->k", X.conj(), X).real
    X = X / np.sqrt(nrm)[:, None]
    S = sigma_fn(X)
    theta = np.einsum("ki,ki->k", X.conj(), S).real
    r = np.linalg.norm(S - theta[:, None] * X, axis=1)
    return theta, r
