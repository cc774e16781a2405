"""Pins of the pivoted-Cholesky oracle (Section 2.5, eq. 41, the one-step
procedure, and eq. 42) against what the mathematics fixes:

* a matrix of rank r is reproduced exactly by r vectors, and the procedure
  stops there;
* with a threshold tau the remaining matrix is positive semidefinite with
  diagonal below tau, so every entry of V - L^T L is at most tau in size;
* a diagonal matrix gives unit vectors scaled by sqrt(V_pp), largest first;
* on the pivots the factor is triangular and equals LAPACK's Cholesky factor
  of the pivoted leading block;
* eq. 42 gives Hermitian L^P_pq, and the integrals built from them equal the
  four-index transform of the factorised AO matrix.
"""
import numpy as np

from adcgen import make_eri, mo_coefficients
from oracle.cholesky import mo_transform, pivoted_cholesky, unpack_pairs


def test_low_rank_is_exact():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((60, 9))
    V = B @ B.T
    L, piv = pivoted_cholesky(V, 1e-10)
    assert L.shape == (9, 60) and len(set(piv.tolist())) == 9
    assert np.abs(V - L.T @ L).max() <= 1e-12 * np.abs(V).max()


def test_threshold_bounds_the_residual():
    V = make_eri(8, seed=2)
    for tau in (1e-2, 1e-4, 1e-7):
        L, piv = pivoted_cholesky(V, tau)
        R = V - L.T @ L
        d = np.diag(R)
        assert d.max() < tau and d.min() > -1e-12
        assert np.linalg.eigvalsh(R).min() > -1e-12
        assert np.abs(R).max() <= tau * (1 + 1e-9)
    # each vector is at the largest remaining diagonal element: the pivot
    # elements decrease along the sequence
    L, piv = pivoted_cholesky(V, 1e-9)
    pv = L[np.arange(len(piv)), piv] ** 2
    assert (np.diff(pv) <= 1e-12).all()


def test_diagonal_matrix():
    d = np.array([0.5, 3.0, 0.0, 2.0, 3.0, 1e-9])
    L, piv = pivoted_cholesky(np.diag(d), 1e-6)
    assert piv.tolist() == [1, 4, 3, 0]       # equal elements: lowest index first
    for k, p in enumerate(piv):
        e = np.zeros(len(d))
        e[p] = np.sqrt(d[p])
        assert np.abs(L[k] - e).max() <= 1e-15 * e.max()


def test_pivoted_block_is_lapack_cholesky():
    V = make_eri(7, seed=3)
    L, piv = pivoted_cholesky(V, 1e-8)
    Lp = L[:, piv]                                # n x n on the pivots
    # vector k vanishes (up to rounding) on the earlier pivots
    assert np.abs(np.tril(Lp, -1)).max() <= 1e-12 * np.abs(Lp).max()
    ref = np.linalg.cholesky(V[np.ix_(piv, piv)]).T
    assert np.abs(Lp - ref).max() <= 1e-10 * np.abs(ref).max()


def test_max_vec_and_zero_matrix():
    V = make_eri(6, seed=4)
    L, piv = pivoted_cholesky(V, 0.0, max_vec=5)
    assert L.shape[0] == 5
    L, piv = pivoted_cholesky(np.zeros((5, 5)), 0.0)
    assert L.shape == (0, 5)


def test_mo_transform():
    n_ao, n_mo = 6, 5
    V = make_eri(n_ao, seed=5)
    L, _ = pivoted_cholesky(V, 1e-12)
    Lao = unpack_pairs(L, n_ao)
    C = mo_coefficients(n_ao, n_mo, seed=6)
    assert np.abs(C.conj().T @ C - np.eye(n_mo)).max() < 1e-13
    Lmo = mo_transform(Lao, C)
    assert np.abs(Lmo - Lmo.conj().transpose(0, 2, 1)).max() < 1e-14
    # (pq|rs) from the MO vectors = the four-index transform of (mu nu|kappa lambda)
    full = np.einsum("Pmn,Pkl->mnkl", Lao, Lao)
    ref = np.einsum("mp,nq,kr,ls,mnkl->pqrs", C.conj(), C, C.conj(), C, full)
    got = np.einsum("Ppq,Prs->pqrs", Lmo, Lmo)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # the factorised AO matrix reproduces V on the packed pairs
    iu = np.triu_indices(n_ao)
    assert np.abs(full[iu[0], iu[1]][:, iu[0], iu[1]] - V).max() < 1e-10 * np.abs(V).max()
