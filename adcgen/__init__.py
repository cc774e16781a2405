"""Seeded synthetic inputs (orbital energies and complex Cholesky vectors).

This module is shared by the CPU oracle and by the GPU path's tests and
benchmark.  It holds no ADC arithmetic: it only draws random numbers in a
fixed order so that every consumer sees identical inputs.

Recipe (stands in for the paper's molecular workloads, which need basis sets,
geometries and an SCF program; shape ratios follow the large runs of the
paper's Section 3.5: N_chol of a few times o+v, v/o of about 6):

1. eps_occ = sort(uniform(-2.0, -0.3, o))    (Eh)
2. eps_vir = sort(uniform(0.1, 4.0, v))      (Eh)
3. X = standard_normal((N, n, n)), then Y = standard_normal((N, n, n))
4. G = (X + iY)/sqrt(2)
5. L^Q = s_Q (G^Q + G^Q^H)/sqrt(2),  s_Q = 0.05 exp(-Q/30), Q = 0..N-1

L^Q is Hermitian in (p, q) for every Q, as the MO transform of real AO
Cholesky vectors is (Section 2.5, the AO->MO transform of the Cholesky
vectors).  Occupied spinors come first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["Problem", "make_problem", "CONFIGS", "config_problem", "c4_draw", "trial_vectors", "make_eri", "mo_coefficients",
           "hermitian_direction", "sample_indices"]


@dataclass
class Problem:
    kind: str          # "EE", "IP" or "EA"
    o: int
    v: int
    n_chol: int
    n_roots: int
    x: float
    eps: np.ndarray    # float64 [o+v], occupied first, ascending within each class
    L: np.ndarray      # complex128 [N][n][n], Hermitian in the last two indices
    seed: int = 0

    @property
    def n(self) -> int:
        return self.o + self.v


def _draw_eps(rng, o, v):
    eps_occ = np.sort(rng.uniform(-2.0, -0.3, o))
    eps_vir = np.sort(rng.uniform(0.1, 4.0, v))
    return np.concatenate([eps_occ, eps_vir])


def make_L(rng, n_chol: int, n: int, scale: float = 0.05, chunk: int = 64) -> np.ndarray:
    """Draw the Cholesky tensor.  X is drawn whole first, then Y chunk by chunk
    over Q; numpy's Generator fills arrays sequentially, so the result is
    identical to drawing Y whole (checked in the tests)."""
    X = rng.standard_normal((n_chol, n, n))
    L = np.empty((n_chol, n, n), dtype=np.complex128)
    inv2 = 1.0 / math.sqrt(2.0)
    for q0 in range(0, n_chol, chunk):
        q1 = min(n_chol, q0 + chunk)
        Y = rng.standard_normal((q1 - q0, n, n))
        G = (X[q0:q1] + 1j * Y) * inv2
        s = scale * np.exp(-np.arange(q0, q1) / 30.0)
        L[q0:q1] = s[:, None, None] * (G + G.conj().transpose(0, 2, 1)) * inv2
    return L


def make_problem(kind: str, o: int, v: int, n_chol: int, seed: int, n_roots: int = 4,
                 x: float = 1.0, scale: float = 0.05) -> Problem:
    rng = np.random.default_rng(seed)
    eps = _draw_eps(rng, o, v)
    L = make_L(rng, n_chol, o + v, scale=scale)
    return Problem(kind, o, v, n_chol, n_roots, float(x), eps, L, seed)


# The five workloads: (kind, o, v, N_chol, k, x, seed).  C3 and C4 carry no x
# in their description; C3 is run at x=1 (named ADC(3)) and C4 at the
# production value x=0.5.
CONFIGS = {
    "C1": ("EE", 6, 18, 80, 4, 1.0, 11),
    "C2": ("EE", 20, 120, 900, 8, 0.5, 21),
    "C3-IP": ("IP", 60, 400, 2400, 6, 1.0, 31),
    "C3-EA": ("EA", 60, 400, 2400, 6, 1.0, 32),
    "C5": ("EE", 16, 96, 600, 4, 1.0, 51),
}


def config_problem(name: str) -> Problem:
    kind, o, v, N, k, x, seed = CONFIGS[name]
    return make_problem(kind, o, v, N, seed, n_roots=k, x=x)


def c4_draw(n_inst: int = 64):
    """Shapes of the batched workload: list of (kind, o, v, N, k, seed)."""
    meta = np.random.default_rng(41)
    out = []
    for t in range(n_inst):
        o = int(meta.integers(8, 41))
        v = int(meta.integers(40, 241))
        k = int(meta.integers(4, 17))
        kind = ("EE", "IP", "EA")[t % 3]
        out.append((kind, o, v, 6 * (o + v), k, 4100 + t))
    return out


def trial_vectors(k: int, dim: int, seed: int) -> np.ndarray:
    """k complex Gaussian vectors of length dim, each of unit norm."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))
    return Z / np.linalg.norm(Z, axis=1, keepdims=True)


def hermitian_direction(shape, seed: int, restrict_q=None) -> np.ndarray:
    """A perturbation of L: Hermitian in the last two indices for every Q,
    optionally zero for Q >= restrict_q, unit Frobenius norm."""
    rng = np.random.default_rng(seed)
    E = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    E = 0.5 * (E + np.conj(np.transpose(E, (0, 2, 1))))
    if restrict_q is not None:
        E[restrict_q:] = 0.0
    return E / np.linalg.norm(E)


def sample_indices(size: int, n: int, seed: int) -> np.ndarray:
    """n distinct flat indices into an array of the given size, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(size, size=min(n, size), replace=False))



def make_eri(n_ao: int, seed: int, rank: int | None = None, decay: float = 8.0) -> np.ndarray:
    """A synthetic electron-repulsion matrix: (mu nu|kappa lambda) over the
    packed pairs mu <= nu, real symmetric positive semidefinite,
    V = sum_R s_R^2 b_R b_R^T with b_R the packed upper triangle of a real
    symmetric Gaussian matrix and s_R = exp(-R / decay) (R = 0 .. rank-1;
    default rank = the number of pairs).  Shape [n_pair][n_pair],
    n_pair = n_ao (n_ao + 1) / 2."""
    rng = np.random.default_rng(seed)
    npair = n_ao * (n_ao + 1) // 2
    rank = npair if rank is None else rank
    iu = np.triu_indices(n_ao)
    B = np.empty((rank, npair))
    for r in range(rank):
        G = rng.standard_normal((n_ao, n_ao))
        B[r] = ((G + G.T) / 2.0)[iu] * math.exp(-r / decay)
    return B.T @ B


def mo_coefficients(n_ao: int, n_mo: int, seed: int) -> np.ndarray:
    """n_mo orthonormal complex columns of length n_ao (the first columns of a
    random unitary: QR of a complex Gaussian matrix), [n_ao][n_mo]."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n_ao, n_ao)) + 1j * rng.standard_normal((n_ao, n_ao))
    Q, R = np.linalg.qr(Z)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]
    return np.ascontiguousarray(Q[:, :n_mo])
