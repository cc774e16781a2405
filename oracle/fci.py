"""O3: full configuration interaction in the N, N-1 and N+1 sectors.

TEST INFRASTRUCTURE ONLY.

Exact excitation, ionisation and attachment energies of H(lam) = H0 + lam V
(Section 2.1: the eigenvalues of the exact secular problem are E_n(N') - E_0(N)).
Used to check that the ISR series of O1 is correct order by order: the
ADC(n) eigenvalue error must vanish as lam^(n+1) for singles-dominated roots.
"""
from __future__ import annotations

import numpy as np

from .isr import FockSpace, core_hamiltonian, hamiltonian


class FCI:
    def __init__(self, eps: np.ndarray, g: np.ndarray, o: int):
        self.o = o
        n = len(eps)
        fs = FockSpace(n)
        h = core_hamiltonian(eps, g, o)
        self._parts = {}
        for dN in (-1, 0, 1):
            N = o + dN
            if N < 0 or N > n:
                continue
            sec = fs.sector(N)
            h0, V = hamiltonian(sec, h, g, eps)
            self._parts[dN] = (h0, V.toarray())

    def energies(self, dN: int, lam: float) -> np.ndarray:
        h0, V = self._parts[dN]
        return np.linalg.eigvalsh(np.diag(h0) + lam * V)

    def omegas(self, kind: str, lam: float) -> np.ndarray:
        """Exact generalized excitation energies, ascending."""
        E0 = self.energies(0, lam)[0]
        if kind == "EE":
            return self.energies(0, lam)[1:] - E0
        if kind == "IP":
            return self.energies(-1, lam) - E0
        if kind == "EA":
            return self.energies(+1, lam) - E0
        raise ValueError(kind)
