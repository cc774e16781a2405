"""O1: the ISR secular matrix computed numerically in determinant space.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

This is the *definition* of the ADC(n) secular matrix used by everything
else (Section 2.1):

* correlated excited states  Psi^0_J = C_J Psi_0  (eq. for the CES), with
  the operator strings of the three manifolds exactly as printed:
    EE: a+_a a_i ;  a+_a a_i a+_b a_j   (a<b, i<j)
    IP: a_i      ;  a+_a a_i a_j        (i<j)
    EA: a+_a     ;  a+_a a+_b a_j       (a<b)
  (the garbled ``\\hat{a}j`` is read as a_j);
* Gram-Schmidt of each class against all lower classes (class 0 is the
  ground state, EE only);
* symmetric orthonormalization within a class with S^{-1/2};
* M_IJ = <Psi~_I | H - E_0 | Psi~_J>;
* perturbation expansion M = M(0) + M(1) + ... (eq. 11) with Moller-Plesset
  partitioning H(lam) = H0 + lam V, H0 = sum_p eps_p p+p, and per-block
  truncation  ADC(2): M11<=2, M12<=1, M22<=0;  ADC(3): M11<=3, M12<=2, M22<=1;
* sm-ADC (the x-scaled variant): M(x) = M_ADC(2) + x (M_ADC(3) - M_ADC(2)).

The ground state is Rayleigh-Schroedinger PT on Phi_0 (occupied spinors
0..o-1) in intermediate normalisation, then normalised as a truncated power
series.  Every quantity is a power series in lam truncated after lam^3; the
coefficients are extracted exactly by series arithmetic, no fitting.

The Hamiltonian is built from the orbital energies eps and antisymmetrized
integrals <pq||rs> (Section 2.5, eq. 43 for the Cholesky form) with
h_pq = eps_p delta_pq - sum_i <pi||qi>, so that the Fock matrix is diag(eps)
(canonical Hartree-Fock reference).

Basis order of the packed ISR vectors (occupied indices first, pairs i<j and
a<b in lexicographic order):
    EE: [ (i,a) i-major | ((i<j),(a<b)) pair-major ]
    IP: [ i | ((i<j), a) ]
    EA: [ a | (i, (a<b)) ]
Cost is exponential; use n = o+v <= 12.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np
import scipy.sparse as sp

NORD = 4  # series orders 0..3


# ----------------------------------------------------------------------------
# integrals (Section 2.5, eq. 43)
# ----------------------------------------------------------------------------
def antisym_integrals(L: np.ndarray) -> np.ndarray:
    """<pq||rs> = sum_Q (L^Q_pr L^Q_qs - L^Q_ps L^Q_qr), no conjugation."""
    J = np.einsum("Qpr,Qqs->pqrs", L, L)
    return J - J.transpose(0, 1, 3, 2)


def core_hamiltonian(eps: np.ndarray, g: np.ndarray, o: int) -> np.ndarray:
    """h with a diagonal Fock matrix: h_pq = eps_p delta_pq - sum_i <pi||qi>."""
    return np.diag(eps).astype(np.complex128) - np.einsum("piqi->pq", g[:, :o, :, :o])


# ----------------------------------------------------------------------------
# determinant space
# ----------------------------------------------------------------------------
class Sector:
    """All determinants of n spinors with N electrons, as bit masks."""

    def __init__(self, n: int, N: int):
        self.n, self.N = n, N
        if 0 <= N <= n:
            self.dets = [sum(1 << p for p in c) for c in itertools.combinations(range(n), N)]
        else:
            self.dets = []
        self.index = {d: k for k, d in enumerate(self.dets)}

    def __len__(self):
        return len(self.dets)


def _sign_below(d: int, p: int) -> int:
    return -1 if bin(d & ((1 << p) - 1)).count("1") & 1 else 1


def _annihilate(d: int, p: int):
    if not (d >> p) & 1:
        return None, 0
    return d ^ (1 << p), _sign_below(d, p)


def _create(d: int, p: int):
    if (d >> p) & 1:
        return None, 0
    return d | (1 << p), _sign_below(d, p)


class FockSpace:
    """Sectors and elementary operator matrices for n spinors."""

    def __init__(self, n: int):
        self.n = n
        self._sec = {}
        self._ops = {}

    def sector(self, N: int) -> Sector:
        if N not in self._sec:
            self._sec[N] = Sector(self.n, N)
        return self._sec[N]

    def op(self, kind: str, p: int, N: int) -> sp.csr_matrix:
        """Matrix of a+_p ('c') or a_p ('a') acting on the N-electron sector."""
        key = (kind, p, N)
        if key not in self._ops:
            src = self.sector(N)
            dst = self.sector(N + 1 if kind == "c" else N - 1)
            rows, cols, vals = [], [], []
            fn = _create if kind == "c" else _annihilate
            for k, d in enumerate(src.dets):
                d2, s = fn(d, p)
                if d2 is not None:
                    rows.append(dst.index[d2])
                    cols.append(k)
                    vals.append(s)
            self._ops[key] = sp.csr_matrix((np.array(vals, dtype=np.float64), (rows, cols)),
                                           shape=(len(dst), len(src)))
        return self._ops[key]

    def apply_string(self, ops, vec: np.ndarray, N: int):
        """Apply an operator string written left to right (so the rightmost acts
        first) to vectors (columns) in sector N.  Returns (result, N_out)."""
        out = vec
        for kind, p in reversed(ops):
            out = self.op(kind, p, N) @ out
            N = N + 1 if kind == "c" else N - 1
        return out, N


def hamiltonian(sec: Sector, h: np.ndarray, g: np.ndarray, eps: np.ndarray):
    """H = sum_pq h_pq p+q + 1/4 sum g_pqrs p+q+sr in the sector, and the
    diagonal of H0 = sum_p eps_p p+p.  Returns (H0_diag, V) with V = H - H0."""
    n = sec.n
    dim = len(sec)
    rows, cols, vals = [], [], []
    h0 = np.zeros(dim)
    for k, d in enumerate(sec.dets):
        occ = [p for p in range(n) if (d >> p) & 1]
        h0[k] = sum(eps[p] for p in occ)
        # one-body part
        for q in occ:
            d1, s1 = _annihilate(d, q)
            for p in range(n):
                d2, s2 = _create(d1, p)
                if d2 is None or h[p, q] == 0:
                    continue
                rows.append(sec.index[d2]); cols.append(k); vals.append(s1 * s2 * h[p, q])
        # two-body part: sum_{p<q, r<s} <pq||rs> p+ q+ s r
        for r, s_ in itertools.combinations(occ, 2):
            d1, t1 = _annihilate(d, r)
            d2, t2 = _annihilate(d1, s_)
            free = [p for p in range(n) if not (d2 >> p) & 1]
            for p, q in itertools.combinations(free, 2):
                val = g[p, q, r, s_]
                if val == 0:
                    continue
                d3, t3 = _create(d2, q)
                d4, t4 = _create(d3, p)
                rows.append(sec.index[d4]); cols.append(k); vals.append(t1 * t2 * t3 * t4 * val)
    H = sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(dim, dim))
    V = H - sp.diags(h0.astype(np.complex128))
    return h0, sp.csr_matrix(V)


# ----------------------------------------------------------------------------
# truncated power series (coefficient arrays along axis 0, orders 0..3)
# ----------------------------------------------------------------------------
def s_mul(a, b):
    """Product of two series of matrices (or scalars / vectors broadcasting
    with @ where both are 2-D)."""
    out = [None] * NORD
    for n_ in range(NORD):
        acc = 0
        for k in range(n_ + 1):
            acc = acc + a[k] @ b[n_ - k]
        out[n_] = acc
    return out


def s_dag(a):
    return [x.conj().T for x in a]


def s_scale(a, c):
    return [x * c for x in a]


def s_add(a, b):
    return [x + y for x, y in zip(a, b)]


def s_invsqrt_unit(S):
    """(I + D)^{-1/2} for a series S whose order-0 part is the identity:
    I - D/2 + 3D^2/8 - 5D^3/16 (exact through lam^3 because D = O(lam))."""
    I = S[0]
    D = [np.zeros_like(I)] + [S[k] for k in range(1, NORD)]
    D2 = s_mul(D, D)
    D3 = s_mul(D2, D)
    out = []
    for n_ in range(NORD):
        term = -0.5 * D[n_] + 0.375 * D2[n_] - 0.3125 * D3[n_]
        if n_ == 0:
            term = term + I
        out.append(term)
    return out


# ----------------------------------------------------------------------------
# ground state: Rayleigh-Schroedinger PT (intermediate normalisation)
# ----------------------------------------------------------------------------
def rspt(h0, V, i0, order=3):
    dim = len(h0)
    E = [h0[i0], V[i0, i0]]
    psi = [np.zeros(dim, dtype=np.complex128)]
    psi[0][i0] = 1.0
    denom = h0[i0] - h0
    denom[i0] = 1.0
    for n_ in range(1, order + 1):
        rhs = V @ psi[n_ - 1]
        for m in range(1, n_ + 1):
            rhs = rhs - E[m] * psi[n_ - m]
        rhs[i0] = 0.0
        pn = rhs / denom
        pn[i0] = 0.0
        psi.append(pn)
        E.append((V @ pn)[i0])
    return np.array(E[: order + 1]), psi


def normalised_ground_state(psi):
    """Psi_0 = psi / sqrt(<psi|psi>) as a truncated series (column vectors)."""
    cols = [p.reshape(-1, 1) for p in psi]
    nrm = s_mul(s_dag(cols), cols)  # 1x1 series, order-0 part is 1
    f = s_invsqrt_unit(nrm)
    return s_mul(cols, f)


# ----------------------------------------------------------------------------
# manifolds and packing
# ----------------------------------------------------------------------------
def pairs(m: int):
    return list(itertools.combinations(range(m), 2))


def manifold(kind: str, o: int, v: int):
    """Operator strings of classes 1 and 2 in packed order, and the electron
    count change of the target sector."""
    occ = list(range(o))
    vir = [o + a for a in range(v)]
    if kind == "EE":
        c1 = [[("c", vir[a]), ("a", occ[i])] for i in range(o) for a in range(v)]
        c2 = [[("c", vir[a]), ("a", occ[i]), ("c", vir[b]), ("a", occ[j])]
              for (i, j) in pairs(o) for (a, b) in pairs(v)]
        dN = 0
    elif kind == "IP":
        c1 = [[("a", occ[i])] for i in range(o)]
        c2 = [[("c", vir[a]), ("a", occ[i]), ("a", occ[j])]
              for (i, j) in pairs(o) for a in range(v)]
        dN = -1
    elif kind == "EA":
        c1 = [[("c", vir[a])] for a in range(v)]
        c2 = [[("c", vir[a]), ("c", vir[b]), ("a", occ[j])]
              for j in range(o) for (a, b) in pairs(v)]
        dN = +1
    else:
        raise ValueError(kind)
    return c1, c2, dN


# ----------------------------------------------------------------------------
# the ISR secular matrix as a series
# ----------------------------------------------------------------------------
class ISR:
    """Numerical ISR for one (kind, eps, L) problem.

    Attributes after construction:
      E0      ground-state energy coefficients E(0..3)
      psi0    normalised ground-state series (N-electron sector)
      M       list of 4 dense matrices: M(lam) = sum_n lam^n M[n]
      n1, n2  class sizes
    """

    def __init__(self, kind: str, eps: np.ndarray, g: np.ndarray, o: int):
        self.kind = kind
        n = len(eps)
        v = n - o
        self.o, self.v, self.n = o, v, n
        fs = FockSpace(n)
        self.fs = fs
        h = core_hamiltonian(eps, g, o)
        secN = fs.sector(o)
        h0N, VN = hamiltonian(secN, h, g, eps)
        i0 = secN.index[(1 << o) - 1]
        E, psi = rspt(h0N, VN, i0, order=3)
        self.E0 = E
        self.h0N, self.VN, self.i0 = h0N, VN, i0
        self.psi_raw = psi
        psi0 = normalised_ground_state(psi)  # series of (dimN x 1)
        self.psi0 = psi0

        c1, c2, dN = manifold(kind, o, v)
        self.n1, self.n2 = len(c1), len(c2)
        Nt = o + dN
        sect = fs.sector(Nt)
        if Nt == o:
            h0T, VT = h0N, VN
        else:
            h0T, VT = hamiltonian(sect, h, g, eps)
        self.h0T, self.VT = h0T, VT

        def ces(strings):
            cols = []
            for n_ in range(NORD):
                vecs = []
                for s in strings:
                    w, Nout = fs.apply_string(s, psi0[n_], o)
                    assert Nout == Nt
                    vecs.append(np.asarray(w).reshape(-1))
                cols.append(np.stack(vecs, axis=1) if vecs else np.zeros((len(sect), 0), complex))
            return cols

        lower = psi0 if kind == "EE" else None  # class 0 exists for EE only
        tilde = []
        for strings in (c1, c2):
            P0 = ces(strings)
            if lower is not None and lower[0].shape[1] > 0:
                ov = s_mul(s_dag(lower), P0)
                P0 = s_add(P0, s_scale(s_mul(lower, ov), -1.0))
            S = s_mul(s_dag(P0), P0)
            if S[0].shape[0]:
                assert np.allclose(S[0], np.eye(S[0].shape[0]), atol=1e-12), "order-0 overlap is not I"
                Sih = s_invsqrt_unit(S)
                Pt = s_mul(P0, Sih)
            else:
                Pt = P0
            tilde.append(Pt)
            lower = Pt if lower is None else [np.concatenate([a, b], axis=1) for a, b in zip(lower, Pt)]
        # all intermediate states of classes >= 1
        Ps = [np.concatenate([a, b], axis=1) for a, b in zip(tilde[0], tilde[1])]
        self.states = Ps
        # (H(lam) - E0(lam)) Psi~
        HP = []
        for n_ in range(NORD):
            acc = h0T[:, None] * Ps[n_]
            if n_ >= 1:
                acc = acc + VT @ Ps[n_ - 1]
            for m in range(n_ + 1):
                acc = acc - E[m] * Ps[n_ - m]
            HP.append(acc)
        self.M = s_mul(s_dag(Ps), HP)

    # ------------------------------------------------------------------
    def block(self, which: str, order: int) -> np.ndarray:
        n1 = self.n1
        Mo = self.M[order]
        return {"11": Mo[:n1, :n1], "12": Mo[:n1, n1:], "21": Mo[n1:, :n1], "22": Mo[n1:, n1:]}[which]

    def adc_matrix(self, level: int, lam: float = 1.0) -> np.ndarray:
        """ADC(2) or ADC(3) matrix at coupling strength lam."""
        lim = {2: (2, 1, 0), 3: (3, 2, 1)}[level]
        n1 = self.n1
        out = np.zeros_like(self.M[0])
        for n_ in range(NORD):
            f = lam ** n_
            if n_ <= lim[0]:
                out[:n1, :n1] += f * self.M[n_][:n1, :n1]
            if n_ <= lim[1]:
                out[:n1, n1:] += f * self.M[n_][:n1, n1:]
                out[n1:, :n1] += f * self.M[n_][n1:, :n1]
            if n_ <= lim[2]:
                out[n1:, n1:] += f * self.M[n_][n1:, n1:]
        return out

    def matrix(self, x: float, lam: float = 1.0) -> np.ndarray:
        """sm-ADC matrix M(x) = M_ADC(2) + x (M_ADC(3) - M_ADC(2))."""
        m2 = self.adc_matrix(2, lam)
        m3 = self.adc_matrix(3, lam)
        return m2 + x * (m3 - m2)


def isr_from_L(kind: str, eps: np.ndarray, L: np.ndarray, o: int) -> ISR:
    return ISR(kind, eps, antisym_integrals(L), o)
