"""O2: explicit-term ADC(2)/ADC(3) secular matrices for EE, IP and EA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

The paper defines M through the ISR construction (Section 2.1) but prints no
working equations.  The term lists below were identified by exact matching
against O1 (``oracle.isr``), block by block and order by order, and are
checked against O1 to ~1e-15 on shapes not used to identify them (see
``tests/test_oracle_terms.py``).  They are written here as data, one line per
tensor product, and evaluated by a small generic einsum interpreter so that a
reader can compare each line with the ADC literature by eye.

Notation of a term line::

    coef  [x=Y] ...  f1(labels) f2(labels) ...

* bra (row) labels are lower case, ket (column) labels upper case; the
  bra/ket labels of a class are
      EE singles ia,  EE doubles ijab,  IP singles i,  IP doubles ija,
      EA singles a,   EA doubles iab
  (doubles are packed with i<j and a<b; the basis states are those of the
  paper's operator strings, see ``oracle.isr``);
* internal labels: k l m n p q (occupied), c d e f g h (virtual);
* ``[x=Y]`` is a Kronecker delta between a bra and a ket label;
* factors:
    g(pqrs)    <pq||rs> = sum_Q (L^Q_pr L^Q_qs - L^Q_ps L^Q_qr)   (eq. 43)
    t(ijab)    first-order doubles   t_ij^ab = <ab||ij> / D_ijab
    t2(ijab)   second-order doubles  (ladder + ring numerator) / D_ijab
    ts(ia)     second-order singles
    a trailing ``*`` means complex conjugate;
  D_ijab = e_i + e_j - e_a - e_b.  The amplitudes are the Rayleigh-
  Schroedinger coefficients of the MP ground state that enters the CES
  (eq. for the CES, Section 2.1); they are pinned to O1's wavefunction.

Diagonal blocks (11, 22) are stored as X with M = X + X^H (the Hermitian part
of the listed terms); the coupling block is stored as M12 with M21 = M12^H.

Per-block truncation (eq. 11): ADC(2) keeps M11 <= 2, M12 <= 1, M22 <= 0;
ADC(3) adds M11(3), M12(2), M22(1).  The x-scaled variant (Section 2.1,
sm-ADC) is read as M(x) = M_ADC(2) + x (M_ADC(3) - M_ADC(2)), so that x=0 is
ADC(2) and x=1 is ADC(3) exactly.
"""
from __future__ import annotations

import re
from fractions import Fraction

import numpy as np

# ----------------------------------------------------------------------------
# term table
# ----------------------------------------------------------------------------
_M11_2_EE = [
    "+1/2  t(ikac) g(IkAc)",
    "-1/4  [i=I] t(klac) g(klAc)",
    "-1/4  [a=A] t(ikcd) g(Ikcd)",
]

TERMS = {
    # ---------------------------------------------------------------- EE
    ("EE", "11", 1): ["+1/2 g(aIiA)"],
    ("EE", "11", 2): _M11_2_EE,
    ("EE", "11", 3): [s.replace(" t(", " t2(") for s in _M11_2_EE] + [
        "-1    ts(ic) g(aIAc)",
        "+1    ts(ka) g(IkiA)",
        "+1    [i=I] ts(kc) g(akAc)",
        "-1    [a=A] ts(kc) g(Ikic)",
        "+1/4  t*(IkAc) g(acde) t(ikde)",
        "-1/2  t*(IkAc) g(alkd) t(ilcd)",
        "-1/2  t*(IkAc) g(clid) t(klad)",
        "+1/4  t*(IkAc) g(lmik) t(lmac)",
        "+1/2  t*(Ikcd) g(acAe) t(ikde)",
        "+1/4  t*(Ikcd) g(aliA) t(klcd)",
        "+1/4  t*(Ikcd) g(alAk) t(ilcd)",
        "-1    t*(Ikcd) g(cliA) t(klad)",
        "+1/4  t*(klAc) g(aIid) t(klcd)",
        "+1/4  t*(klAc) g(Icid) t(klad)",
        "+1/2  t*(klAc) g(Imik) t(lmac)",
        "-1/8  [i=I] t*(klAc) g(acde) t(klde)",
        "-1/2  [i=I] t*(klAc) g(amkd) t(lmcd)",
        "-1/4  [i=I] t*(klcd) g(acAe) t(klde)",
        "+1/4  [i=I] t*(klcd) g(amAk) t(lmcd)",
        "-1/2  [a=A] t*(Ikcd) g(clie) t(klde)",
        "-1/8  [a=A] t*(Ikcd) g(lmik) t(lmcd)",
        "+1/4  [a=A] t*(klcd) g(Icie) t(klde)",
        "-1/4  [a=A] t*(klcd) g(Imik) t(lmcd)",
    ],
    ("EE", "12", 1): [
        "+1 [i=I] g(aJAB)",
        "-1 [i=J] g(aIAB)",
        "-1 [a=A] g(IJiB)",
        "+1 [a=B] g(IJiA)",
    ],
    ("EE", "12", 2): [
        "+1    t*(IJAc) g(aciB)",
        "-1    t*(IJBc) g(aciA)",
        "-1    t*(IkAB) g(aJik)",
        "+1    t*(JkAB) g(aIik)",
        "-1    [i=I] t*(JkAc) g(acBk)",
        "+1    [i=I] t*(JkBc) g(acAk)",
        "+1/2  [i=I] t*(klAB) g(aJkl)",
        "+1    [i=J] t*(IkAc) g(acBk)",
        "-1    [i=J] t*(IkBc) g(acAk)",
        "-1/2  [i=J] t*(klAB) g(aIkl)",
        "-1/2  [a=A] t*(IJcd) g(cdiB)",
        "+1    [a=A] t*(IkBc) g(Jcik)",
        "-1    [a=A] t*(JkBc) g(Icik)",
        "+1/2  [a=B] t*(IJcd) g(cdiA)",
        "-1    [a=B] t*(IkAc) g(Jcik)",
        "+1    [a=B] t*(JkAc) g(Icik)",
    ],
    ("EE", "22", 1): [
        "+1/2 [i=I] [j=J] g(abAB)",
        "+1/2 [i=I] [a=A] g(bJjB)",
        "-1   [i=I] [a=B] g(bJjA)",
        "+1/2 [i=I] [b=B] g(aJjA)",
        "-1   [i=J] [a=A] g(bIjB)",
        "+1   [i=J] [a=B] g(bIjA)",
        "+1   [i=J] [b=A] g(aIjB)",
        "-1   [i=J] [b=B] g(aIjA)",
        "+1/2 [j=J] [a=A] g(bIiB)",
        "-1   [j=J] [a=B] g(bIiA)",
        "+1/2 [j=J] [b=B] g(aIiA)",
        "+1/2 [a=A] [b=B] g(IJij)",
    ],
    # ---------------------------------------------------------------- IP
    ("IP", "11", 1): [],
    ("IP", "11", 2): ["-1/4 t(ikcd) g(Ikcd)"],
    ("IP", "11", 3): [
        "-1/4  t2(ikcd) g(Ikcd)",
        "-1    ts(kc) g(Ikic)",
        "-1/2  t*(Ikcd) g(clie) t(klde)",
        "-1/8  t*(Ikcd) g(lmik) t(lmcd)",
        "+1/4  t*(klcd) g(Icie) t(klde)",
        "-1/4  t*(klcd) g(Imik) t(lmcd)",
    ],
    ("IP", "12", 1): ["+1 g(IJiA)"],
    ("IP", "12", 2): [
        "+1/2  t*(IJcd) g(cdiA)",
        "-1    t*(IkAc) g(Jcik)",
        "+1    t*(JkAc) g(Icik)",
    ],
    ("IP", "22", 1): [
        "+1/2 [i=I] g(aJjA)",
        "-1   [i=J] g(aIjA)",
        "+1/2 [j=J] g(aIiA)",
        "+1/2 [a=A] g(IJij)",
    ],
    # ---------------------------------------------------------------- EA
    ("EA", "11", 1): [],
    ("EA", "11", 2): ["-1/4 t(klac) g(klAc)"],
    ("EA", "11", 3): [
        "-1/4  t2(klac) g(klAc)",
        "+1    ts(kc) g(akAc)",
        "-1/8  t*(klAc) g(acde) t(klde)",
        "-1/2  t*(klAc) g(amkd) t(lmcd)",
        "-1/4  t*(klcd) g(acAe) t(klde)",
        "+1/4  t*(klcd) g(amAk) t(lmcd)",
    ],
    ("EA", "12", 1): ["+1 g(aIAB)"],
    ("EA", "12", 2): [
        "-1    t*(IkAc) g(acBk)",
        "+1    t*(IkBc) g(acAk)",
        "+1/2  t*(klAB) g(aIkl)",
    ],
    ("EA", "22", 1): [
        "+1/2 [i=I] g(abAB)",
        "+1/2 [a=A] g(bIiB)",
        "-1   [a=B] g(bIiA)",
        "+1/2 [b=B] g(aIiA)",
    ],
}

BRA = {("EE", 1): "ia", ("EE", 2): "ijab", ("IP", 1): "i", ("IP", 2): "ija",
       ("EA", 1): "a", ("EA", 2): "iab"}
OCC = set("ijklmnpqIJKLMNPQ")

_TERM_RE = re.compile(r"([a-z0-9]+\*?)\(([A-Za-z]+)\)")
_DELTA_RE = re.compile(r"\[([A-Za-z])=([A-Za-z])\]")


def parse_term(s: str):
    toks = s.split()
    coef = Fraction(toks[0])
    deltas = _DELTA_RE.findall(s)
    factors = _TERM_RE.findall(s)
    return coef, factors, deltas


# ----------------------------------------------------------------------------
# integrals and MP amplitudes
# ----------------------------------------------------------------------------
class Ints:
    """Antisymmetrized integrals (eq. 43) by orbital class, cached, and the MP
    ground-state amplitudes that enter the ISR."""

    def __init__(self, eps: np.ndarray, L: np.ndarray, o: int):
        self.eps = np.asarray(eps, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.complex128)
        self.o = o
        self.v = len(eps) - o
        self._g = {}
        self._amp = {}

    def sl(self, c):
        return slice(0, self.o) if c == "o" else slice(self.o, self.o + self.v)

    def g(self, classes: str) -> np.ndarray:
        """<pq||rs> for the orbital classes of p,q,r,s (e.g. 'vvoo')."""
        if classes not in self._g:
            p, q, r, s = (self.sl(c) for c in classes)
            L = self.L
            J1 = np.einsum("Qpr,Qqs->pqrs", L[:, p, r], L[:, q, s], optimize=True)
            J2 = np.einsum("Qps,Qqr->pqrs", L[:, p, s], L[:, q, r], optimize=True)
            self._g[classes] = J1 - J2
        return self._g[classes]

    def D2(self):
        e = self.eps
        eo, ev = e[: self.o], e[self.o:]
        return eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]

    def amp(self, name: str) -> np.ndarray:
        if name not in self._amp:
            if name == "t":
                # first-order doubles: <ab||ij> / (e_i + e_j - e_a - e_b)
                self._amp[name] = self.g("vvoo").transpose(2, 3, 0, 1) / self.D2()
            elif name == "t2":
                # second-order doubles: (V_N acting on t in the doubles space) / D
                t = self.amp("t")
                num = (0.5 * np.einsum("abcd,ijcd->ijab", self.g("vvvv"), t, optimize=True)
                       + 0.5 * np.einsum("klij,klab->ijab", self.g("oooo"), t, optimize=True))
                ring = np.einsum("kbjc,ikac->ijab", self.g("ovov"), t, optimize=True)
                ring = ring - ring.transpose(1, 0, 2, 3)
                ring = ring - ring.transpose(0, 1, 3, 2)
                self._amp[name] = (num - ring) / self.D2()
            elif name == "ts":
                # second-order singles: <Phi_i^a|V|Psi(1)> / (e_i - e_a)
                t = self.amp("t")
                num = (0.5 * np.einsum("ajbc,ijbc->ia", self.g("vovv"), t, optimize=True)
                       - 0.5 * np.einsum("jkib,jkab->ia", self.g("ooov"), t, optimize=True))
                e = self.eps
                self._amp[name] = num / (e[: self.o, None] - e[None, self.o:])
            else:
                raise KeyError(name)
        return self._amp[name]

    def factor(self, name: str, labels: str) -> np.ndarray:
        conj = name.endswith("*")
        base = name.rstrip("*")
        if base == "g":
            arr = self.g("".join("o" if c in OCC else "v" for c in labels))
        else:
            arr = self.amp(base)
        return arr.conj() if conj else arr


# ----------------------------------------------------------------------------
# packing
# ----------------------------------------------------------------------------
def dims(kind: str, o: int, v: int):
    Po, Pv = o * (o - 1) // 2, v * (v - 1) // 2
    return {"EE": (o * v, Po * Pv), "IP": (o, Po * v), "EA": (v, o * Pv)}[kind]


def packed_index(kind: str, cls: int, o: int, v: int):
    """Index arrays (one per label of the class) in packed order."""
    iu_o = np.triu_indices(o, 1)
    iu_v = np.triu_indices(v, 1)
    if cls == 1:
        if kind == "EE":
            i, a = np.meshgrid(np.arange(o), np.arange(v), indexing="ij")
            return (i.ravel(), a.ravel())
        return (np.arange(o),) if kind == "IP" else (np.arange(v),)
    if kind == "EE":
        P, Q = np.meshgrid(np.arange(len(iu_o[0])), np.arange(len(iu_v[0])), indexing="ij")
        P, Q = P.ravel(), Q.ravel()
        return (iu_o[0][P], iu_o[1][P], iu_v[0][Q], iu_v[1][Q])
    if kind == "IP":
        P, A = np.meshgrid(np.arange(len(iu_o[0])), np.arange(v), indexing="ij")
        P, A = P.ravel(), A.ravel()
        return (iu_o[0][P], iu_o[1][P], A)
    I, Q = np.meshgrid(np.arange(o), np.arange(len(iu_v[0])), indexing="ij")
    I, Q = I.ravel(), Q.ravel()
    return (I, iu_v[0][Q], iu_v[1][Q])


def class_shape(kind, cls, o, v):
    labels = BRA[(kind, cls)]
    return tuple(o if c in OCC else v for c in labels)


def embed(kind, cls, o, v, Yp):
    """Packed vectors (k, n_cls) -> unpacked (k, ...) holding values only at
    packed positions (zero elsewhere)."""
    k = Yp.shape[0]
    out = np.zeros((k,) + class_shape(kind, cls, o, v), dtype=np.complex128)
    idx = packed_index(kind, cls, o, v)
    out[(slice(None),) + idx] = Yp
    return out


def extract(kind, cls, o, v, S):
    idx = packed_index(kind, cls, o, v)
    return S[(slice(None),) + idx]


# ----------------------------------------------------------------------------
# generic evaluation of sigma contributions
# ----------------------------------------------------------------------------
def _eval(ints: Ints, term: str, out_labels: str, in_labels: str, Yu: np.ndarray, swap: bool):
    """sum over in-labels of F(out, in) Y(in) for one term line.  With
    swap=True the term's bra/ket roles are exchanged and its factors
    conjugated, i.e. the contribution of X^H."""
    coef, factors, deltas = parse_term(term)
    fac = []
    for name, lab in factors:
        if swap:
            lab = "".join(c.swapcase() if c in _EXT else c for c in lab)
            name = name[:-1] if name.endswith("*") else name + "*"
        fac.append((name, lab))
    dl = [(a.swapcase(), b.swapcase()) if swap else (a, b) for a, b in deltas]
    # with swap, delta pairs read (bra', ket') = (upper->lower)...; substitute ket by bra
    sub = {}
    for a, b in dl:
        # one of the pair is an out label, the other an in label
        if a in out_labels:
            sub[b] = a
        else:
            sub[a] = b
    ops, subs = [], []
    for name, lab in fac:
        ops.append(ints.factor(name, lab))
        subs.append("".join(sub.get(c, c) for c in lab))
    ysub = "z" + "".join(sub.get(c, c) for c in in_labels)
    spec = ",".join(subs + [ysub]) + "->z" + out_labels
    return float(coef) * contract(spec, *ops, Yu)


_EXT = set("ijabIJAB")
# contraction order of a term line: numpy's path search, allowed
# intermediates of up to 2^28 elements (its default cap, the largest operand,
# can leave no pairwise step and fall back to one nested loop over every
# label); the order does not change what is summed
_PATH = ("optimal", 1 << 28)


def contract(spec: str, *ops: np.ndarray) -> np.ndarray:
    """np.einsum(spec, *ops) for a spec with explicit output, evaluated pair
    by pair in the order numpy's path search picks, every pair as one batched
    matrix product (labels shared by both factors and still needed later are
    the batch; labels needed nowhere later are summed first).  The same sum
    as einsum's, in another order; einsum itself runs a pair with a batch
    label as an unthreaded loop."""
    ins, out = spec.split("->")
    labels = ins.split(",")
    arrs = list(ops)
    # repeated labels within one factor (a Kronecker delta substituted into
    # it): take the diagonal first
    for n, (a, la) in enumerate(zip(arrs, labels)):
        if len(set(la)) < len(la):
            u = "".join(dict.fromkeys(la))
            arrs[n], labels[n] = np.einsum(f"{la}->{u}", a), u
    if len(arrs) == 1:
        return np.einsum(f"{labels[0]}->{out}", arrs[0])
    path = np.einsum_path(",".join(labels) + "->" + out, *arrs, optimize=_PATH)[0][1:]
    for i, j in path:
        i, j = sorted((i, j))
        A, la = arrs[i], labels[i]
        B, lb = arrs[j], labels[j]
        rest = "".join(labels[n] for n in range(len(labels)) if n not in (i, j)) + out
        # labels of one factor needed nowhere else: summed out at once
        for X, lx, ly in ((0, la, lb), (1, lb, la)):
            drop = [c for c in lx if c not in ly and c not in rest]
            if drop:
                keep = "".join(c for c in lx if c not in drop)
                if X == 0:
                    A, la = np.einsum(f"{la}->{keep}", A), keep
                else:
                    B, lb = np.einsum(f"{lb}->{keep}", B), keep
        bat = [c for c in la if c in lb and c in rest]
        red = [c for c in la if c in lb and c not in rest]
        ma = [c for c in la if c not in lb]
        nb = [c for c in lb if c not in la]
        size = {c: A.shape[la.index(c)] for c in la}
        size.update({c: B.shape[lb.index(c)] for c in lb})
        prod = lambda cs: int(np.prod([size[c] for c in cs])) if cs else 1  # noqa: E731
        At = np.transpose(A, [la.index(c) for c in bat + ma + red]).reshape(prod(bat), prod(ma), prod(red))
        Bt = np.transpose(B, [lb.index(c) for c in bat + red + nb]).reshape(prod(bat), prod(red), prod(nb))
        C = np.matmul(At, Bt).reshape([size[c] for c in bat + ma + nb])
        for n in (j, i):
            del arrs[n], labels[n]
        arrs.append(C)
        labels.append("".join(bat + ma + nb))
    (R,), (lr,) = arrs, labels
    if lr != out:
        drop = "".join(c for c in lr if c not in out)
        if drop:
            R, lr = np.einsum(f"{lr}->{''.join(c for c in lr if c in out)}", R), "".join(c for c in lr if c in out)
        R = np.transpose(R, [lr.index(c) for c in out])
    return R


def _dense_term(ints: Ints, term: str, out_labels: str, in_labels: str, swap: bool) -> np.ndarray:
    """F(out, in) of one term line as a dense tensor (deltas expanded)."""
    coef, factors, deltas = parse_term(term)
    fac = []
    for name, lab in factors:
        if swap:
            lab = "".join(c.swapcase() if c in _EXT else c for c in lab)
            name = name[:-1] if name.endswith("*") else name + "*"
        fac.append((name, lab))
    dl = [(a.swapcase(), b.swapcase()) if swap else (a, b) for a, b in deltas]
    sub = {}
    for a, b in dl:
        if a in out_labels:
            sub[b] = a
        else:
            sub[a] = b
    ops, subs = [], []
    for name, lab in fac:
        ops.append(ints.factor(name, lab))
        subs.append("".join(sub.get(c, c) for c in lab))
    free_in = [c for c in in_labels if c not in sub]
    all_labels = out_labels + "".join(free_in)
    present = set("".join(subs))
    red_labels = "".join(c for c in all_labels if c in present)
    red = contract(",".join(subs) + "->" + red_labels, *ops)
    size = {c: (ints.o if c in OCC else ints.v) for c in out_labels + in_labels}
    full = np.zeros([size[c] for c in out_labels + in_labels], dtype=np.complex128)
    grids = np.indices([size[c] for c in all_labels])
    pos = {c: grids[k] for k, c in enumerate(all_labels)}
    idx = tuple(pos[c] for c in out_labels) + tuple(pos[sub.get(c, c)] for c in in_labels)
    full[idx] = float(coef) * red[tuple(pos[c] for c in red_labels)]
    return full


def m11_block(ints: Ints, kind: str, order: int) -> np.ndarray:
    """Dense singles-singles block at one order (packed rows and columns),
    cached: it is n1 x n1 and is applied as a matrix product."""
    key = ("M11", kind, order)
    if key not in ints._amp:
        o, v = ints.o, ints.v
        n1 = dims(kind, o, v)[0]
        if order == 0:
            M = np.diag(diag0(ints, kind, 1)).astype(np.complex128)
        else:
            bra = BRA[(kind, 1)]
            F = 0
            for s in TERMS.get((kind, "11", order), []):
                F = F + _dense_term(ints, s, bra, bra.upper(), swap=False)
                F = F + _dense_term(ints, s, bra, bra.upper(), swap=True)
            M = np.reshape(F, (n1, n1)) if not np.isscalar(F) else np.zeros((n1, n1), complex)
        ints._amp[key] = M
    return ints._amp[key]


DENSE_SINGLES_MAX = 512


def sigma_block(ints: Ints, kind: str, block: str, order: int, Y_in: np.ndarray,
                dense_singles: bool | None = None) -> np.ndarray:
    """Contribution of block ``block`` ('11','12','21','22') at perturbation
    order ``order`` to sigma, for packed input vectors Y_in (k, n_in).
    Returns packed (k, n_out).

    The singles block is applied either as the dense matrix of m11_block or
    matrix-free, term line by term line like the other blocks (the same
    lines; forming it densely costs far more than applying the lines to a few
    vectors once n1 is in the thousands).  Default: dense for n1 <= 512."""
    o, v = ints.o, ints.v
    r, c = int(block[0]), int(block[1])
    k = Y_in.shape[0]
    if block == "11" and order > 0:
        if dense_singles is None:
            dense_singles = dims(kind, o, v)[0] <= DENSE_SINGLES_MAX
        if dense_singles:
            return Y_in @ m11_block(ints, kind, order).T
    if order == 0:
        if r != c:
            return np.zeros((k, dims(kind, o, v)[r - 1]), dtype=np.complex128)
        return diag0(ints, kind, r)[None, :] * Y_in
    bra = BRA[(kind, r)]
    ket_lower = BRA[(kind, c)]
    Yu = embed(kind, c, o, v, Y_in)
    out = None
    if r == c:
        # X and X^H
        for s in TERMS.get((kind, f"{r}{c}", order), []):
            for swap in (False, True):
                val = _eval(ints, s, bra, ket_lower.upper(), Yu, swap=swap)
                out = val if out is None else out + val
    elif (r, c) == (1, 2):
        for s in TERMS.get((kind, "12", order), []):
            val = _eval(ints, s, bra, ket_lower.upper(), Yu, swap=False)
            out = val if out is None else out + val
    else:  # M21 = M12^H: out = doubles labels, in = singles labels
        for s in TERMS.get((kind, "12", order), []):
            val = _eval(ints, s, bra, ket_lower.upper(), Yu, swap=True)
            out = val if out is None else out + val
    if out is None:
        return np.zeros((k, dims(kind, o, v)[r - 1]), dtype=np.complex128)
    return extract(kind, r, o, v, out)


def diag0(ints: Ints, kind: str, cls: int) -> np.ndarray:
    """Zeroth-order (diagonal) energies of the packed basis."""
    o, v = ints.o, ints.v
    eo, ev = ints.eps[:o], ints.eps[o:]
    idx = packed_index(kind, cls, o, v)
    if kind == "EE":
        if cls == 1:
            return ev[idx[1]] - eo[idx[0]]
        return ev[idx[2]] + ev[idx[3]] - eo[idx[0]] - eo[idx[1]]
    if kind == "IP":
        if cls == 1:
            return -eo[idx[0]]
        return ev[idx[2]] - eo[idx[0]] - eo[idx[1]]
    if cls == 1:
        return ev[idx[0]]
    return ev[idx[1]] + ev[idx[2]] - eo[idx[0]]


ADC2_ORDERS = {"11": (0, 1, 2), "12": (1,), "21": (1,), "22": (0,)}
X_ORDERS = {"11": (3,), "12": (2,), "21": (2,), "22": (1,)}


def sigma(ints: Ints, kind: str, x: float, Y: np.ndarray) -> np.ndarray:
    """Matrix-free S = M(x) Y for packed vectors Y (k, dim)."""
    o, v = ints.o, ints.v
    n1, n2 = dims(kind, o, v)
    Y = np.atleast_2d(Y)
    Y1, Y2 = Y[:, :n1], Y[:, n1:]
    S1 = np.zeros_like(Y1)
    S2 = np.zeros_like(Y2)
    for blk in ("11", "12", "21", "22"):
        r, c = int(blk[0]), int(blk[1])
        src = Y1 if c == 1 else Y2
        if src.shape[1] == 0 or (r == 2 and n2 == 0):
            continue
        for od, f in [(od, 1.0) for od in ADC2_ORDERS[blk]] + [(od, x) for od in X_ORDERS[blk]]:
            if f == 0.0:
                continue
            val = f * sigma_block(ints, kind, blk, od, src)
            if r == 1:
                S1 += val
            else:
                S2 += val
    return np.concatenate([S1, S2], axis=1)


def dense_matrix(ints: Ints, kind: str, x: float, chunk: int = 512) -> np.ndarray:
    """Dense M(x), column blocks of sigma applied to unit vectors."""
    n1, n2 = dims(kind, ints.o, ints.v)
    dim = n1 + n2
    M = np.zeros((dim, dim), dtype=np.complex128)
    for c0 in range(0, dim, chunk):
        c1 = min(dim, c0 + chunk)
        E = np.zeros((c1 - c0, dim), dtype=np.complex128)
        E[np.arange(c1 - c0), np.arange(c0, c1)] = 1.0
        M[:, c0:c1] = sigma(ints, kind, x, E).T
    return M


def block_matrix(ints: Ints, kind: str, block: str, order: int) -> np.ndarray:
    """Dense block at one order (rows = block row class)."""
    n1, n2 = dims(kind, ints.o, ints.v)
    nc = n1 if block[1] == "1" else n2
    E = np.eye(nc, dtype=np.complex128)
    return sigma_block(ints, kind, block, order, E).T
