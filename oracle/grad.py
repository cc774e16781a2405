"""Oracle gradients of the ADC secular matrix with respect to the Cholesky
vectors and the third-order scaling x.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

The quantity differentiated is the real functional

    f(L, x) = Re sum_z  Sbar_z^H  M(L, x) Y_z

for fixed packed vectors Y and Sbar.  With Sbar = Y = an eigenvector y of the
Hermitian M this is y^H M y, whose derivative along any Hermitian
perturbation is the eigenvalue derivative (Hellmann-Feynman; the paper makes
the secular problem Hermitian in Section 2.1, eq. 10).

The derivative is obtained by automatic differentiation, not by a hand
derived adjoint: ``TorchInts`` and ``sigma_t`` evaluate exactly the term
lines of ``oracle.adc_terms`` (same TERMS table, same index bookkeeping) with
torch CPU complex128 operations, and torch's reverse mode differentiates
them.  ``tests/test_oracle_grad.py`` pins this evaluation to the numpy
oracle (sigma equal to ~1e-14) and the gradient to central finite
differences of the numpy oracle.

Gradient convention: for a complex tensor Z, G_Z = df/dRe Z + i df/dIm Z.
L^Q is Hermitian in (p, q) for every Q (eq. 42 with real AO vectors), and only
Hermitian perturbations keep M Hermitian, so the reported dL is the
projection G <- (G + G^H) / 2 per Q.  The x derivative is exact because M is
affine in x: df/dx = f(L, 1) - f(L, 0) with the same L.
"""
from __future__ import annotations

import numpy as np
import torch

from .adc_terms import (ADC2_ORDERS, BRA, OCC, TERMS, X_ORDERS, _EXT, diag0, dims, packed_index,
                        parse_term)


def _E(spec, *ops):
    """torch.einsum, contracted pairwise in the order numpy's einsum_path
    picks (torch alone contracts several operands in one step)."""
    if len(ops) <= 2:
        return torch.einsum(spec, *ops)
    ins, out = spec.split("->")
    subs = ins.split(",")
    shapes = [np.broadcast_to(np.zeros((), complex), tuple(t.shape)) for t in ops]
    path = np.einsum_path(spec, *shapes, optimize="greedy")[0][1:]
    ops, subs = list(ops), list(subs)
    for pair in path:
        pair = sorted(pair, reverse=True)
        picked = [(subs.pop(i), ops.pop(i)) for i in pair]
        rest = "".join(subs) + out
        keep = "".join(dict.fromkeys(c for s_, _ in picked for c in s_ if c in rest))
        res = torch.einsum(",".join(s_ for s_, _ in picked) + "->" + keep, *[t for _, t in picked])
        subs.append(keep)
        ops.append(res)
    return torch.einsum(subs[0] + "->" + out, ops[0])


class TorchInts:
    """Antisymmetrized integrals (eq. 43) and MP amplitudes, as in
    ``oracle.adc_terms.Ints``, on a torch complex128 L (may require grad)."""

    def __init__(self, eps: np.ndarray, L: torch.Tensor, o: int):
        self.eps = np.asarray(eps, dtype=np.float64)
        self.L = L
        self.o = o
        self.v = len(eps) - o
        self._g = {}
        self._amp = {}

    def sl(self, c):
        return slice(0, self.o) if c == "o" else slice(self.o, self.o + self.v)

    def g(self, classes: str) -> torch.Tensor:
        if classes not in self._g:
            p, q, r, s = (self.sl(c) for c in classes)
            L = self.L
            self._g[classes] = (_E("Qpr,Qqs->pqrs", L[:, p, r], L[:, q, s])
                                - _E("Qps,Qqr->pqrs", L[:, p, s], L[:, q, r]))
        return self._g[classes]

    def D2(self) -> torch.Tensor:
        e = self.eps
        eo, ev = e[: self.o], e[self.o:]
        d = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
        return torch.from_numpy(d)

    def amp(self, name: str) -> torch.Tensor:
        if name not in self._amp:
            if name == "t":
                self._amp[name] = self.g("vvoo").permute(2, 3, 0, 1) / self.D2()
            elif name == "t2":
                t = self.amp("t")
                num = 0.5 * _E("abcd,ijcd->ijab", self.g("vvvv"), t) + 0.5 * _E("klij,klab->ijab", self.g("oooo"), t)
                ring = _E("kbjc,ikac->ijab", self.g("ovov"), t)
                ring = ring - ring.permute(1, 0, 2, 3)
                ring = ring - ring.permute(0, 1, 3, 2)
                self._amp[name] = (num - ring) / self.D2()
            elif name == "ts":
                t = self.amp("t")
                num = 0.5 * _E("ajbc,ijbc->ia", self.g("vovv"), t) - 0.5 * _E("jkib,jkab->ia", self.g("ooov"), t)
                e = self.eps
                self._amp[name] = num / torch.from_numpy(e[: self.o, None] - e[None, self.o:])
            else:
                raise KeyError(name)
        return self._amp[name]

    def factor(self, name: str, labels: str) -> torch.Tensor:
        conj = name.endswith("*")
        base = name.rstrip("*")
        if base == "g":
            arr = self.g("".join("o" if c in OCC else "v" for c in labels))
        else:
            arr = self.amp(base)
        return arr.conj() if conj else arr


def _factors(term, out_labels, swap):
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
    return coef, fac, sub


def _eval(ints, term, out_labels, in_labels, Yu, swap):
    coef, fac, sub = _factors(term, out_labels, swap)
    ops, subs = [], []
    for name, lab in fac:
        ops.append(ints.factor(name, lab))
        subs.append("".join(sub.get(c, c) for c in lab))
    ysub = "z" + "".join(sub.get(c, c) for c in in_labels)
    return float(coef) * _E(",".join(subs + [ysub]) + "->z" + out_labels, *ops, Yu)


def _dense_term(ints, term, out_labels, in_labels, swap):
    coef, fac, sub = _factors(term, out_labels, swap)
    ops, subs = [], []
    for name, lab in fac:
        ops.append(ints.factor(name, lab))
        subs.append("".join(sub.get(c, c) for c in lab))
    free_in = [c for c in in_labels if c not in sub]
    all_labels = out_labels + "".join(free_in)
    present = set("".join(subs))
    red_labels = "".join(c for c in all_labels if c in present)
    red = _E(",".join(subs) + "->" + red_labels, *ops)
    size = {c: (ints.o if c in OCC else ints.v) for c in out_labels + in_labels}
    full = torch.zeros([size[c] for c in out_labels + in_labels], dtype=torch.complex128)
    grids = np.indices([size[c] for c in all_labels])
    pos = {c: torch.from_numpy(grids[k]) for k, c in enumerate(all_labels)}
    idx = tuple(pos[c] for c in out_labels) + tuple(pos[sub.get(c, c)] for c in in_labels)
    full = full.index_put(idx, float(coef) * red[tuple(pos[c] for c in red_labels)])
    return full


def _embed(kind, cls, o, v, Yp):
    labels = BRA[(kind, cls)]
    shape = tuple(o if c in OCC else v for c in labels)
    out = torch.zeros((Yp.shape[0],) + shape, dtype=torch.complex128)
    idx = tuple(torch.from_numpy(i) for i in packed_index(kind, cls, o, v))
    out[(slice(None),) + idx] = Yp
    return out


def _extract(kind, cls, o, v, S):
    idx = tuple(torch.from_numpy(i) for i in packed_index(kind, cls, o, v))
    return S[(slice(None),) + idx]


def _m11(ints, kind, order):
    o, v = ints.o, ints.v
    n1 = dims(kind, o, v)[0]
    if order == 0:
        return torch.diag(torch.from_numpy(diag0(ints, kind, 1)).to(torch.complex128))
    bra = BRA[(kind, 1)]
    F = torch.zeros([o if c in OCC else v for c in bra + bra], dtype=torch.complex128)
    for s in TERMS.get((kind, "11", order), []):
        F = F + _dense_term(ints, s, bra, bra.upper(), swap=False)
        F = F + _dense_term(ints, s, bra, bra.upper(), swap=True)
    return F.reshape(n1, n1)


def _block(ints, kind, block, order, Y_in):
    o, v = ints.o, ints.v
    r, c = int(block[0]), int(block[1])
    k = Y_in.shape[0]
    zero = torch.zeros((k, dims(kind, o, v)[r - 1]), dtype=torch.complex128)
    if block == "11":
        return Y_in @ _m11(ints, kind, order).T
    if order == 0:
        if r != c:
            return zero
        return torch.from_numpy(diag0(ints, kind, r))[None, :] * Y_in
    bra = BRA[(kind, r)]
    ket = BRA[(kind, c)].upper()
    Yu = _embed(kind, c, o, v, Y_in)
    out = None
    if r == c:
        lines = [(s, sw) for s in TERMS.get((kind, f"{r}{c}", order), []) for sw in (False, True)]
    elif (r, c) == (1, 2):
        lines = [(s, False) for s in TERMS.get((kind, "12", order), [])]
    else:
        lines = [(s, True) for s in TERMS.get((kind, "12", order), [])]
    for s, sw in lines:
        val = _eval(ints, s, bra, ket, Yu, swap=sw)
        out = val if out is None else out + val
    if out is None:
        return zero
    return _extract(kind, r, o, v, out)


def sigma_t(ints: TorchInts, kind: str, x: float, Y: torch.Tensor) -> torch.Tensor:
    """S = M(x) Y in torch (same blocks and orders as ``adc_terms.sigma``)."""
    o, v = ints.o, ints.v
    n1, n2 = dims(kind, o, v)
    Y1, Y2 = Y[:, :n1], Y[:, n1:]
    S1 = torch.zeros_like(Y1)
    S2 = torch.zeros_like(Y2)
    for blk in ("11", "12", "21", "22"):
        r, c = int(blk[0]), int(blk[1])
        src = Y1 if c == 1 else Y2
        if src.shape[1] == 0 or (r == 2 and n2 == 0):
            continue
        for od, f in [(od, 1.0) for od in ADC2_ORDERS[blk]] + [(od, x) for od in X_ORDERS[blk]]:
            if f == 0.0:
                continue
            val = f * _block(ints, kind, blk, od, src)
            if r == 1:
                S1 = S1 + val
            else:
                S2 = S2 + val
    return torch.cat([S1, S2], dim=1)


def herm_project(G: np.ndarray) -> np.ndarray:
    """(G + G^H) / 2 for every Q of a [N][n][n] gradient."""
    return 0.5 * (G + np.conj(np.transpose(G, (0, 2, 1))))


def vjp(kind: str, eps, L: np.ndarray, o: int, x: float, Y: np.ndarray, Sbar: np.ndarray):
    """Gradient of f = Re sum_z Sbar_z^H M(L, x) Y_z.

    Returns (dL, dx): dL [N][n][n] complex128, Hermitian-projected per Q;
    dx = f(L, 1) - f(L, 0) (M is affine in x)."""
    Lt = torch.tensor(np.asarray(L, dtype=np.complex128), requires_grad=True)
    Yt = torch.from_numpy(np.atleast_2d(np.asarray(Y, dtype=np.complex128)))
    St = torch.from_numpy(np.atleast_2d(np.asarray(Sbar, dtype=np.complex128)))
    S = sigma_t(TorchInts(eps, Lt, o), kind, x, Yt)
    f = torch.real((St.conj() * S).sum())
    (G,) = torch.autograd.grad(f, Lt)
    with torch.no_grad():
        ints = TorchInts(eps, Lt.detach(), o)
        f1 = torch.real((St.conj() * sigma_t(ints, kind, 1.0, Yt)).sum())
        f0 = torch.real((St.conj() * sigma_t(ints, kind, 0.0, Yt)).sum())
    return herm_project(G.numpy()), float(f1 - f0)


def functional(kind: str, eps, L: np.ndarray, o: int, x: float, Y: np.ndarray, Sbar: np.ndarray) -> float:
    """f = Re sum_z Sbar_z^H M(L, x) Y_z with the numpy oracle (for finite differences)."""
    from .adc_terms import Ints, sigma
    S = sigma(Ints(eps, L, o), kind, x, np.atleast_2d(Y))
    return float(np.real(np.sum(np.conj(np.atleast_2d(Sbar)) * S)))
