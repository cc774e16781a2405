"""Root-specific state-specific frozen natural spinors (Section 2.4).

For EE and EA the paper solves each root in its own truncated basis:

1. canonical ADC(2) for the n_roots lowest roots (adc_davidson at x = 0);
2. for root k, the state-specific virtual density D^MP2 + D^ADC(2)(k) of
   eq. 31, its natural spinors, the eta_crit cut and the semicanonical basis
   (eqs. 26-30), with the problem and the ADC(2) eigenvector of root k
   carried into that basis (adc_fns);
3. one instance per root, all solved in one batched handle (lanes over the
   device streams), each by the root-specific Davidson solver (root_follow)
   started from its transformed ADC(2) vector: ADC(2) and ADC(2)+x(3) in the
   truncated basis;
4. the truncation correction of eq. 32,
   omega(k) = omega_ADC(3)^SS-FNS(k) + omega_ADC(2)^canonical(k) - omega_ADC(2)^SS-FNS(k).

IP uses MP2 FNS without the correction (the paper's choice): one truncated
problem for all roots (frozen_natural_spinor_roots).  Every step is a call of
the library; this module only passes buffers between the calls.
"""
from __future__ import annotations

import numpy as np

from . import Batch, Handle


def ss_fns_roots(kind, o, v, eps, L, n_roots, eta_crit, x=1.0, precision="fp64", conv_tol=1e-7, verbose=False):
    """Root-specific SS-FNS-ADC(2)+x(3) roots with the eq. 32 correction.

    kind 'EE' or 'EA'; L numpy [N][n][n] or a complex128 cuda tensor.
    Returns a dict of numpy arrays per root: omega_corrected, omega_fns (the
    uncorrected truncated root), omega2_fns, omega2_canonical, n_vir (kept
    virtual spinors per root), and converged."""
    if kind not in ("EE", "EA"):
        raise ValueError("state-specific FNS is built for EE and EA (IP uses MP2 FNS)")
    h2 = Handle(kind, o, v, eps, L, n_roots, x=0.0, precision=precision, conv_tol=conv_tol)
    r2 = h2.davidson(want_vectors=True)
    bases = [h2.fns(eta_crit, X=r2["vectors"][k].contiguous()) for k in range(n_roots)]
    h2.close()
    out = {}
    for xv, name in ((0.0, "omega2_fns"), (x, "omega_fns")):
        probs = [dict(kind=kind, o=o, v=b["n_vir"], eps=b["eps"], L=b["L"].contiguous(), n_roots=1, x=xv)
                 for b in bases]
        B = Batch(probs, precision=precision, conv_tol=conv_tol, root_follow=True, verbose=verbose)
        res, rc = B.davidson(guesses=[b["X"][None].contiguous() for b in bases])
        out[name] = np.array([r["omega"][0] for r in res])
        out.setdefault("converged", np.ones(n_roots, dtype=bool))
        out["converged"] &= np.array([bool(r["converged"][0]) for r in res])
        B.close()
    out["omega2_canonical"] = r2["omega"].copy()
    out["omega_corrected"] = out["omega_fns"] + out["omega2_canonical"] - out["omega2_fns"]
    out["n_vir"] = np.array([b["n_vir"] for b in bases])
    return out


def frozen_natural_spinor_roots(kind, o, v, eps, L, n_roots, eta_crit, x=1.0, precision="fp64", conv_tol=1e-7):
    """MP2 FNS (eqs. 25-30) and the n_roots lowest roots in the truncated basis
    (the IP scheme of the paper, no correction).  Returns (omega, n_vir)."""
    h = Handle(kind, o, v, eps, L, n_roots, x=x, precision="fp64")
    b = h.fns(eta_crit)
    h.close()
    ht = Handle(kind, o, b["n_vir"], b["eps"], b["L"].contiguous(), n_roots, x=x, precision=precision,
                conv_tol=conv_tol)
    r = ht.davidson(want_vectors=False)
    ht.close()
    return r["omega"], b["n_vir"]
