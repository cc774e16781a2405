"""Write c5_adjoint.json: the oracle gradient of f = Re Sbar^H M(L, x) Y at
the adjoint configuration (EE-ADC(3), o=16, v=96, Nchol=600, seed 51) for
seeded unit trial vectors, reduced to values a test can compare: dx, the
directional derivatives along seeded Hermitian directions, sampled entries
and the largest entries of the Hermitian-projected dL.

Calls only oracle/ and the input generators (adcgen).  Takes a few minutes:
    python tests/golden/make_c5_adjoint.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from adcgen import config_problem, hermitian_direction, sample_indices, trial_vectors  # noqa: E402
from oracle.adc_terms import dims  # noqa: E402
from oracle.grad import vjp  # noqa: E402

Y_SEED, SBAR_SEED, K = 501, 502, 1
DIR_SEEDS = [511, 512, 513]
SAMPLE_SEED, N_SAMPLES, N_TOP = 521, 256, 16


def main():
    P = config_problem("C5")
    n1, n2 = dims(P.kind, P.o, P.v)
    Y = trial_vectors(K, n1 + n2, Y_SEED)
    Sb = trial_vectors(K, n1 + n2, SBAR_SEED)
    G, dx = vjp(P.kind, P.eps, P.L, P.o, P.x, Y, Sb)
    flat = G.reshape(-1)
    idx = sample_indices(flat.size, N_SAMPLES, SAMPLE_SEED)
    top = np.argsort(-np.abs(flat))[:N_TOP]
    proj = []
    for s in DIR_SEEDS:
        rq = 30 if s == DIR_SEEDS[0] else None
        D = hermitian_direction(P.L.shape, s, restrict_q=rq)
        proj.append({"seed": s, "restrict_q": rq, "value": float(np.real(np.vdot(G, D)))})
    out = {
        "what": "oracle gradient of Re Sbar^H M(L,x) Y, Hermitian-projected dL, dx = f(x=1) - f(x=0)",
        "config": "C5", "kind": P.kind, "o": P.o, "v": P.v, "n_chol": P.n_chol, "x": P.x, "seed": P.seed,
        "k": K, "y_seed": Y_SEED, "sbar_seed": SBAR_SEED,
        "dx": dx, "max_abs": float(np.abs(flat).max()), "fro": float(np.linalg.norm(flat)),
        "projections": proj,
        "samples": [[int(i), float(flat[i].real), float(flat[i].imag)] for i in idx],
        "top": [[int(i), float(flat[i].real), float(flat[i].imag)] for i in top],
    }
    with open(os.path.join(HERE, "c5_adjoint.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
