"""Per-root certification of the GPU eigenpairs against the oracle.

At the adjoint workload (EE-ADC(3), x = 1, o = 16, v = 96, N_chol = 600,
4 roots), the Ritz vectors of the FP64 solve and of the mixed solve
(split-bf16 sweeps, then FP64 refinement) are handed to the oracle, which
forms M y with its own FP64 term-by-term sigma.  For a normalised y with
Rayleigh quotient theta and residual r = M y - theta y, the Hermitian M has an
eigenvalue within |r|^2 / gap of theta, gap being the distance from theta to
the rest of the spectrum (Section 2.1, eq. 10: M is Hermitian).  The gap is
taken from an FP64 solve for two roots more.  Asserted per root:
|omega_gpu - theta| + |r|^2 / gap <= 1e-8 Eh (FP64) and <= 1e-6 Eh (mixed).
"""
import numpy as np
import pytest

from adcgen import config_problem
from oracle.adc_terms import Ints
from oracle.adc_terms import sigma as osigma
from oracle.davidson import rayleigh_certificate

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_c5_roots_certified_by_the_oracle():
    P = config_problem("C5")
    k = P.n_roots
    print("case C5 certification: FP64 and mixed Davidson, oracle sigma of the Ritz vectors", flush=True)
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, conv_tol=1e-7)
    r64 = h.davidson()
    h.close()
    hm = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision="split_bf16", conv_tol=3e-5)
    rm = hm.davidson()
    hm.close()
    hw = adc.Handle("EE", P.o, P.v, P.eps, P.L, k + 2, x=P.x, conv_tol=1e-7)
    rw = hw.davidson(want_vectors=False)
    hw.close()
    assert r64["converged"].all() and rm["converged"].all() and rw["converged"].all()
    # the k lowest of the wider solve are the same roots
    assert np.abs(rw["omega"][:k] - r64["omega"]).max() < 1e-8
    X = torch.cat([r64["vectors"], rm["vectors"]]).cpu().numpy()
    print("  GPU solves done; oracle sigma of", X.shape[0], "vectors", flush=True)
    ints = Ints(P.eps, P.L, P.o)
    theta, rn = rayleigh_certificate(lambda Z: osigma(ints, "EE", P.x, Z), X)
    spec = rw["omega"]
    for name, om, th, r, bar in (("fp64", r64["omega"], theta[:k], rn[:k], 1e-8),
                                 ("mixed", rm["omega"], theta[k:], rn[k:], 1e-6)):
        for j in range(k):
            gap = np.min(np.abs(np.delete(spec, j) - th[j]))
            bound = abs(om[j] - th[j]) + r[j] ** 2 / gap
            print(f"  {name} root {j}: omega {om[j]:.12f} theta {th[j]:.12f} |r| {r[j]:.2e} gap {gap:.3e} "
                  f"certified error <= {bound:.2e}", flush=True)
            assert bound <= bar, (name, j, bound)
