"""GPU parity of the ISR properties (adc_properties, Section 2.2) against the
oracle's closed forms, themselves pinned to O1's determinant-space series:
excited-state densities and transition densities of the Davidson roots, and
the expectation values and transition moments of a Hermitian one-particle
operator, elementwise to 1e-12 of the largest element."""
import numpy as np
import pytest

from adcgen import config_problem, make_problem
from oracle.adc_terms import Ints
from oracle.props import state_density, transition_density

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _check(P, k, seed):
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, conv_tol=1e-8)
    r = h.davidson()
    n = P.o + P.v
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    d = 0.5 * (d + d.conj().T)
    out = h.properties(r["vectors"].contiguous(), torch.from_numpy(d).cuda())
    ints = Ints(P.eps, P.L, P.o)
    t, ts = ints.amp("t"), ints.amp("ts")
    Yh = r["vectors"].cpu().numpy()
    rho, tdm = out["rho"].cpu().numpy(), out["tdm"].cpu().numpy()
    for z in range(k):
        y = Yh[z] / np.linalg.norm(Yh[z])
        R = state_density(P.o, P.v, t, ts, y)
        Tm = transition_density(P.o, P.v, t, y)
        assert np.abs(rho[z] - R).max() <= 1e-12 * np.abs(R).max(), z
        assert np.abs(tdm[z] - Tm).max() <= 1e-12 * np.abs(Tm).max(), z
        assert abs(out["D"][z] - np.sum(d * R)) <= 1e-11 * max(1.0, abs(np.sum(d * R)))
        assert abs(out["T"][z] - np.sum(d * Tm)) <= 1e-11 * max(1.0, abs(np.sum(d * Tm)))
        assert abs(np.trace(rho[z]).real - P.o) < 1e-10
        assert abs(out["D"][z].imag) < 1e-10       # Hermitian d, Hermitian density
        print(f"  root {z}: omega {r['omega'][z]:.8f} D {out['D'][z].real:.8f} |T| {abs(out['T'][z]):.6f}",
              flush=True)
    h.close()


def test_properties_small():
    print("case properties EE o=5 v=14", flush=True)
    _check(make_problem("EE", 5, 14, 50, seed=95, n_roots=3, x=1.0, scale=0.1), 3, 95)


def test_properties_adjoint_configuration():
    print("case properties C5", flush=True)
    _check(config_problem("C5"), 4, 96)
