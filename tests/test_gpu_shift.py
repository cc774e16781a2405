"""A property of M that holds at any size, checked on the HIP path at the
benchmark sizes: every energy denominator of the method (the MP amplitudes and
the ADC blocks, section 2.1) is a difference of equally many occupied and
virtual orbital energies, so shifting all of them by c moves M by the change of
particle number times c (EE: 0, IP: -c, EA: +c).  The library forms the
amplitudes, the zeroth-order diagonal and the singles block from eps itself,
so a slip in any of them shows here as a residue beyond rounding.  The same
property pins the oracle (test_oracle_terms.py).
"""
import numpy as np
import pytest

from adcgen import config_problem, make_problem

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu

C = 0.731
CASES = [
    # C2, the timed workload (EE o=20 v=120 N_chol=900)
    ("C2", None),
    # IP and EA at sizes that span many tiles with ragged tails
    ("IP-o30-v150", ("IP", 30, 150, 900, 4, 0.5, 611)),
    ("EA-o20-v120", ("EA", 20, 120, 900, 4, 0.5, 612)),
]


@pytest.mark.parametrize("name,spec", CASES, ids=[c[0] for c in CASES])
def test_uniform_orbital_energy_shift(name, spec):
    if spec is None:
        P = config_problem("C2")
    else:
        kind, o, v, N, k, x, seed = spec
        P = make_problem(kind, o, v, N, seed, n_roots=k, x=x)
    sign = {"EE": 0.0, "IP": -1.0, "EA": 1.0}[P.kind]
    print(f"case {name}: sigma at eps and eps + {C}", flush=True)
    h0 = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    h1 = adc.Handle(P.kind, P.o, P.v, P.eps + C, P.L, P.n_roots, x=P.x)
    assert h0.dim == h1.dim
    rng = np.random.default_rng(613)
    Y = torch.from_numpy(rng.standard_normal((2, h0.dim)) + 1j * rng.standard_normal((2, h0.dim))).cuda()
    for prec, tol in (("fp64", 1e-12), ("split_bf16", 2e-5)):
        S0 = h0.sigma(Y, precision=prec)
        S1 = h1.sigma(Y, precision=prec)
        torch.cuda.synchronize()
        scale = S0.abs().max().item()
        err = ((S1 - S0 - sign * C * Y).abs().max() / scale).item()
        print(f"  {prec}: max |S(eps + c) - S(eps) - {sign:+.0f} c Y| / max|S| = {err:.2e}", flush=True)
        assert err < tol, (name, prec, err)
        # the shift itself is far above the tolerance where it is not zero
        if sign != 0.0:
            assert C * Y.abs().max().item() / scale > 100 * tol
    h0.close()
    h1.close()
