"""GPU parity of the one-step pivoted Cholesky (adc_cholesky, Section 2.5,
eq. 41) and of the transform to the molecular basis (adc_cholesky_mo,
eq. 42) against the oracle, and the pipeline ERI -> vectors -> molecular
vectors -> sigma build.

The pivots are integers decided by comparisons of FP64 diagonal elements on
both sides: they must agree exactly.  Element i of vector k is
(V[p][i] - sum_{q<k} L_q[i] L_q[p]) / sqrt(d_p); each of the k products is at
most max|V| in size, so both sides round that sum to ~k u max|V| (u = 1.1e-16)
and the division by sqrt(d_p) magnifies it for the late vectors, whose pivot
elements d_p approach tau.  Vector k is compared within
1e-13 (k + 1) max|V| / sqrt(d_p), and the reconstruction L^T L, which carries
no such magnification, within 1e-12 max|V|.
"""
import numpy as np
import pytest

from adcgen import make_eri, mo_coefficients
from oracle.adc_terms import Ints
from oracle.adc_terms import sigma as osigma
from oracle.cholesky import mo_transform, pivoted_cholesky, unpack_pairs

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_ao,seed,tau,max_vec", [(12, 1, 1e-10, None), (40, 2, 1e-9, None), (40, 3, 1e-4, None),
                                                    (64, 4, 1e-8, 300), (96, 5, 1e-6, None)])
def test_cholesky_matches_oracle(n_ao, seed, tau, max_vec):
    print(f"case cholesky n_ao={n_ao} seed={seed} tau={tau} max_vec={max_vec}", flush=True)
    V = make_eri(n_ao, seed=seed)
    Lref, pref = pivoted_cholesky(V, tau, max_vec)
    L, piv = adc.cholesky(torch.from_numpy(V).cuda(), tau, max_vec)
    L = L.cpu().numpy()
    print(f"  {len(pref)} vectors (oracle), {len(piv)} (device)", flush=True)
    assert piv.tolist() == pref.tolist()
    vmax = np.abs(V).max()
    dp = Lref[np.arange(len(pref)), pref] ** 2
    tol = 1e-13 * (np.arange(len(pref)) + 1) * vmax / np.sqrt(dp)
    worst = (np.abs(L - Lref).max(axis=1) / tol).max()
    print(f"  worst vector difference / its bound {worst:.2e}", flush=True)
    assert worst <= 1.0
    assert np.abs(L.T @ L - Lref.T @ Lref).max() <= 1e-12 * vmax
    R = V - L.T @ L
    assert np.diag(R).max() < tau or len(piv) == max_vec


def test_cholesky_rank_deficient_and_errors():
    print("case cholesky rank 7 and bad input", flush=True)
    rng = np.random.default_rng(7)
    B = rng.standard_normal((300, 7))
    V = B @ B.T
    L, piv = adc.cholesky(torch.from_numpy(V).cuda(), 1e-10)
    assert len(piv) == 7
    assert np.abs(V - L.cpu().numpy().T @ L.cpu().numpy()).max() <= 1e-12 * np.abs(V).max()
    Vn = V.copy()
    Vn[3, 3] = np.nan
    with pytest.raises(adc.AdcError) as e:
        adc.cholesky(torch.from_numpy(Vn).cuda(), 1e-10)
    assert e.value.code == -2
    with pytest.raises(adc.AdcError) as e:
        adc.cholesky(torch.from_numpy(V).cuda(), -1.0)
    assert e.value.code == -1


def test_cholesky_to_sigma_pipeline():
    """ERI -> pivoted Cholesky -> molecular vectors -> EE sigma build, each
    step on the device, against the oracle's own pipeline."""
    print("case ERI -> Cholesky -> MO -> sigma", flush=True)
    n_ao, o = 16, 4
    V = make_eri(n_ao, seed=8) * 0.05
    Lref, _ = pivoted_cholesky(V, 1e-9)
    C = mo_coefficients(n_ao, n_ao, seed=9)
    Lmo_ref = mo_transform(unpack_pairs(Lref, n_ao), C)
    Ld, piv = adc.cholesky(torch.from_numpy(V).cuda(), 1e-9)
    Lmo = adc.cholesky_mo(Ld.contiguous(), n_ao, torch.from_numpy(C).cuda())
    # eq. 42 on the same vectors: FP64 GEMMs against the oracle's einsum
    Lmo_dev_ref = mo_transform(unpack_pairs(Ld.cpu().numpy(), n_ao), C)
    assert np.abs(Lmo.cpu().numpy() - Lmo_dev_ref).max() <= 1e-13 * np.abs(Lmo_dev_ref).max()
    eps = np.concatenate([np.sort(np.random.default_rng(10).uniform(-2.0, -0.3, o)),
                          np.sort(np.random.default_rng(11).uniform(0.1, 4.0, n_ao - o))])
    h = adc.Handle("EE", o, n_ao - o, eps, Lmo, 3, x=0.5)
    Y = np.random.default_rng(12).standard_normal((2, h.dim)) + 0j
    S = h.sigma(torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = osigma(Ints(eps, Lmo_ref, o), "EE", 0.5, Y)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    print(f"  sigma rel err {err:.2e}", flush=True)
    assert err < 1e-11
