"""Pins of the oracle gradient (oracle.grad) on the CPU.

The torch evaluation must reproduce the numpy oracle's sigma, and its
autograd gradient must match central finite differences of the numpy oracle
(an independent route: no derivative is formed by hand anywhere).  The
eigenvalue form (Hellmann-Feynman, M Hermitian by Section 2.1, eq. 10) is
pinned against finite differences of dense eigenvalues."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from adcgen import make_problem  # noqa: E402
from oracle.adc_terms import Ints, dense_matrix, dims, sigma  # noqa: E402
from oracle.grad import TorchInts, functional, herm_project, sigma_t, vjp  # noqa: E402

CASES = [("EE", 3, 6, 12, 1.0, 1), ("EE", 2, 5, 8, 0.5, 2), ("EE", 1, 5, 8, 1.0, 3), ("IP", 3, 5, 10, 0.5, 4),
         ("IP", 1, 4, 6, 1.0, 5), ("EA", 3, 5, 10, 0.7, 6), ("EA", 2, 4, 6, 0.0, 7)]


def _herm(rng, shape):
    E = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return 0.5 * (E + np.conj(np.transpose(E, (0, 2, 1))))


def _vecs(rng, k, dim):
    return rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))


@pytest.mark.parametrize("kind,o,v,N,x,seed", CASES)
def test_torch_sigma_equals_numpy_oracle(kind, o, v, N, x, seed):
    P = make_problem(kind, o, v, N, seed=seed, x=x, scale=0.2)
    rng = np.random.default_rng(seed)
    n1, n2 = dims(kind, o, v)
    Y = _vecs(rng, 2, n1 + n2)
    ref = sigma(Ints(P.eps, P.L, o), kind, x, Y)
    got = sigma_t(TorchInts(P.eps, torch.from_numpy(P.L), o), kind, x, torch.from_numpy(Y)).numpy()
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("kind,o,v,N,x,seed", CASES)
def test_gradient_matches_finite_differences(kind, o, v, N, x, seed):
    P = make_problem(kind, o, v, N, seed=seed, x=x, scale=0.2)
    rng = np.random.default_rng(100 + seed)
    n1, n2 = dims(kind, o, v)
    Y, Sb = _vecs(rng, 2, n1 + n2), _vecs(rng, 2, n1 + n2)
    G, dx = vjp(kind, P.eps, P.L, o, x, Y, Sb)
    # the projection is idempotent and leaves a Hermitian gradient
    assert np.abs(herm_project(G) - G).max() == 0.0
    h = 1e-5
    for _ in range(2):
        E = _herm(rng, P.L.shape)
        fd = (functional(kind, P.eps, P.L + h * E, o, x, Y, Sb)
              - functional(kind, P.eps, P.L - h * E, o, x, Y, Sb)) / (2 * h)
        an = float(np.real(np.sum(np.conj(G) * E)))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
    fdx = (functional(kind, P.eps, P.L, o, x + h, Y, Sb) - functional(kind, P.eps, P.L, o, x - h, Y, Sb)) / (2 * h)
    assert abs(fdx - dx) <= 1e-7 * max(1.0, abs(dx)), (fdx, dx)


def test_eigenvalue_gradient_is_hellmann_feynman():
    """d omega_r along a Hermitian dL equals Re <G(y_r, y_r), dL>, checked
    against central differences of dense eigenvalues."""
    kind, o, v, N, x = "EE", 2, 4, 6, 1.0
    P = make_problem(kind, o, v, N, seed=9, x=x, scale=0.2)
    w, U = np.linalg.eigh(dense_matrix(Ints(P.eps, P.L, o), kind, x))
    rng = np.random.default_rng(9)
    E = _herm(rng, P.L.shape)
    h = 1e-5
    wp = np.linalg.eigh(dense_matrix(Ints(P.eps, P.L + h * E, o), kind, x))[0]
    wm = np.linalg.eigh(dense_matrix(Ints(P.eps, P.L - h * E, o), kind, x))[0]
    for r in range(3):
        assert min(abs(w[r] - w[r - 1]) if r else 1.0, abs(w[r + 1] - w[r])) > 1e-6
        y = U[:, r][None, :]
        G, dx = vjp(kind, P.eps, P.L, o, x, y, y)
        an = float(np.real(np.sum(np.conj(G) * E)))
        fd = (wp[r] - wm[r]) / (2 * h)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (r, fd, an)
