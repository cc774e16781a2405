"""O2 (explicit terms, matrix-free) against O1 and against invariants of M.

O2's term list was identified by matching O1; here it is checked on shapes
and seeds not used for that, block by block and order by order, and then
through properties every correct M has (Hermiticity, spinor-phase gauge,
Q-mixing, real case, the L -> 0 limit, x-affinity), and its CPU Davidson
against dense diagonalisation.
"""
import numpy as np
import pytest

from adcgen import config_problem, make_problem
from oracle.adc_terms import Ints, block_matrix, dense_matrix, diag0, dims, sigma
from oracle.davidson import davidson, rayleigh_certificate
from oracle.isr import ISR, antisym_integrals

CASES = [("EE", 4, 6, 901), ("EE", 3, 7, 902), ("EE", 2, 5, 910), ("IP", 4, 7, 903),
         ("IP", 5, 6, 904), ("EA", 4, 6, 905), ("EA", 3, 7, 906), ("EE", 1, 6, 907),
         ("EA", 1, 6, 909)]


@pytest.mark.parametrize("kind,o,v,seed", CASES)
def test_blocks_match_isr(kind, o, v, seed):
    P = make_problem(kind, o, v, 15, seed=seed, scale=0.3)
    isr = ISR(kind, P.eps, antisym_integrals(P.L), o)
    ints = Ints(P.eps, P.L, o)
    for blk, orders in [("11", (0, 1, 2, 3)), ("12", (0, 1, 2)), ("21", (0, 1, 2)), ("22", (0, 1))]:
        for od in orders:
            a = isr.block(blk, od)
            if a.size == 0:
                continue
            assert np.abs(a - block_matrix(ints, kind, blk, od)).max() < 1e-12, (blk, od)
    for x in (0.0, 0.5, 1.0, 1.3):
        assert np.abs(isr.matrix(x) - dense_matrix(ints, kind, x)).max() < 1e-12


def _M(P, kind, x=1.0, L=None):
    return dense_matrix(Ints(P.eps, P.L if L is None else L, P.o), kind, x)


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_invariants(kind):
    o, v = 3, 6
    P = make_problem(kind, o, v, 25, seed=77, scale=0.2)
    M = _M(P, kind)
    w = np.linalg.eigvalsh(M)
    assert np.abs(M - M.conj().T).max() < 1e-14
    # spinor-phase gauge: L_pq -> e^{-i phi_p} L_pq e^{i phi_q}
    phi = np.random.default_rng(1).uniform(0, 2 * np.pi, o + v)
    Lg = np.exp(-1j * phi)[None, :, None] * P.L * np.exp(1j * phi)[None, None, :]
    assert np.abs(np.linalg.eigvalsh(_M(P, kind, L=Lg)) - w).max() < 1e-12
    # real orthogonal mixing of the Cholesky vectors leaves <pq||rs> unchanged
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((25, 25)))
    Lq = np.einsum("QP,Ppq->Qpq", Q, P.L)
    assert np.abs(_M(P, kind, L=Lq) - M).max() < 1e-13
    # x-affinity
    M0, Mh = _M(P, kind, 0.0), _M(P, kind, 0.5)
    assert np.abs(Mh - 0.5 * (M0 + M)).max() < 1e-14
    # real L gives a real symmetric M
    Mr = _M(P, kind, L=P.L.real.astype(np.complex128))
    assert np.abs(Mr.imag).max() < 1e-15 and np.abs(Mr - Mr.T).max() < 1e-14
    # L -> 0: eigenvalues are the zeroth-order energies
    ints0 = Ints(P.eps, 0 * P.L, o)
    d = np.sort(np.concatenate([diag0(ints0, kind, 1), diag0(ints0, kind, 2)]))
    assert np.abs(np.linalg.eigvalsh(_M(P, kind, L=0 * P.L)) - d).max() < 1e-14


@pytest.mark.parametrize("kind,o,v", [("EE", 4, 9), ("IP", 5, 10), ("EA", 4, 9)])
def test_davidson_matches_dense(kind, o, v):
    P = make_problem(kind, o, v, 40, seed=12)
    ints = Ints(P.eps, P.L, o)
    M = dense_matrix(ints, kind, 1.0)
    w = np.linalg.eigvalsh(M)[:4]
    n1 = dims(kind, o, v)[0]
    d = np.concatenate([diag0(ints, kind, 1), diag0(ints, kind, 2)])
    wd, X, rn, it, conv = davidson(lambda Y: sigma(ints, kind, 1.0, Y), d, np.diag(M).real[:n1], 4, tol=1e-8)
    assert conv.all()
    assert np.abs(wd - w).max() < 1e-10
    theta, r = rayleigh_certificate(lambda Y: sigma(ints, kind, 1.0, Y), X)
    assert np.abs(theta - w).max() < 1e-10 and r.max() < 1e-7


@pytest.mark.slow
def test_c1_davidson_vs_dense_eigh():
    P = config_problem("C1")
    ints = Ints(P.eps, P.L, P.o)
    M = dense_matrix(ints, "EE", P.x)
    w = np.linalg.eigvalsh(M)[:4]
    n1 = dims("EE", P.o, P.v)[0]
    d = np.concatenate([diag0(ints, "EE", 1), diag0(ints, "EE", 2)])
    wd, X, rn, it, conv = davidson(lambda Y: sigma(ints, "EE", P.x, Y), d, np.diag(M).real[:n1], 4)
    assert np.abs(wd - w).max() < 1e-10


@pytest.mark.parametrize("kind,o,v", [("EE", 3, 6), ("IP", 4, 6), ("EA", 3, 7)])
def test_dense_singles_block_equals_matrix_free(kind, o, v):
    """m11_block forms the singles block densely from the same term lines that
    sigma applies matrix-free; both must agree (the dense form serves the
    Davidson guesses of the tests)."""
    from oracle.adc_terms import m11_block, sigma_block
    P = make_problem(kind, o, v, 20, seed=31, scale=0.3)
    ints = Ints(P.eps, P.L, o)
    E = np.eye(dims(kind, o, v)[0], dtype=complex)
    for od in range(4):
        mf = sigma_block(ints, kind, "11", od, E, dense_singles=False).T
        assert np.abs(m11_block(ints, kind, od) - mf).max() < 1e-14, od


def test_pairwise_contraction_equals_einsum():
    """The oracle evaluates each term line pair by pair as batched matrix
    products (oracle.adc_terms.contract); on every line of the term table,
    with random factors and the labels' delta substitutions, it must equal a
    plain einsum of the same line."""
    from oracle.adc_terms import TERMS, BRA, OCC, contract, parse_term
    rng = np.random.default_rng(5)
    o, v = 3, 4
    for (kind, blk, od), lines in TERMS.items():
        r, c = int(blk[0]), int(blk[1])
        out_l, in_l = BRA[(kind, r)], BRA[(kind, c)].upper()
        for line in lines:
            _, factors, deltas = parse_term(line)
            sub = {}
            for a, b in deltas:
                if a in out_l:
                    sub[b] = a
                else:
                    sub[a] = b
            subs = ["".join(sub.get(ch, ch) for ch in lab) for _, lab in factors]
            ysub = "z" + "".join(sub.get(ch, ch) for ch in in_l)
            spec = ",".join(subs + [ysub]) + "->z" + out_l
            size = lambda ch: 2 if ch == "z" else (o if ch in OCC else v)  # noqa: E731
            ops = [rng.standard_normal([size(ch) for ch in lab]) + 1j * rng.standard_normal([size(ch) for ch in lab])
                   for lab in spec.split("->")[0].split(",")]
            ref = np.einsum(spec, *ops)
            assert np.abs(contract(spec, *ops) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), (kind, line)


@pytest.mark.parametrize("kind", ["IP", "EA"])
def test_adc2_column_depends_only_on_its_orbitals(kind):
    """At x = 0 the column of a doubles basis state holds the first-order
    coupling and the zeroth-order diagonal only, so it is the same column of
    the sub-problem of the orbitals it involves: IP (k<l, b) all occupied
    orbitals and b alone as the virtual space, EA (i, a<b) i alone as the
    occupied space and all virtual orbitals (the reading the full-size C3
    parity tests rely on).  Checked against the full problem at small sizes,
    where the sub-problem must not need the <vv||vv> class."""
    o, v = (5, 6) if kind == "IP" else (4, 7)
    P = make_problem(kind, o, v, 30, seed=77, n_roots=2, x=0.0)
    full = Ints(P.eps, P.L, o)
    n1, n2 = dims(kind, o, v)
    Pv = v * (v - 1) // 2
    # IP (k, l, b) with k < l; EA (i, a, b) with a < b
    states = [(0, 1, 0), (1, 3, 5), (2, 3, 2)] if kind == "IP" else [(0, 2, 3), (1, 4, 6), (2, 4, 5)]
    for (p, q, r) in states:
        if kind == "IP":
            pk = p * (2 * o - p - 1) // 2 + (q - p - 1)
            pos, pos_sub = pk * v + r, pk
            idx, o_sub = list(range(o)) + [o + r], o
            D = P.eps[o + r] - P.eps[p] - P.eps[q]
        else:
            i, a, b = p, q, r
            pab = a * (2 * v - a - 1) // 2 + (b - a - 1)
            pos, pos_sub = i * Pv + pab, pab
            idx, o_sub = [i] + list(range(o, o + v)), 1
            D = P.eps[o + a] + P.eps[o + b] - P.eps[i]
        Y = np.zeros((1, n1 + n2), dtype=np.complex128)
        Y[0, n1 + pos] = 1.0
        col = sigma(full, kind, 0.0, Y)[0]
        sub = Ints(P.eps[idx], P.L[:, idx][:, :, idx], o_sub)
        n1s, n2s = dims(kind, o_sub, len(idx) - o_sub)
        Ys = np.zeros((1, n1s + n2s), dtype=np.complex128)
        Ys[0, n1s + pos_sub] = 1.0
        ref = sigma(sub, kind, 0.0, Ys)[0]
        assert np.abs(col[:n1] - ref[:n1]).max() <= 1e-13 * np.abs(col[:n1]).max()
        assert np.abs(col[:n1]).max() > 1e-6
        d = np.zeros(n2, dtype=np.complex128)
        d[pos] = D
        assert np.abs(col[n1:] - d).max() <= 1e-14
        assert "vvvv" not in sub._g


@pytest.mark.parametrize("kind,sign", [("EE", 0.0), ("IP", -1.0), ("EA", 1.0)])
def test_uniform_orbital_energy_shift(kind, sign):
    """Every denominator of the perturbation series (§2.1, the MP amplitudes
    and the ADC blocks order by order) is a difference with as many occupied
    as virtual energies, so eps -> eps + c shifts the Hamiltonian by c times
    the particle number and leaves all of them alone: M moves by the change of
    particle number times c (EE 0, IP -c, EA +c), all of it in the zeroth-order
    diagonal blocks.  Checked on the Fock-space construction (O1) and block by
    block, order by order on the matrix-free terms, where a wrong sign or
    index in any energy denominator breaks it."""
    o, v, c = 3, 5, 0.731
    P = make_problem(kind, o, v, 20, seed=314, scale=0.3)
    n1, n2 = dims(kind, o, v)
    g = antisym_integrals(P.L)
    for x in (0.0, 1.0):
        dM = ISR(kind, P.eps + c, g, o).matrix(x) - ISR(kind, P.eps, g, o).matrix(x)
        assert np.abs(dM - sign * c * np.eye(n1 + n2)).max() < 1e-12, x
    ints, ints_c = Ints(P.eps, P.L, o), Ints(P.eps + c, P.L, o)
    for blk, orders in [("11", (0, 1, 2, 3)), ("12", (0, 1, 2)), ("21", (0, 1, 2)), ("22", (0, 1))]:
        for od in orders:
            a, b = block_matrix(ints, kind, blk, od), block_matrix(ints_c, kind, blk, od)
            if a.size == 0:
                continue
            ref = sign * c * np.eye(a.shape[0]) if (od == 0 and blk[0] == blk[1]) else 0.0
            assert np.abs(b - a - ref).max() < 1e-12, (blk, od)
            if od >= 2 or (od == 1 and blk != "11"):
                assert np.abs(a).max() > 1e-6, (blk, od)  # the block is not trivially zero


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_block_order_is_its_degree_in_the_integrals(kind):
    """L -> s L scales every antisymmetrised integral by s^2 (eq. 43) and
    leaves the orbital energies alone, so the order-n part of each block
    (section 2.1: n powers of the fluctuation potential, counting each MP
    amplitude by its own order) scales as s^(2n) exactly.  A term filed under
    the wrong order, or missing or repeating an integral or amplitude
    factor, breaks it."""
    o, v, s = 3, 5, 1.7
    P = make_problem(kind, o, v, 20, seed=2718, scale=0.3)
    ints, ints_s = Ints(P.eps, P.L, o), Ints(P.eps, s * P.L, o)
    for blk, orders in [("11", (0, 1, 2, 3)), ("12", (1, 2)), ("21", (1, 2)), ("22", (0, 1))]:
        for od in orders:
            a, b = block_matrix(ints, kind, blk, od), block_matrix(ints_s, kind, blk, od)
            if a.size == 0 or np.abs(a).max() == 0.0:
                continue
            assert np.abs(b - s ** (2 * od) * a).max() <= 1e-12 * np.abs(b).max(), (blk, od)
