"""Parity at the full benchmark sizes, where the oracle cannot form the whole
matrix: on outputs it can compute, and through properties that hold at any
size.

* C2 (EE, the timed workload): the complete sigma build for one trial vector
  whose singles part is zero (only the M12 and M22 blocks of the oracle),
  and for a general vector (every block, M11 included, from the oracle's
  matrix-free sigma), FP64, FP32 and split-bf16, in the launch configuration
  bench.py times;
* C3-EA: sampled rows of the particle-particle ladder, each <ab||cd> row formed
  by the oracle from L on its own; Hermiticity of the whole sigma;
* C3-IP: Hermiticity of the whole sigma;
* C3-IP and C3-EA at x = 0: whole columns of M (unit doubles vectors: the
  first-order coupling in the singles, the diagonal in the doubles), each
  from the oracle on the sub-problem of the orbitals that column involves.
"""
import numpy as np
import pytest

from adcgen import config_problem
from oracle.adc_terms import Ints, dims, sigma, sigma_block

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402

pytestmark = pytest.mark.gpu


def _herm_check(h, rng):
    """FP64 <Z, M Y> - <M Z, Y>, relative to max|MY| sum|Z|."""
    Y = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    Z = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    SY, SZ = h.sigma(Y, precision="fp64"), h.sigma(Z, precision="fp64")
    a = (Z.conj() * SY).sum(1)
    b = (SZ.conj() * Y).sum(1)
    return ((a - b).abs().max() / (SY.abs().max() * Z.abs().sum())).item()


def test_c2_full_sigma_doubles_input():
    P = config_problem("C2")
    print("case C2 EE full sigma, zero-singles trial vector", flush=True)
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    n1, n2 = dims("EE", P.o, P.v)
    rng = np.random.default_rng(22)
    Y = np.zeros((1, n1 + n2), complex)
    Y[0, n1:] = rng.standard_normal(n2) + 1j * rng.standard_normal(n2)
    S64 = h.sigma(torch.from_numpy(Y).cuda(), precision="fp64").cpu().numpy()
    S32 = h.sigma(torch.from_numpy(Y).cuda(), precision="fp32").cpu().numpy()
    Sbf = h.sigma(torch.from_numpy(Y).cuda(), precision="split_bf16").cpu().numpy()
    ints = Ints(P.eps, P.L, P.o)
    Y2 = Y[:, n1:]
    ref1 = sigma_block(ints, "EE", "12", 1, Y2) + P.x * sigma_block(ints, "EE", "12", 2, Y2)
    ref2 = sigma_block(ints, "EE", "22", 0, Y2) + P.x * sigma_block(ints, "EE", "22", 1, Y2)
    ref = np.concatenate([ref1, ref2], axis=1)
    e64 = np.abs(S64 - ref).max() / np.abs(ref).max()
    e32 = np.abs(S32 - ref).max() / np.abs(ref).max()
    ebf = np.abs(Sbf - ref).max() / np.abs(ref).max()
    print("C2 rel err fp64", e64, "fp32", e32, "split-bf16", ebf)
    assert e64 < 1e-12
    assert e32 < 1e-6
    # split-bf16 (the arithmetic bench.py times): 16 significant bits per
    # operand, one split product per term (see the ladder test below for two)
    assert 1e-12 < ebf < 1e-5


def test_c2_full_sigma_general_vector():
    """Every block of M (eq. 11), singles included, at the benchmark size."""
    P = config_problem("C2")
    print("case C2 EE full sigma, general trial vector", flush=True)
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    rng = np.random.default_rng(23)
    Y = rng.standard_normal((1, h.dim)) + 1j * rng.standard_normal((1, h.dim))
    Yd = torch.from_numpy(Y).cuda()
    S64 = h.sigma(Yd, precision="fp64").cpu().numpy()
    S32 = h.sigma(Yd, precision="fp32").cpu().numpy()
    Sbf = h.sigma(Yd, precision="split_bf16").cpu().numpy()
    h.close()
    ref = sigma(Ints(P.eps, P.L, P.o), "EE", P.x, Y)
    e64 = np.abs(S64 - ref).max() / np.abs(ref).max()
    e32 = np.abs(S32 - ref).max() / np.abs(ref).max()
    ebf = np.abs(Sbf - ref).max() / np.abs(ref).max()
    print("C2 general vector rel err fp64", e64, "fp32", e32, "split-bf16", ebf)
    assert e64 < 1e-12
    assert e32 < 1e-6
    # the particle-particle ladder chains two split products (reading of the
    # tolerances: about 2 * 2^-16 of the output scale at most)
    assert 1e-12 < ebf < 3e-5


def test_c3_ea_ladder_rows_and_hermiticity():
    P = config_problem("C3-EA")
    print("case C3-EA ladder rows + hermiticity", flush=True)
    h = adc.Handle("EA", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, precision="fp32", mem_budget=32 << 30)
    rng = np.random.default_rng(32)
    Y = torch.from_numpy(rng.standard_normal((2, h.dim)) + 1j * rng.standard_normal((2, h.dim))).cuda()
    S = h.sigma_term("ladder", Y, precision="fp64").cpu().numpy()
    Sbf = h.sigma_term("ladder", Y, precision="split_bf16").cpu().numpy()
    Yh = Y.cpu().numpy()
    o, v = P.o, P.v
    Lvv = P.L[:, o:, o:]
    iu = np.triu_indices(v, 1)
    Pv = len(iu[0])
    worst = worst_bf = 0.0
    for (i, a, b) in [(0, 0, 1), (7, 3, 250), (59, 398, 399), (31, 100, 101), (12, 5, 377), (44, 250, 251)]:
        W = np.einsum("Qc,Qd->cd", Lvv[:, a, :], Lvv[:, b, :])
        g = (W - W.T)[iu]                       # <ab||cd>, c<d
        p = a * (2 * v - a - 1) // 2 + (b - a - 1)
        ref = P.x * (Yh[:, v + i * Pv: v + (i + 1) * Pv] @ g)
        got = S[:, v + i * Pv + p]
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
        worst_bf = max(worst_bf, np.abs(Sbf[:, v + i * Pv + p] - ref).max() / np.abs(ref).max())
    print("C3-EA ladder sampled rel err", worst, "split-bf16", worst_bf)
    assert worst < 1e-12
    # two split-bf16 products in a row (the <ab||cd> assembly over N = 2400,
    # then the contraction over P_v = 79,800): each operand split carries up
    # to 2^-16 relative error and the three-product form drops lo*lo'
    # (<= 2^-16), so each product term is off by ~2^-16 of its size at
    # random; the two chained products give ~2 * 2^-16 = 3e-5 relative to the
    # output scale
    assert worst_bf < 3e-5
    assert _herm_check(h, rng) < 1e-13


def test_c3_ip_hermiticity():
    P = config_problem("C3-IP")
    print("case C3-IP hermiticity", flush=True)
    h = adc.Handle("IP", P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    assert _herm_check(h, np.random.default_rng(31)) < 1e-13


def _pidx(k, l, n):
    """Packed position of the pair k < l among n orbitals."""
    return k * (2 * n - k - 1) // 2 + (l - k - 1)


def test_c3_ip_coupling_columns_at_x0():
    """C3-IP at x = 0 (ADC(2), Section 2.1 eq. 10): for a unit doubles vector
    e_d, d = (k<l, b), the build returns column d of M: the first-order
    coupling M12[:, d] in the singles, D_d = e_b - e_k - e_l at d and zero in
    the rest of the doubles.  That column involves only the occupied orbitals
    and the virtual b (each element one antisymmetrised integral, eq. 43), so
    the oracle computes it on the sub-problem of those orbitals: all o
    occupied and b alone as the virtual space."""
    P = config_problem("C3-IP")
    o, v = P.o, P.v
    print("case C3-IP coupling columns at x=0", flush=True)
    h = adc.Handle("IP", o, v, P.eps, P.L, P.n_roots, x=0.0)
    cols = [(0, 1, 0), (17, 42, 399), (58, 59, 200), (3, 31, 123)]
    pos = [o + _pidx(k, l, o) * v + b for (k, l, b) in cols]
    Y = torch.zeros((len(cols), h.dim), dtype=torch.complex128)
    for r, q in enumerate(pos):
        Y[r, q] = 1.0
    Y = Y.cuda()
    S64 = h.sigma(Y, precision="fp64").cpu().numpy()
    Sbf = h.sigma(Y, precision="split_bf16").cpu().numpy()
    h.close()
    n1s, n2s = dims("IP", o, 1)
    worst = worst_bf = 0.0
    for r, (k, l, b) in enumerate(cols):
        idx = list(range(o)) + [o + b]
        sub = Ints(P.eps[idx], P.L[:, idx][:, :, idx], o)
        Ys = np.zeros((1, n1s + n2s), dtype=np.complex128)
        Ys[0, n1s + _pidx(k, l, o)] = 1.0
        ref = sigma(sub, "IP", 0.0, Ys)[0]
        D = P.eps[o + b] - P.eps[k] - P.eps[l]
        # the oracle's own column: its diagonal entry is D_d
        assert abs(ref[n1s + _pidx(k, l, o)] - D) < 1e-14 * abs(D)
        scale = np.abs(ref[:o]).max()
        assert scale > 0
        worst = max(worst, np.abs(S64[r, :o] - ref[:o]).max() / scale)
        worst_bf = max(worst_bf, np.abs(Sbf[r, :o] - ref[:o]).max() / scale)
        for S in (S64, Sbf):
            assert abs(S[r, pos[r]] - D) < 1e-12 * abs(D)
            rest = S[r, o:].copy()
            rest[pos[r] - o] = 0.0
            assert np.abs(rest).max() == 0.0
    print(f"C3-IP coupling columns: rel err fp64 {worst:.1e}, split-bf16 {worst_bf:.1e}", flush=True)
    assert worst < 1e-12
    # one split-bf16 product per coupling element (the stored integral class
    # times the unit vector): each split carries at most 2^-16 relative error
    assert worst_bf < 3e-5


def test_c3_ea_coupling_columns_at_x0():
    """C3-EA at x = 0 (ADC(2), Section 2.1 eq. 10): for a unit doubles vector
    e_d, d = (i, a<b), the build returns column d of M: the first-order
    coupling M12[:, d] in the singles (from the stored three-external class),
    D_d = e_a + e_b - e_i at d and zero in the rest of the doubles.  That
    column involves only the occupied orbital i and the virtual orbitals, so
    the oracle computes it on the sub-problem with i alone as the occupied
    space (no <vv||vv> class is needed there)."""
    P = config_problem("C3-EA")
    o, v = P.o, P.v
    Pv = v * (v - 1) // 2
    print("case C3-EA coupling columns at x=0", flush=True)
    h = adc.Handle("EA", o, v, P.eps, P.L, P.n_roots, x=0.0)
    cols = [(0, 0, 1), (31, 17, 398), (59, 200, 201)]
    pos = [v + i * Pv + _pidx(a, b, v) for (i, a, b) in cols]
    Y = torch.zeros((len(cols), h.dim), dtype=torch.complex128)
    for r, q in enumerate(pos):
        Y[r, q] = 1.0
    Y = Y.cuda()
    S64 = h.sigma(Y, precision="fp64").cpu().numpy()
    Sbf = h.sigma(Y, precision="split_bf16").cpu().numpy()
    h.close()
    n1s, n2s = dims("EA", 1, v)
    worst = worst_bf = 0.0
    for r, (i, a, b) in enumerate(cols):
        idx = [i] + list(range(o, o + v))
        sub = Ints(P.eps[idx], P.L[:, idx][:, :, idx], 1)
        Ys = np.zeros((1, n1s + n2s), dtype=np.complex128)
        Ys[0, n1s + _pidx(a, b, v)] = 1.0
        ref = sigma(sub, "EA", 0.0, Ys)[0]
        D = P.eps[o + a] + P.eps[o + b] - P.eps[i]
        assert abs(ref[n1s + _pidx(a, b, v)] - D) < 1e-14 * abs(D)
        scale = np.abs(ref[:v]).max()
        assert scale > 0
        worst = max(worst, np.abs(S64[r, :v] - ref[:v]).max() / scale)
        worst_bf = max(worst_bf, np.abs(Sbf[r, :v] - ref[:v]).max() / scale)
        for S in (S64, Sbf):
            assert abs(S[r, pos[r]] - D) < 1e-12 * abs(D)
            rest = S[r, v:].copy()
            rest[pos[r] - v] = 0.0
            assert np.abs(rest).max() == 0.0
    print(f"C3-EA coupling columns: rel err fp64 {worst:.1e}, split-bf16 {worst_bf:.1e}", flush=True)
    assert worst < 1e-12
    # one split-bf16 product per coupling element: at most 2^-16 relative
    # error per split
    assert worst_bf < 3e-5
