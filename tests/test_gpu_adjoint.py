"""GPU parity of the adjoint of the sigma build (adc_sigma_backward) and of the
torch.autograd bindings.

* Vector-Jacobian product: dL and dx of f = Re sum_z Sbar_z^H M(L, x) Y_z
  against the oracle gradient (torch CPU autograd of the oracle's terms),
  elementwise, max|d dL| / max|dL| <= 1e-11, on seeded Y and Sbar.
* Eigenvalue gradients (Hellmann-Feynman): directional derivatives against
  central finite differences of the FP64 GPU eigenvalues (h = 1e-5).
"""
import numpy as np
import pytest

from adcgen import config_problem, make_problem
from oracle.adc_terms import sigma as osigma, Ints
from oracle.grad import vjp

torch = pytest.importorskip("torch")
import paper_2511_21640_amd as adc  # noqa: E402
from paper_2511_21640_amd.autograd import ADCRoots, ADCSigma  # noqa: E402

pytestmark = pytest.mark.gpu


def _rand(rng, k, dim):
    return rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))


def _herm(rng, shape):
    E = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return 0.5 * (E + np.conj(np.transpose(E, (0, 2, 1))))


CASES = [("EE", 3, 6, 20, 1.0, 1), ("EE", 4, 7, 30, 0.5, 2), ("EE", 2, 5, 10, 0.0, 3), ("EE", 1, 6, 10, 1.0, 4),
         ("EE", 6, 21, 70, 0.7, 5),
         ("IP", 3, 6, 20, 1.0, 6), ("IP", 4, 7, 24, 0.5, 7), ("IP", 1, 5, 8, 1.0, 8),
         ("EA", 3, 6, 20, 1.0, 9), ("EA", 4, 7, 24, 0.5, 10), ("EA", 1, 6, 10, 1.0, 11), ("EA", 5, 17, 50, 0.8, 12)]


def _check_vjp(P, k, seed, **kw):
    h = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, **kw)
    rng = np.random.default_rng(seed)
    Y, Sb = _rand(rng, k, h.dim), _rand(rng, k, h.dim)
    dL, dx = h.sigma_backward(torch.from_numpy(Sb).cuda(), torch.from_numpy(Y).cuda())
    dL = dL.cpu().numpy()
    ref, rdx = vjp(P.kind, P.eps, P.L, P.o, P.x, Y, Sb)
    scale = np.abs(ref).max()
    if scale == 0.0:
        # IP with one occupied spinor: M = -e_0 does not depend on L; the
        # device sweep cancels the two exchange terms only up to rounding
        assert np.abs(dL).max() <= 1e-13
    else:
        err = np.abs(dL - ref).max() / scale
        assert err <= 1e-11, err
    assert abs(dx - rdx) <= 1e-11 * max(1.0, abs(rdx)), (dx, rdx)
    h.close()


@pytest.mark.parametrize("kind,o,v,N,x,seed", CASES)
def test_vjp_matches_oracle_gradient(kind, o, v, N, x, seed):
    print(f"case {kind} o={o} v={v} N={N} x={x} seed={seed}", flush=True)
    P = make_problem(kind, o, v, N, seed=seed, x=x, scale=0.2)
    _check_vjp(P, 2, seed)


@pytest.mark.parametrize("kind", ["EE", "IP", "EA"])
def test_vjp_small_workspace(kind):
    """A tiny workspace splits every batch (ladder, its adjoint, M11 pieces)."""
    print(f"case {kind} tiny mem_budget", flush=True)
    P = make_problem(kind, 4, 9, 30, seed=21, x=0.9, scale=0.2)
    _check_vjp(P, 3, 21, mem_budget=1 << 16)


def test_autograd_sigma_matches_library_and_oracle():
    print("case ADCSigma EE o=3 v=7", flush=True)
    P = make_problem("EE", 3, 7, 24, seed=31, x=0.6, scale=0.2)
    spec = dict(kind="EE", o=P.o, v=P.v, eps=P.eps)
    rng = np.random.default_rng(31)
    n = P.o + P.v
    L = torch.from_numpy(P.L).cuda().requires_grad_(True)
    x = torch.tensor(P.x, dtype=torch.float64, device="cuda", requires_grad=True)
    h0 = adc.Handle("EE", P.o, P.v, P.eps, P.L, 1, x=P.x)
    Y = torch.from_numpy(_rand(rng, 2, h0.dim)).cuda().requires_grad_(True)
    W = torch.from_numpy(_rand(rng, 2, h0.dim)).cuda()
    S = ADCSigma.apply(L, x, Y, spec)
    f = torch.real((W.conj() * S).sum())
    gL, gx, gY = torch.autograd.grad(f, (L, x, Y))
    refL, refx = vjp("EE", P.eps, P.L, P.o, P.x, Y.detach().cpu().numpy(), W.cpu().numpy())
    assert gL.shape == (P.L.shape[0], n, n)
    assert np.abs(gL.cpu().numpy() - refL).max() <= 1e-11 * np.abs(refL).max()
    assert abs(gx.item() - refx) <= 1e-11 * max(1.0, abs(refx))
    # G_Y = M^H W = M W
    refY = osigma(Ints(P.eps, P.L, P.o), "EE", P.x, W.cpu().numpy())
    assert np.abs(gY.cpu().numpy() - refY).max() <= 1e-12 * np.abs(refY).max()
    h0.close()


def _omegas(P, L, x, k, tol=1e-9):
    h = adc.Handle(P.kind, P.o, P.v, P.eps, L, k, x=x, precision="fp64", conv_tol=tol, max_iter=300)
    r = h.davidson(want_vectors=False)
    h.close()
    assert r["converged"].all()
    return r["omega"]


def _fd_check(P, k, dirs_seed, restrict_q=None, tol=1e-6):
    spec = dict(kind=P.kind, o=P.o, v=P.v, eps=P.eps, n_roots=k, conv_tol=1e-9, max_iter=300)
    L = torch.from_numpy(P.L).cuda().requires_grad_(True)
    x = torch.tensor(P.x, dtype=torch.float64, device="cuda", requires_grad=True)
    w = ADCRoots.apply(L, x, spec)
    wn = w.detach().cpu().numpy()
    gaps = np.diff(wn)
    assert (gaps > 1e-8).all(), "degenerate roots: gradients undefined"
    grads = []
    for r in range(k):
        gL, gx = torch.autograd.grad(w[r], (L, x), retain_graph=True)
        grads.append((gL.cpu().numpy(), gx.item()))
    rng = np.random.default_rng(dirs_seed)
    E = _herm(rng, P.L.shape)
    if restrict_q is not None:
        E[restrict_q:] = 0.0
    E /= np.linalg.norm(E)
    G0 = grads[0][0]
    dirs = [E, G0 / np.linalg.norm(G0)]
    h = 1e-5
    for D in dirs:
        wp = _omegas(P, P.L + h * D, P.x, k)
        wm = _omegas(P, P.L - h * D, P.x, k)
        for r in range(k):
            an = float(np.real(np.sum(np.conj(grads[r][0]) * D)))
            fd = (wp[r] - wm[r]) / (2 * h)
            print(f"root {r}: dL analytic {an:.10e} fd {fd:.10e}", flush=True)
            assert abs(an - fd) <= tol * max(1.0, abs(an)), (r, an, fd)
    wp = _omegas(P, P.L, P.x + h, k)
    wm = _omegas(P, P.L, P.x - h, k)
    for r in range(k):
        fd = (wp[r] - wm[r]) / (2 * h)
        print(f"root {r}: dx analytic {grads[r][1]:.10e} fd {fd:.10e}", flush=True)
        assert abs(grads[r][1] - fd) <= tol * max(1.0, abs(fd)), (r, grads[r][1], fd)


@pytest.mark.parametrize("kind,o,v,N,seed", [("EE", 4, 10, 30, 41), ("IP", 4, 9, 30, 42), ("EA", 4, 9, 30, 43)])
def test_root_gradients_match_finite_differences(kind, o, v, N, seed):
    print(f"case roots {kind} o={o} v={v} N={N}", flush=True)
    P = make_problem(kind, o, v, N, seed=seed, x=1.0, scale=0.2, n_roots=3)
    _fd_check(P, 3, seed)


@pytest.mark.slow
def test_c5_root_gradients_match_finite_differences():
    """The adjoint configuration: 4 lowest EE-ADC(3) roots at o=16, v=96,
    Nchol=600; directions: a random Hermitian dL on Q < 30 (unit norm), the
    gradient direction, and x."""
    print("case C5 root gradients", flush=True)
    P = config_problem("C5")
    _fd_check(P, P.n_roots, 55, restrict_q=30)


def test_c5_vjp_matches_oracle_gradient():
    """Adjoint configuration (EE-ADC(3), o=16, v=96, Nchol=600): the device dL
    and dx against the oracle gradient stored by tests/golden/make_c5_adjoint.py
    (sampled and largest entries, norms, directional derivatives)."""
    import json
    import os
    import time

    from adcgen import hermitian_direction, trial_vectors

    print("case C5 vjp vs stored oracle gradient", flush=True)
    with open(os.path.join(os.path.dirname(__file__), "golden", "c5_adjoint.json")) as f:
        ref = json.load(f)
    P = config_problem(ref["config"])
    h = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    Y = torch.from_numpy(trial_vectors(ref["k"], h.dim, ref["y_seed"])).cuda()
    Sb = torch.from_numpy(trial_vectors(ref["k"], h.dim, ref["sbar_seed"])).cuda()
    h.sigma_backward(Sb, Y)  # warm the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dL, dx = h.sigma_backward(Sb, Y)
    torch.cuda.synchronize()
    print(f"C5 backward {1e3 * (time.perf_counter() - t0):.0f} ms (init {h.init_ms:.0f} ms)", flush=True)
    G = dL.cpu().numpy()
    flat = G.reshape(-1)
    mx = ref["max_abs"]
    for i, re, im in ref["samples"] + ref["top"]:
        assert abs(flat[i] - complex(re, im)) <= 1e-11 * mx, (i, flat[i], re, im)
    assert abs(np.abs(flat).max() - mx) <= 1e-11 * mx
    assert abs(np.linalg.norm(flat) - ref["fro"]) <= 1e-11 * ref["fro"]
    for pr in ref["projections"]:
        D = hermitian_direction(P.L.shape, pr["seed"], restrict_q=pr["restrict_q"])
        got = float(np.real(np.vdot(G, D)))
        assert abs(got - pr["value"]) <= 1e-10 * ref["fro"], (pr, got)
    assert abs(dx - ref["dx"]) <= 1e-11 * max(1.0, abs(ref["dx"])), (dx, ref["dx"])
    h.close()


def test_c5_mixed_vjp_and_root_gradients():
    """The adjoint configuration in mixed precision: a split-bf16 handle runs
    the sigma part of the recomputation and its reverse in split-bf16 (the
    one-off part, dx and the gradient accumulation stay FP64).  Its dL must
    equal the FP64 handle's within 1e-4 relative (max |d dL| / max |dL|), and
    the eigenvalue gradients of the mixed roots (split-bf16 Davidson with FP64
    refinement, mixed backward) the FP64 ones within 1e-4 relative."""
    from adcgen import trial_vectors

    print("case C5 mixed vjp and root gradients", flush=True)
    P = config_problem("C5")
    h64 = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x)
    hbf = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, precision="split_bf16")
    Y = torch.from_numpy(trial_vectors(2, h64.dim, 81)).cuda()
    Sb = torch.from_numpy(trial_vectors(2, h64.dim, 82)).cuda()
    dL64, dx64 = h64.sigma_backward(Sb, Y)
    dLbf, dxbf = hbf.sigma_backward(Sb, Y)
    err = ((dLbf - dL64).abs().max() / dL64.abs().max()).item()
    print(f"  vjp dL mixed vs fp64 {err:.2e}, dx {dxbf:.12e} vs {dx64:.12e}", flush=True)
    assert 1e-12 < err <= 1e-4
    assert abs(dxbf - dx64) <= 1e-10 * max(1.0, abs(dx64))
    h64.close()
    hbf.close()
    grads = {}
    for prec in ("fp64", "split_bf16"):
        # the gradient y^H dM y is first order in the eigenvector error
        # (~|r|/gap), so both solves end with an FP64 residual of 1e-7
        spec = dict(kind=P.kind, o=P.o, v=P.v, eps=P.eps, n_roots=P.n_roots, precision=prec, conv_tol=1e-7)
        L = torch.from_numpy(P.L).cuda().requires_grad_(True)
        x = torch.tensor(P.x, dtype=torch.float64, device="cuda", requires_grad=True)
        w = ADCRoots.apply(L, x, spec)
        grads[prec] = [torch.autograd.grad(w[r], (L, x), retain_graph=True) for r in range(P.n_roots)]
    for r in range(P.n_roots):
        g64, x64 = grads["fp64"][r]
        gbf, xbf = grads["split_bf16"][r]
        e = ((gbf - g64).abs().max() / g64.abs().max()).item()
        ex = abs(xbf.item() - x64.item()) / max(1.0, abs(x64.item()))
        print(f"  root {r}: dw/dL mixed vs fp64 {e:.2e}, dw/dx {ex:.2e}", flush=True)
        assert e <= 1e-4 and ex <= 1e-4, (r, e, ex)


@pytest.mark.parametrize("kind,precision", [("EE", "fp64"), ("EA", "fp64"), ("IP", "fp64"), ("EE", "split_bf16")])
def test_repeated_backward_reuses_the_recorded_setup(kind, precision):
    """The first adc_sigma_backward call records the one-off part (integrals,
    amplitudes, intermediates) and keeps it; later calls on the same handle
    record only the sigma build on top.  Each of three calls with different
    (Sbar, Y), and of different k, equals the single call of a fresh handle
    (deterministic tile choices), and the FP64 ones equal the oracle."""
    P = make_problem(kind, 4, 9, 30, seed=61, n_roots=2, x=0.6)
    print(f"case repeated backward {kind} {precision}", flush=True)
    kw = dict(x=P.x, precision=precision, deterministic=True)
    h = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, **kw)
    rng = np.random.default_rng(62)
    import time
    for call, k in enumerate((2, 3, 1)):
        Y, Sb = _rand(rng, k, h.dim), _rand(rng, k, h.dim)
        Yd, Sd = torch.from_numpy(Y).cuda(), torch.from_numpy(Sb).cuda()
        t0 = time.perf_counter()
        dL, dx = h.sigma_backward(Sd, Yd)
        t1 = time.perf_counter()
        f = adc.Handle(P.kind, P.o, P.v, P.eps, P.L, P.n_roots, **kw)
        dL1, dx1 = f.sigma_backward(Sd, Yd)
        f.close()
        print(f"  call {call}: {1e3 * (t1 - t0):.1f} ms on the kept setup", flush=True)
        dL, dL1 = dL.cpu().numpy(), dL1.cpu().numpy()
        assert np.abs(dL - dL1).max() <= 1e-14 * np.abs(dL1).max(), call
        assert abs(dx - dx1) <= 1e-14 * max(1.0, abs(dx1)), call
        if precision == "fp64":
            ref, rdx = vjp(P.kind, P.eps, P.L, P.o, P.x, Y, Sb)
            assert np.abs(dL - ref).max() <= 1e-11 * np.abs(ref).max(), call
            assert abs(dx - rdx) <= 1e-11 * max(1.0, abs(rdx)), call
    h.close()
