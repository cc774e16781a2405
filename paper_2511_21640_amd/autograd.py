"""torch.autograd bindings of the sigma build and of the Davidson roots.

Both run every step on the device library (adc_init, adc_sigma,
adc_davidson, adc_sigma_backward); torch supplies device memory, streams and
the autograd graph.  Gradients follow torch's complex convention
(G = df/dRe + i df/dIm for a real objective f), and the gradient with respect
to L is projected onto Hermitian L^Q, (G + G^H)/2 per Q, because only
Hermitian perturbations of the Cholesky vectors keep the secular matrix
Hermitian (Section 2.1, eq. 10; eq. 42).

    ADCSigma.apply(L, x, Y, spec)  -> S = M(L, x) Y
    ADCRoots.apply(L, x, spec)     -> omega, the spec["n_roots"] lowest roots

``spec`` is a dict with keys kind, o, v, eps (float64 [o+v]) and optional
n_roots, precision, conv_tol, max_iter.  The eigenvalue gradient uses the
Hellmann-Feynman form d omega_r = y_r^H (dM) y_r with the converged Ritz
vectors y_r; it is undefined for degenerate roots.
"""
import torch

from . import Handle


def _handle(L, x, spec, n_roots=1):
    return Handle(spec["kind"], spec["o"], spec["v"], spec["eps"], L.detach().contiguous(),
                  spec.get("n_roots", n_roots), x=float(x), precision=spec.get("precision", "fp64"),
                  conv_tol=spec.get("conv_tol", 1e-9), max_iter=spec.get("max_iter", 200))


class ADCSigma(torch.autograd.Function):
    """S = M(L, x) Y for packed complex128 cuda vectors Y [k][dim]."""

    @staticmethod
    def forward(ctx, L, x, Y, spec):
        h = _handle(L, x, spec)
        Yc = Y.detach().contiguous()
        S = h.sigma(Yc)
        ctx.h = h
        ctx.save_for_backward(Yc)
        return S

    @staticmethod
    def backward(ctx, gS):
        (Y,) = ctx.saved_tensors
        h = ctx.h
        gS = gS.contiguous()
        dL = dx = dY = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            dL_, dx_ = h.sigma_backward(gS, Y, want_dL=ctx.needs_input_grad[0], want_dx=ctx.needs_input_grad[1])
            dL = dL_
            if dx_ is not None:
                dx = torch.tensor(dx_, dtype=torch.float64, device=Y.device)
        if ctx.needs_input_grad[2]:
            # M is Hermitian: G_Y = M^H G_S = M G_S
            dY = h.sigma(gS)
        return dL, dx, dY, None


class ADCRoots(torch.autograd.Function):
    """The n_roots lowest eigenvalues of M(L, x) (float64 [n_roots])."""

    @staticmethod
    def forward(ctx, L, x, spec):
        h = _handle(L, x, spec)
        r = h.davidson(want_vectors=True)
        if not r["converged"].all():
            raise RuntimeError(f"Davidson did not converge: residuals {r['resnorm']}")
        ctx.h = h
        ctx.save_for_backward(r["vectors"])
        return torch.as_tensor(r["omega"], dtype=torch.float64, device=L.device)

    @staticmethod
    def backward(ctx, gw):
        (Y,) = ctx.saved_tensors
        Sbar = (gw.to(torch.complex128)[:, None] * Y).contiguous()
        dL, dx_ = ctx.h.sigma_backward(Sbar, Y, want_dL=ctx.needs_input_grad[0], want_dx=ctx.needs_input_grad[1])
        dx = torch.tensor(dx_, dtype=torch.float64, device=Y.device) if dx_ is not None else None
        return dL, dx, None
