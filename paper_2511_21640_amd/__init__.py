"""Python binding of libadc (C ABI in include/adc.h).

Argument marshalling only: every step of the sigma build and of the Davidson
solver runs in the library's HIP kernels.  torch supplies device memory and
the stream.  Importing this package does not build anything; ``build()``
compiles the library for gfx950.  Using a handle without the library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadc.so")

KINDS = {"EE": 0, "IP": 1, "EA": 2}
PREC = {"fp64": 0, "fp32": 1, "split_bf16": 2}

ADC_OK = 0
ADC_NOT_CONVERGED = 1
ERRORS = {-1: "INVALID_ARG", -2: "NONFINITE_INPUT", -3: "NOT_HERMITIAN", -4: "OUT_OF_MEMORY",
          -5: "HIP_ERROR", -6: "UNSUPPORTED", -7: "SCRATCH"}

# Every symbol include/adc.h declares.
EXPORTS = ["adc_init", "adc_dims", "adc_sigma", "adc_sigma_term", "adc_sigma_noalloc", "adc_davidson",
           "adc_sigma_backward", "adc_properties", "adc_fns", "adc_cholesky", "adc_cholesky_mo", "adc_init_ms",
           "adc_free", "adc_strerror", "adc_last_error"]
TERMS = {"all": 0, "ladder": 1}


class AdcProblem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_occ", ctypes.c_int), ("n_vir", ctypes.c_int),
                ("n_chol", ctypes.c_int), ("n_roots", ctypes.c_int),
                ("eps", ctypes.POINTER(ctypes.c_double)), ("L", ctypes.c_void_p),
                ("L_on_device", ctypes.c_int), ("x", ctypes.c_double)]


class AdcOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("conv_tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("max_subspace", ctypes.c_int), ("refine_fp64", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("mem_budget", ctypes.c_size_t), ("verbose", ctypes.c_int), ("n_streams", ctypes.c_int),
                ("graphs", ctypes.c_int), ("autotune", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("deterministic", ctypes.c_int), ("root_follow", ctypes.c_int), ("precond", ctypes.c_int)]


GRAPHS = {False: 0, True: 1, "uncaptured": 2}


PRECOND = {"singles": 0, "diagonal": 1}


def _options(precision, conv_tol, max_iter, max_subspace, refine_fp64, stream, mem_budget, verbose, n_streams,
             graphs, autotune, tune_cache, deterministic, root_follow=False, precond="singles"):
    """graphs: False (host-driven iteration), True (captured sigma of small
    instances and the device iteration from captured graphs) or 'uncaptured'
    (the device iteration launched kernel by kernel).  precond: 'singles'
    (exact singles block, diagonal doubles) or 'diagonal'."""
    return AdcOptions(PREC[precision], conv_tol, max_iter, max_subspace, 1 if refine_fp64 else -1,
                      ctypes.c_void_p(stream), mem_budget, int(verbose), int(n_streams), GRAPHS[graphs],
                      1 if autotune else 0, tune_cache.encode() if tune_cache else None, 1 if deterministic else 0,
                      1 if root_follow else 0, PRECOND[precond])


class AdcError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        detail = ""
        if _lib is not None:
            d = _lib.adc_last_error()
            detail = f" ({d.decode(errors='replace')})" if d else ""
        super().__init__(f"{what}: {ERRORS.get(code, code)}{detail}")


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libadc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libadc.so not built ({path}); run paper_2511_21640_amd.build.build()")
    lib = ctypes.CDLL(path)
    lib.adc_init.argtypes = [ctypes.POINTER(AdcProblem), ctypes.c_int, ctypes.POINTER(AdcOptions),
                             ctypes.POINTER(ctypes.c_void_p)]
    lib.adc_init.restype = ctypes.c_int
    lib.adc_dims.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                             ctypes.POINTER(ctypes.c_longlong)]
    lib.adc_sigma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_int]
    lib.adc_sigma_term.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_int]
    lib.adc_sigma_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_int]
    lib.adc_davidson.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.adc_sigma_backward.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.adc_properties.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.adc_fns.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                            ctypes.c_void_p, ctypes.c_void_p]
    lib.adc_cholesky.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]
    lib.adc_cholesky_mo.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p]
    lib.adc_init_ms.argtypes = [ctypes.c_void_p]
    lib.adc_init_ms.restype = ctypes.c_double
    lib.adc_free.argtypes = [ctypes.c_void_p]
    lib.adc_free.restype = None
    lib.adc_strerror.argtypes = [ctypes.c_int]
    lib.adc_strerror.restype = ctypes.c_char_p
    lib.adc_last_error.argtypes = []
    lib.adc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def build():
    from .build import build as _b
    return _b()


class Handle:
    """One problem instance on the current HIP device.

    eps: float64 [o+v]; L: complex128 [N][n][n] (numpy host array, or a torch
    cuda tensor which is borrowed).  precision: 'fp64' | 'fp32' | 'split_bf16'.
    """

    def __init__(self, kind, o, v, eps, L, n_roots, x=1.0, precision="fp64", conv_tol=1e-7, max_iter=200,
                 max_subspace=0, stream=None, mem_budget=0, verbose=False, graphs=False, autotune=False,
                 refine_fp64=True, tune_cache=None, deterministic=False, root_follow=False, precond="singles"):
        import torch
        self._lib = load()
        self.kind, self.o, self.v = kind, int(o), int(v)
        self.n_roots = int(n_roots)
        self._eps = np.ascontiguousarray(eps, dtype=np.float64)
        on_dev = hasattr(L, "is_cuda") and L.is_cuda
        if on_dev:
            assert L.dtype == torch.complex128 and L.is_contiguous()
            self._L = L
            Lptr = L.data_ptr()
        else:
            self._L = np.ascontiguousarray(L, dtype=np.complex128)
            Lptr = self._L.ctypes.data
        n_chol = int(self._L.shape[0])
        prob = AdcProblem(KINDS[kind], self.o, self.v, n_chol, self.n_roots,
                          self._eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), Lptr, 1 if on_dev else 0,
                          float(x))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        opts = _options(precision, conv_tol, max_iter, max_subspace, refine_fp64, stream, mem_budget, verbose, 0,
                        graphs, autotune, tune_cache, deterministic, root_follow, precond)
        h = ctypes.c_void_p()
        rc = self._lib.adc_init(ctypes.byref(prob), 1, ctypes.byref(opts), ctypes.byref(h))
        if rc != ADC_OK:
            raise AdcError(rc, "adc_init")
        self._h = h
        n1, n2 = ctypes.c_longlong(), ctypes.c_longlong()
        self._lib.adc_dims(h, 0, ctypes.byref(n1), ctypes.byref(n2))
        self.n1, self.n2 = n1.value, n2.value
        self.dim = self.n1 + self.n2

    @property
    def init_ms(self):
        return self._lib.adc_init_ms(self._h)

    def sigma(self, Y, S=None, precision=None):
        """S = M(x) Y for a torch complex128 cuda tensor Y [k][dim]."""
        import torch
        assert Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.shape[-1] == self.dim
        Y2 = Y.reshape(-1, self.dim)
        if S is None:
            S = torch.empty_like(Y2)
        p = -1 if precision is None else PREC[precision]
        rc = self._lib.adc_sigma(self._h, 0, ctypes.c_void_p(Y2.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                 Y2.shape[0], p)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_sigma")
        return S.reshape(Y.shape)

    def sigma_noalloc(self, Y, S=None, precision=None):
        """adc_sigma_noalloc: the same build with every temporary in the
        library's fixed device scratch (no allocation inside the call)."""
        import torch
        assert Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.shape[-1] == self.dim
        Y2 = Y.reshape(-1, self.dim)
        if S is None:
            S = torch.empty_like(Y2)
        p = -1 if precision is None else PREC[precision]
        rc = self._lib.adc_sigma_noalloc(self._h, 0, ctypes.c_void_p(Y2.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                         Y2.shape[0], p)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_sigma_noalloc")
        return S.reshape(Y.shape)

    def sigma_term(self, term, Y, S=None, precision=None):
        """One term of the sigma build (see adc_sigma_term)."""
        import torch
        assert Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.shape[-1] == self.dim
        Y2 = Y.reshape(-1, self.dim)
        if S is None:
            S = torch.empty_like(Y2)
        p = -1 if precision is None else PREC[precision]
        rc = self._lib.adc_sigma_term(self._h, 0, TERMS[term], ctypes.c_void_p(Y2.data_ptr()),
                                      ctypes.c_void_p(S.data_ptr()), Y2.shape[0], p)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_sigma_term")
        return S.reshape(Y.shape)

    def sigma_backward(self, Sbar, Y, want_dL=True, want_dx=True):
        """Vector-Jacobian product of the sigma build (see adc_sigma_backward):
        gradients of f = Re sum_z Sbar_z^H M(L, x) Y_z.  Returns (dL, dx): dL a
        complex128 cuda tensor shaped like L, Hermitian-projected per Q (or
        None), dx a float (or None)."""
        import torch
        for T in (Sbar, Y):
            assert T.is_cuda and T.dtype == torch.complex128 and T.is_contiguous() and T.shape[-1] == self.dim
        Y2 = Y.reshape(-1, self.dim)
        S2 = Sbar.reshape(-1, self.dim)
        assert S2.shape == Y2.shape
        n = self.o + self.v
        n_chol = int(self._L.shape[0])
        dL = torch.empty((n_chol, n, n), dtype=torch.complex128, device=Y.device) if want_dL else None
        dx = ctypes.c_double(0.0)
        torch.cuda.current_stream().synchronize()
        rc = self._lib.adc_sigma_backward(self._h, 0, ctypes.c_void_p(S2.data_ptr()), ctypes.c_void_p(Y2.data_ptr()),
                                          Y2.shape[0], ctypes.c_void_p(dL.data_ptr()) if dL is not None else None,
                                          ctypes.byref(dx) if want_dx else None)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_sigma_backward")
        return dL, (dx.value if want_dx else None)

    def davidson(self, guess=None, want_vectors=True):
        """Lowest n_roots eigenpairs.  guess: optional complex128 cuda tensor
        [n_roots][dim] of start vectors (contiguous)."""
        import torch
        k = self.n_roots
        if guess is not None:
            if not (hasattr(guess, "is_cuda") and guess.is_cuda and guess.dtype == torch.complex128
                    and guess.is_contiguous() and tuple(guess.shape) == (k, self.dim)):
                raise ValueError(f"guess must be a contiguous complex128 cuda tensor of shape ({k}, {self.dim})")
        omega = np.zeros(k)
        res = np.zeros(k)
        iters = (ctypes.c_int * 1)()
        conv = (ctypes.c_int * k)()
        vecs = torch.empty((k, self.dim), dtype=torch.complex128, device="cuda") if want_vectors else None
        g_arr = (ctypes.c_void_p * 1)(guess.data_ptr()) if guess is not None else None
        v_arr = (ctypes.c_void_p * 1)(vecs.data_ptr()) if vecs is not None else None
        rc = self._lib.adc_davidson(self._h, g_arr, omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v_arr,
                                    res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), iters, conv)
        if rc not in (ADC_OK, ADC_NOT_CONVERGED):
            raise AdcError(rc, "adc_davidson")
        return dict(omega=omega, resnorm=res, iters=iters[0], converged=np.array(conv[:], dtype=bool),
                    vectors=vecs, status=rc)

    def properties(self, Y, d=None):
        """adc_properties for EE vectors Y (complex128 cuda [k][dim]): returns
        dict(rho, tdm) as complex128 cuda [k][n][n], and with a one-particle
        operator d (complex128 cuda [n][n]) also D (state expectation values)
        and T (transition moments) as complex numpy arrays [k]."""
        import torch
        assert Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.shape[-1] == self.dim
        Y2 = Y.reshape(-1, self.dim)
        k, n = Y2.shape[0], self.o + self.v
        rho = torch.empty((k, n, n), dtype=torch.complex128, device="cuda")
        tdm = torch.empty_like(rho)
        dk = np.zeros(2 * k)
        tk = np.zeros(2 * k)
        if d is not None:
            assert d.is_cuda and d.dtype == torch.complex128 and d.is_contiguous() and tuple(d.shape) == (n, n)
        pd = ctypes.c_void_p(d.data_ptr()) if d is not None else None
        rc = self._lib.adc_properties(self._h, 0, ctypes.c_void_p(Y2.data_ptr()), k, ctypes.c_void_p(rho.data_ptr()),
                                      ctypes.c_void_p(tdm.data_ptr()), pd,
                                      dk.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if d is not None else None,
                                      tk.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if d is not None else None)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_properties")
        out = dict(rho=rho, tdm=tdm)
        if d is not None:
            out["D"] = dk[0::2] + 1j * dk[1::2]
            out["T"] = tk[0::2] + 1j * tk[1::2]
        return out

    def fns(self, eta_crit, X=None, want_B=False):
        """adc_fns: frozen (or, with X, state-specific) natural spinors.
        Returns dict(n_vir, eps (numpy [o + v']), L (complex128 cuda
        [N][o+v'][o+v']), eta (numpy [v], descending), B (cuda [v][v'] or
        None), X (X in the truncated basis, cuda [dim'], or None))."""
        import torch
        o, v = self.o, self.v
        n = o + v
        n_chol = int(self._L.shape[0])
        Lbuf = torch.empty(n_chol * n * n, dtype=torch.complex128, device="cuda")
        eps = np.zeros(n)
        eta = np.zeros(v)
        nv = ctypes.c_int(0)
        Bbuf = torch.empty(v * v, dtype=torch.complex128, device="cuda") if want_B else None
        Xin = Xbuf = None
        if X is not None:
            assert X.is_cuda and X.dtype == torch.complex128 and X.is_contiguous() and X.numel() == self.dim
            Xin = X
            Xbuf = torch.empty(self.dim, dtype=torch.complex128, device="cuda")
        rc = self._lib.adc_fns(self._h, 0, ctypes.c_void_p(Xin.data_ptr()) if Xin is not None else None,
                               float(eta_crit), ctypes.byref(nv), eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_void_p(Lbuf.data_ptr()), eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_void_p(Bbuf.data_ptr()) if Bbuf is not None else None,
                               ctypes.c_void_p(Xbuf.data_ptr()) if Xbuf is not None else None)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_fns")
        v2 = nv.value
        n2 = o + v2
        Po, Pv2 = o * (o - 1) // 2, v2 * (v2 - 1) // 2
        dim2 = {"EE": o * v2 + Po * Pv2, "IP": o + Po * v2, "EA": v2 + o * Pv2}[self.kind]
        return dict(n_vir=v2, eps=eps[:n2].copy(), L=Lbuf[: n_chol * n2 * n2].view(n_chol, n2, n2), eta=eta,
                    B=Bbuf[: v * v2].view(v, v2) if Bbuf is not None else None,
                    X=Xbuf[:dim2] if Xbuf is not None else None)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.adc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cholesky(V, tau, max_vec=None):
    """adc_cholesky: one-step pivoted Cholesky of a float64 cuda tensor V
    [m][m] (symmetric positive semidefinite).  Returns (L [n_vec][m] cuda
    tensor, pivots numpy int array)."""
    import torch
    lib = load()
    assert V.is_cuda and V.dtype == torch.float64 and V.is_contiguous() and V.dim() == 2 and V.shape[0] == V.shape[1]
    m = int(V.shape[0])
    max_vec = m if max_vec is None else int(max_vec)
    L = torch.empty((max(max_vec, 1), m), dtype=torch.float64, device=V.device)
    piv = (ctypes.c_int * max(max_vec, 1))()
    n = ctypes.c_int(0)
    rc = lib.adc_cholesky(ctypes.c_void_p(V.data_ptr()), m, float(tau), max_vec, ctypes.c_void_p(L.data_ptr()), piv,
                          ctypes.byref(n), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != ADC_OK:
        raise AdcError(rc, "adc_cholesky")
    return L[: n.value], np.array(piv[: n.value], dtype=np.int64)


def cholesky_mo(Lp, n_ao, C):
    """adc_cholesky_mo: vectors over the pairs mu <= nu (float64 cuda [n_vec]
    [n_ao (n_ao+1)/2]) to the molecular basis with complex128 cuda C
    [n_ao][n_mo]; returns complex128 cuda [n_vec][n_mo][n_mo]."""
    import torch
    lib = load()
    assert Lp.is_cuda and Lp.dtype == torch.float64 and Lp.is_contiguous()
    assert C.is_cuda and C.dtype == torch.complex128 and C.is_contiguous() and C.shape[0] == n_ao
    assert Lp.shape[1] == n_ao * (n_ao + 1) // 2
    n_vec, n_mo = int(Lp.shape[0]), int(C.shape[1])
    out = torch.empty((n_vec, n_mo, n_mo), dtype=torch.complex128, device=Lp.device)
    rc = lib.adc_cholesky_mo(ctypes.c_void_p(Lp.data_ptr()), n_vec, n_ao, ctypes.c_void_p(C.data_ptr()), n_mo,
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != ADC_OK:
        raise AdcError(rc, "adc_cholesky_mo")
    return out


class Batch:
    """Several independent instances in one handle (adc_init with
    n_problems > 1).  problems: list of dicts with keys kind, o, v, eps, L
    (numpy), n_roots and optionally x.  The instances are spread over
    n_streams lanes (longest first) and solved concurrently."""

    def __init__(self, problems, precision="fp64", conv_tol=1e-7, max_iter=200, max_subspace=0, stream=None,
                 mem_budget=0, verbose=False, n_streams=0, graphs=False, autotune=False, refine_fp64=True,
                 tune_cache=None, deterministic=False, root_follow=False, precond="singles"):
        import torch
        self._lib = load()
        self._keep = []
        arr = (AdcProblem * len(problems))()
        self._dev = []  # borrowed device L tensors, kept alive with the handle
        for i, p in enumerate(problems):
            eps = np.ascontiguousarray(p["eps"], dtype=np.float64)
            L = p["L"]
            if hasattr(L, "is_cuda") and L.is_cuda:
                assert L.dtype == torch.complex128 and L.is_contiguous()
                self._dev.append(L)
                Lptr, on_dev = L.data_ptr(), 1
            else:
                L = np.ascontiguousarray(L, dtype=np.complex128)
                Lptr, on_dev = L.ctypes.data, 0
            self._keep += [eps, L]
            arr[i] = AdcProblem(KINDS[p["kind"]], int(p["o"]), int(p["v"]), int(L.shape[0]), int(p["n_roots"]),
                                eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), Lptr, on_dev,
                                float(p.get("x", 1.0)))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        opts = _options(precision, conv_tol, max_iter, max_subspace, refine_fp64, stream, mem_budget, verbose,
                        n_streams, graphs, autotune, tune_cache, deterministic, root_follow, precond)
        h = ctypes.c_void_p()
        rc = self._lib.adc_init(arr, len(problems), ctypes.byref(opts), ctypes.byref(h))
        self._keep = []  # host copies are no longer needed
        if rc != ADC_OK:
            raise AdcError(rc, "adc_init")
        self._h = h
        self.n_roots = [int(p["n_roots"]) for p in problems]
        self.dims = []
        for i in range(len(problems)):
            n1, n2 = ctypes.c_longlong(), ctypes.c_longlong()
            self._lib.adc_dims(h, i, ctypes.byref(n1), ctypes.byref(n2))
            self.dims.append(n1.value + n2.value)

    @property
    def init_ms(self):
        return self._lib.adc_init_ms(self._h)

    def sigma(self, inst, Y, precision=None):
        import torch
        assert Y.is_cuda and Y.dtype == torch.complex128 and Y.is_contiguous() and Y.shape[-1] == self.dims[inst]
        Y2 = Y.reshape(-1, self.dims[inst])
        S = torch.empty_like(Y2)
        p = -1 if precision is None else PREC[precision]
        rc = self._lib.adc_sigma(self._h, inst, ctypes.c_void_p(Y2.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                 Y2.shape[0], p)
        if rc != ADC_OK:
            raise AdcError(rc, "adc_sigma")
        return S.reshape(Y.shape)

    def davidson(self, want_vectors=False, guesses=None):
        """Solve every instance.  guesses: None, or a list with, per
        instance, None or a contiguous complex128 cuda tensor [n_roots][dim]."""
        import torch
        n = len(self.dims)
        g_arr = None
        if guesses is not None:
            assert len(guesses) == n
            for g, k, d in zip(guesses, self.n_roots, self.dims):
                if g is not None and not (g.is_cuda and g.dtype == torch.complex128 and g.is_contiguous()
                                          and tuple(g.shape) == (k, d)):
                    raise ValueError(f"guess must be a contiguous complex128 cuda tensor of shape ({k}, {d})")
            g_arr = (ctypes.c_void_p * n)(*[g.data_ptr() if g is not None else None for g in guesses])
        tot = sum(self.n_roots)
        omega, res = np.zeros(tot), np.zeros(tot)
        iters = (ctypes.c_int * n)()
        conv = (ctypes.c_int * tot)()
        vecs = [torch.empty((k, d), dtype=torch.complex128, device="cuda") for k, d in zip(self.n_roots, self.dims)] \
            if want_vectors else None
        v_arr = (ctypes.c_void_p * n)(*[v.data_ptr() for v in vecs]) if vecs is not None else None
        rc = self._lib.adc_davidson(self._h, g_arr, omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v_arr,
                                    res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), iters, conv)
        if rc not in (ADC_OK, ADC_NOT_CONVERGED):
            raise AdcError(rc, "adc_davidson")
        out, o = [], 0
        for i, k in enumerate(self.n_roots):
            out.append(dict(omega=omega[o:o + k], resnorm=res[o:o + k], iters=iters[i],
                            converged=np.array(conv[o:o + k], dtype=bool),
                            vectors=vecs[i] if vecs is not None else None))
            o += k
        return out, rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.adc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

