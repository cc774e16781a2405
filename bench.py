#!/usr/bin/env python3
"""Sigma-build throughput on one MI355X.

Workload: EE-ADC(2)+x(3), x = 0.5, o = 20, v = 120 spinors, N_chol = 900,
8 trial vectors (the plain-vs-mixed configuration), synthetic seeded inputs
(``adcgen``).  One step = one sigma build S = M(x) Y for all 8 vectors, inputs
resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision split_bf16|fp32|fp64]
                  [--no-cpu] [--no-eig]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sigma builds/s + MFMA TFLOP/s, mixed vs FP64 GPU at ≤1e-6 Eh eigval error"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0}
# HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by a plain 1 GiB copy) of one
# split-bf16 ladder term at this workload, from the counter runs summarised in
# profiles/ladder_c2_split_bf16.md; None for the other precisions (not measured)
LADDER_TRAFFIC_BYTES = {"split_bf16": 6.372e9 + 1.323e9}
DTYPE = {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16x3"}
# MFMA counters of one split-bf16 ladder term at this workload, from the
# counter run summarised in profiles/ladder_c2_split_bf16.md: executed MFMA
# flop (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512) / 2.5 PFLOP/s / kernel time, and
# SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCC x 1024 SIMDs); None for
# the precisions not measured
MFMA_COUNTERS = {"split_bf16": {"exec_frac": 0.42, "busy_frac": 0.49}}


def core_terms(o, v, N, k):
    """Algorithmic work of one EE sigma build in complex MACs, per term, as
    the cost model counts it: every unique <ab||cd> (a<b, c<d) formed once
    from two Cholesky sums (assembly 2 N Pv^2, whatever symmetry the build
    exploits), the pp-ladder k Po Pv^2, the ring k (ov)^3, the hh-ladder
    k Po^2 Pv and the first-order coupling N o v^3 + k o^2 v^3 + k o^3 v^2
    (three-external class assembled, contracted, plus the three-internal
    terms).  8 flop per complex MAC."""
    Po, Pv = o * (o - 1) // 2, v * (v - 1) // 2
    return {"assembly": 2 * N * Pv * Pv, "pp_ladder": k * Po * Pv * Pv, "ring": k * (o * v) ** 3,
            "hh_ladder": k * Po * Po * Pv, "coupling_a8": N * o * v ** 3 + k * o * o * v ** 3 + k * o ** 3 * v * v}


def core_flops(o, v, N, k):
    """(core flop of one build, flop of the ladder term = assembly + pp-ladder)."""
    t = core_terms(o, v, N, k)
    return 8.0 * sum(t.values()), 8.0 * (t["assembly"] + t["pp_ladder"])


def cpu_info():
    """Host description for the CPU baseline: model, logical CPUs, the
    threads this process may use, and numpy's BLAS."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = "", None
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = max(d.get("num_threads", 1) for d in info)
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "blas": blas, "blas_threads": threads}


def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# The three largest split-bf16 products of the C2 build as complex shapes
# (M, N, K): a complex MAC in split-bf16 is 12 real bf16 products, i.e. the
# same flop as one real bf16 GEMM of M x 2N x 6K
VENDOR_SHAPES = [("ring product", 19200, 2400, 2400),
                 ("ladder contraction", 1520, 7140, 7168),
                 ("ladder assembly, largest block", 1920, 14280, 928)]


def vendor_gemm(steps, warmup):
    """Times torch's bf16 matmul (hipBLASLt) on the real GEMMs with the flop of
    the build's largest split-bf16 products, for comparison with this
    library's kernels in the same run (a measurement aid; no part of the
    library uses it)."""
    import torch
    out = []
    stream = torch.cuda.current_stream()
    for name, M, N, K in VENDOR_SHAPES:
        A = torch.randn(M, 6 * K, device="cuda", dtype=torch.bfloat16)
        Bt = torch.randn(2 * N, 6 * K, device="cuda", dtype=torch.bfloat16)
        C = torch.empty(M, 2 * N, device="cuda", dtype=torch.bfloat16)
        ms = time_calls(lambda: torch.matmul(A, Bt.t(), out=C), steps, warmup, stream)
        fl = 24.0 * M * N * K
        out.append({"product": name, "complex_MNK": [M, N, K], "real_bf16_MNK": [M, 2 * N, 6 * K],
                    "ms": ms, "tflops": fl / ms / 1e9})
        print(f"[bench] vendor bf16 GEMM for the {name} ({M}x{2 * N}x{6 * K}): {ms:.3f} ms, "
              f"{fl / ms / 1e9:.0f} TFLOP/s", file=sys.stderr, flush=True)
        del A, Bt, C
    torch.cuda.empty_cache()
    return out


def oracle_build(P, X):
    """The oracle's matrix-free FP64 sigma (every block and order, M11
    included) of the rows of X on the host: (S, seconds of the integral and
    amplitude setup, seconds of the sigma itself)."""
    from oracle.adc_terms import Ints, sigma
    t0 = time.perf_counter()
    ints = Ints(P.eps, P.L, P.o)
    for c in ("vvvv", "ovvv", "vovv", "ovov", "oovv", "vvoo", "ooov", "oooo"):
        ints.g(c)
    for a in ("t", "t2", "ts"):
        ints.amp(a)
    t1 = time.perf_counter()
    S = sigma(ints, P.kind, P.x, X)
    return S, t1 - t0, time.perf_counter() - t1


def certify(P, X, omega, spec, roots):
    """Per-root certificate of GPU Ritz vectors X (rows) with eigenvalues
    omega: theta = y^H M y and |r| = |M y - theta y| from the oracle's sigma of
    the normalised rows; the Hermitian M has an eigenvalue within |r|^2 / gap
    of theta, gap = distance from theta to the other eigenvalues (from spec,
    a solve for more roots; roots[j] = the index of row j's root in spec).
    Returns (per-root records, oracle timings)."""
    nrm = np.sqrt(np.einsum("ki,ki->k", X.conj(), X).real)
    Xn = X / nrm[:, None]
    S, t_setup, t_sigma = oracle_build(P, Xn)
    theta = np.einsum("ki,ki->k", Xn.conj(), S).real
    rn = np.linalg.norm(S - theta[:, None] * Xn, axis=1)
    out = []
    for j in range(len(omega)):
        gap = float(np.min(np.abs(np.delete(spec, roots[j]) - theta[j])))
        out.append({"omega_gpu": float(omega[j]), "theta_oracle": float(theta[j]), "resnorm_oracle": float(rn[j]),
                    "gap": gap, "abs_omega_minus_theta": float(abs(omega[j] - theta[j])),
                    "bound_Eh": float(abs(omega[j] - theta[j]) + rn[j] ** 2 / gap)})
    return out, t_setup, t_sigma


def c4_device_gb(kind, o, v, N, k):
    """Rough device memory of one instance of the batched workload, GB:
    (resident, transient).  Resident: L blocks, stored integral classes,
    amplitudes and intermediates, M11, the cached split-bf16 planes.
    Transient (while its lane solves it): Davidson subspace (6k vectors of V and S, three k-blocks), the sigma
    workspace of one pass (unpacked doubles, at most 16 GiB), the ladder
    batch (4 GiB) and the planes of all packed <ab||cd> rows where they take
    at most 16 GiB."""
    n = o + v
    Po, Pv = o * (o - 1) // 2, v * (v - 1) // 2
    n1 = {"EE": o * v, "IP": o, "EA": v}[kind]
    dim = {"EE": o * v + Po * Pv, "IP": o + Po * v, "EA": v + o * Pv}[kind]
    unp = {"EE": o * o * v * v, "IP": o * o * v, "EA": o * v * v}[kind]
    res = N * n * n + 6 * o * o * v * v + o ** 4 + 2 * o ** 3 * v + 2 * n1 * n1
    if kind != "IP":
        res += 2 * o * v ** 3
    if kind == "EE":
        res += o * v * v * (v + o) + o * o * v * (2 * o + v) + o * v ** 3 + o ** 3 * v
    elif kind == "EA":
        res += o * v ** 3
    else:
        res += o ** 3 * v
    # split-bf16 planes of the frozen trial-independent operands (at most
    # their own size in bytes)
    res += (res - N * n * n - 2 * n1 * n1)
    tr = (2 * 6 * k + 3 * k) * dim + min(k * 6 * unp, (16 << 30) // 16) + (4 << 30) // 16
    planes = 8 * Pv * (-(-Pv // 32) * 32)
    if kind != "IP" and planes <= (16 << 30):  # split-bf16 planes of all packed <ab||cd> rows
        tr += planes // 16
    return res * 16 / 1e9, tr * 16 / 1e9


def c4_certify(draw, res, vec_host, budget_s):
    """Rayleigh-quotient certificates of batched-solve roots from the oracle's
    FP64 sigma, cheapest instances first while the CPU time budget lasts.
    Per root: theta = y^H M y and |r| = |M y - theta y| for the normalised GPU
    Ritz vector y; an eigenvalue lies within |r| of theta (no gap needed) and
    within |r|^2 / gap, with the gap estimated from the instance's other GPU
    roots."""
    from adcgen import make_problem
    t_start = time.perf_counter()
    done, per = [], []
    for i in sorted(vec_host, key=lambda i: draw[i][2]):
        kind, o, v, N, k, seed = draw[i]
        est = 48.0 * v ** 5 / 6e10
        if time.perf_counter() - t_start + est > budget_s:
            continue
        P = make_problem(kind, o, v, N, seed, n_roots=k, x=0.5)
        X = vec_host[i]
        nrm = np.sqrt(np.einsum("ki,ki->k", X.conj(), X).real)
        S, _, _ = oracle_build(P, X / nrm[:, None])
        Xn = X / nrm[:, None]
        theta = np.einsum("ki,ki->k", Xn.conj(), S).real
        rn = np.linalg.norm(S - theta[:, None] * Xn, axis=1)
        om = np.asarray(res[i]["omega"])
        gap = np.array([np.min(np.abs(np.delete(om, j) - theta[j])) if k > 1 else np.inf for j in range(k)])
        dw = np.abs(om - theta)
        rec = {"instance": int(i), "kind": kind, "o": o, "v": v, "roots": k,
               "max_abs_omega_minus_theta": float(dw.max()), "max_resnorm_oracle": float(rn.max()),
               "max_bound_gap_free_Eh": float((dw + rn).max()),
               "max_bound_est_gap_Eh": float((dw + rn ** 2 / gap).max())}
        per.append(rec)
        done.append(i)
        print(f"[c4] certified instance {i} {kind} o={o} v={v} k={k}: max |w-theta| {rec['max_abs_omega_minus_theta']:.1e},"
              f" max |r| {rec['max_resnorm_oracle']:.1e}, bound (est. gap) {rec['max_bound_est_gap_Eh']:.1e}",
              file=sys.stderr, flush=True)
    kinds = [draw[i][0] for i in done]
    return {"instances": len(done), "EE": kinds.count("EE"), "IP": kinds.count("IP"), "EA": kinds.count("EA"),
            "cpu_s": time.perf_counter() - t_start, "budget_s": budget_s,
            "max_abs_omega_minus_theta": max((r["max_abs_omega_minus_theta"] for r in per), default=None),
            "max_bound_est_gap_Eh": max((r["max_bound_est_gap_Eh"] for r in per), default=None),
            "per_instance": per}


def run_c3(args):
    """IP and EA on the large configuration (o=60, v=400, N_chol=2400, 6 roots,
    x as configured): the split-bf16 solve (reduced-precision sweeps, then FP64
    to the tolerance) against the FP64 solve, per root, each on its own handle
    (one instance of this size at a time fits the device)."""
    import torch
    import paper_2511_21640_amd as adc
    from adcgen import config_problem

    out = {"metric": "eigenvalues, split-bf16 vs FP64 GPU solve", "data": "synthetic", "conv_tol": 3e-5,
           "iteration": "device (captured graphs)", "kinds": {}}
    for kind in args.c3_kinds.split(","):
        P = config_problem("C3-" + kind)
        rec = {"o": P.o, "v": P.v, "n_chol": P.L.shape[0], "roots": P.n_roots, "x": P.x}
        for prec in args.c3_precisions.split(","):
            t0 = time.perf_counter()
            h = adc.Handle(kind, P.o, P.v, P.eps, P.L, P.n_roots, x=P.x, precision=prec, conv_tol=3e-5, graphs=True,
                           verbose=args.verbose)
            t_init = time.perf_counter() - t0
            t0 = time.perf_counter()
            r = h.davidson(want_vectors=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            h.close()
            torch.cuda.empty_cache()
            rec[prec] = {"omega": r["omega"].tolist(), "iters": int(r["iters"]), "solve_s": t, "init_s": t_init,
                         "converged": bool(r["converged"].all()), "max_resnorm": float(r["resnorm"].max())}
            print(f"[c3] {kind} {prec}: init {t_init:.1f} s, solve {t:.1f} s, {r['iters']} iterations", file=sys.stderr,
                  flush=True)
        out["kinds"][kind] = rec
        if "split_bf16" not in rec or "fp64" not in rec:
            continue
        d = np.abs(np.array(rec["split_bf16"]["omega"]) - np.array(rec["fp64"]["omega"]))
        rec["per_root_diff_Eh"] = d.tolist()
        rec["max_abs_diff_Eh"] = float(d.max())
        print(f"[c3] {kind}: max |omega mixed - omega fp64| {d.max():.2e} Eh", file=sys.stderr, flush=True)
    print(json.dumps(out))


def run_c4(args):
    """Batched workload: uneven EE/IP/EA instances (the 64-instance draw),
    solved in waves whose estimated device memory fits the budget; each wave
    is one handle (lanes, captured sigma graphs, autotuned GEMMs)."""
    import torch
    import paper_2511_21640_amd as adc
    from adcgen import c4_draw, make_problem

    draw = c4_draw()[: args.c4]
    mem = [c4_device_gb(*d[:5]) for d in draw]
    order = sorted(range(len(draw)), key=lambda i: -(mem[i][0] + mem[i][1]))
    # waves: resident memory of every member plus the four largest transients
    waves, cur = [], []

    def need(ids):
        tr = sorted((mem[i][1] for i in ids), reverse=True)[:4]
        return sum(mem[i][0] for i in ids) + sum(tr)

    for i in order:
        if cur and need(cur + [i]) > args.c4_budget_gb:
            waves.append(cur)
            cur = []
        cur.append(i)
    if cur:
        waves.append(cur)
    flop_build = 0.0
    for kind, o, v, N, k, seed in draw:
        Po, Pv = o * (o - 1) // 2, v * (v - 1) // 2
        if kind == "EE":
            c = 2 * N * Pv * Pv + k * (Po * Pv * Pv + (o * v) ** 3 + o * o * v ** 3)
        elif kind == "IP":
            c = k * (o * (o * v) ** 2 + Po * Po * v) + N * o * o * v * v
        else:
            c = 2 * N * Pv * Pv + k * (o * Pv * Pv + v * (o * v) ** 2)
        flop_build += 8.0 * c
    res = {}
    vec_host = {}
    t_init = t_build = t_solve = t_tune = 0.0
    for w, idx in enumerate(waves):
        print(f"[c4] wave {w + 1}/{len(waves)}: {len(idx)} instances, drawing inputs", file=sys.stderr, flush=True)
        probs = []
        for i in idx:
            kind, o, v, N, k, seed = draw[i]
            P = make_problem(kind, o, v, N, seed, n_roots=k, x=0.5)
            probs.append(dict(kind=kind, o=o, v=v, eps=P.eps, L=P.L, n_roots=k, x=0.5))
        t0 = time.perf_counter()
        B = adc.Batch(probs, precision=args.precision, conv_tol=3e-5, n_streams=4, graphs=True, autotune=True,
                      verbose=args.verbose)
        torch.cuda.synchronize()
        t_init += time.perf_counter() - t0
        del probs
        print(f"[c4] wave {w + 1}: init {B.init_ms / 1e3:.1f} s", file=sys.stderr, flush=True)
        rng = np.random.default_rng(7)
        Ys = [torch.from_numpy(rng.standard_normal((kk, d)) + 0j).cuda() for kk, d in zip(B.n_roots, B.dims)]
        for j in range(len(idx)):  # warm-up (tuning, planes)
            B.sigma(j, Ys[j])
        torch.cuda.synchronize()
        # tuning pass: the GEMM shape classes of the solve (new-direction row
        # counts in powers of two up to k, split-bf16 and the FP64
        # refinement) are timed here once instead of inside the solve; with a
        # tune_cache file from an earlier run this pass finds them all cached
        t0 = time.perf_counter()
        for j in range(len(idx)):
            kk = B.n_roots[j]
            for r in sorted({kk} | {1 << e for e in range(kk.bit_length()) if (1 << e) < kk}):
                Yr = Ys[j][:r].contiguous()
                B.sigma(j, Yr)
                B.sigma(j, Yr, precision="fp64")
        torch.cuda.synchronize()
        t_tune += time.perf_counter() - t0
        t0 = time.perf_counter()
        for j in range(len(idx)):
            B.sigma(j, Ys[j])
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        del Ys
        t0 = time.perf_counter()
        out, rc = B.davidson(want_vectors=args.c4_certify_s > 0)
        t_solve += time.perf_counter() - t0
        for j, i in enumerate(idx):
            res[i] = out[j]
            # Ritz vectors of instances the oracle can certify within the
            # budget are kept on the host (the oracle's setup builds all of
            # <ab||cd>, about 48 v^5 flop)
            if args.c4_certify_s > 0 and 48.0 * draw[i][2] ** 5 / 6e10 < min(args.c4_certify_s, 90.0):
                vec_host[i] = out[j]["vectors"].cpu().numpy()
            out[j]["vectors"] = None
        print(f"[c4] wave {w + 1}: solve {time.perf_counter() - t0:.1f} s, rc {rc}", file=sys.stderr, flush=True)
        B.close()
        torch.cuda.empty_cache()
    cert = c4_certify(draw, res, vec_host, args.c4_certify_s) if args.c4_certify_s > 0 else None
    iters = [res[i]["iters"] for i in range(len(draw))]
    conv = all(bool(res[i]["converged"].all()) for i in range(len(draw)))
    kinds = [d[0] for d in draw]
    out = {"metric": "batched solve of uneven EE/IP/EA instances", "workload": f"{len(draw)} instances of the "
           f"64-instance draw (EE {kinds.count('EE')}, IP {kinds.count('IP')}, EA {kinds.count('EA')}), x=0.5",
           "precision": args.precision, "waves": len(waves), "roots": int(sum(d[4] for d in draw)),
           "init_s": t_init, "tune_s": t_tune, "all_instance_build_s": t_build, "core_flop_all_instance_build": flop_build,
           "all_instance_build_tflops": flop_build / t_build / 1e12, "solve_s": t_solve,
           "iters_min_max_mean": [min(iters), max(iters), float(np.mean(iters))], "converged": conv,
           "data": "synthetic"}
    if cert is not None:
        out["certificate"] = cert
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="split_bf16", choices=["fp32", "split_bf16", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-eig", action="store_true")
    ap.add_argument("--certify", default="both", choices=["none", "mixed", "both"],
                    help="oracle certificate of the mixed (and FP64) Ritz vectors at the end (CPU)")
    ap.add_argument("--only-ladder", action="store_true",
                    help="time only the ladder term (for counter runs)")
    ap.add_argument("--only-sigma", action="store_true",
                    help="time only the sigma build at --precision (for kernel traces)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--vendor-gemm", action="store_true",
                    help="with --only-sigma: also time torch's bf16 GEMM (hipBLASLt) on the flop of the build's "
                         "largest split-bf16 products")
    ap.add_argument("--c3", action="store_true",
                    help="IP and EA on the large configuration: split-bf16 vs FP64 solves, per root")
    ap.add_argument("--c3-kinds", default="IP,EA", help="with --c3: comma-separated subset of IP,EA")
    ap.add_argument("--c3-precisions", default="split_bf16,fp64",
                    help="with --c3: comma-separated subset of split_bf16,fp64 (the per-root difference needs both)")
    ap.add_argument("--c4", type=int, default=0,
                    help="instead: batched solve of the first N instances of the 64-instance draw")
    ap.add_argument("--c4-budget-gb", type=float, default=200.0)
    ap.add_argument("--c4-certify-s", type=float, default=0.0,
                    help="with --c4: CPU seconds for oracle certificates of the roots (cheapest instances first)")
    ap.add_argument("--verbose", action="store_true", help="one line per Davidson iteration on stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on one GPU; "
              f"sharding over several is not built)", file=sys.stderr)
        sys.exit(2)
    for opt, val, allowed in (("--c3-kinds", args.c3_kinds, ("IP", "EA")),
                              ("--c3-precisions", args.c3_precisions, ("split_bf16", "fp64"))):
        if not val or any(v not in allowed for v in val.split(",")):
            ap.error(f"{opt} takes a comma-separated subset of {','.join(allowed)}")
    if args.c3:
        run_c3(args)
        return
    if args.c4:
        run_c4(args)
        return

    import torch
    import paper_2511_21640_amd as adc
    from adcgen import config_problem

    P = config_problem("C2")
    k = P.n_roots
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    h = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision=args.precision, conv_tol=1e-7)
    init_wall = time.perf_counter() - t0
    rng = np.random.default_rng(3)
    Y = torch.from_numpy(rng.standard_normal((k, h.dim)) + 1j * rng.standard_normal((k, h.dim))).cuda()
    S = torch.empty_like(Y)
    print(f"[bench] C2 dim={h.dim} init {h.init_ms:.0f} ms; timing {args.precision}", file=sys.stderr, flush=True)

    if args.calib_copy:
        src = torch.empty(1 << 26, dtype=torch.complex128, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 1073741824 bytes read, 1073741824 bytes written", file=sys.stderr,
              flush=True)
        del src, dst
    if args.only_ladder:
        ms_lad = time_calls(lambda: h.sigma_term("ladder", Y, S, precision=args.precision), args.steps,
                            args.warmup, stream)
        print(f"[bench] ladder term {ms_lad:.2f} ms", file=sys.stderr, flush=True)
        h.close()
        return
    ms = time_calls(lambda: h.sigma(Y, S, precision=args.precision), args.steps, args.warmup, stream)
    print(f"[bench] {args.precision} sigma {ms:.2f} ms/build", file=sys.stderr, flush=True)
    if args.only_sigma:
        h.close()
        if args.vendor_gemm:
            print(json.dumps({"vendor_gemm": vendor_gemm(args.steps, args.warmup)}))
        return
    ms64 = time_calls(lambda: h.sigma(Y, S, precision="fp64"), max(3, args.steps // 2), 1, stream)
    print(f"[bench] fp64 sigma {ms64:.2f} ms/build", file=sys.stderr, flush=True)
    ms_lad = time_calls(lambda: h.sigma_term("ladder", Y, S, precision=args.precision), args.steps, 1, stream)
    print(f"[bench] ladder term {ms_lad:.2f} ms", file=sys.stderr, flush=True)

    terms = core_terms(P.o, P.v, P.n_chol, k)
    flops, lad_flops = core_flops(P.o, P.v, P.n_chol, k)
    peak = PEAK_TFLOPS[args.precision]
    eff_peak = peak / 3.0 if args.precision == "split_bf16" else peak
    achieved = lad_flops / (ms_lad * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "sigma builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "EE-ADC(2)+x(3) x=0.5, o=20 v=120 Nchol=900, 8 trial vectors (C2)",
                   "kind": "EE", "o": P.o, "v": P.v, "n_chol": P.n_chol, "k": k, "x": P.x,
                   "dim": h.dim, "precision": args.precision},
        "tflops_core": flops / (ms * 1e-3) / 1e12,
        "core_flop_per_build": flops,
        "core_cmac_per_term": terms,
        "core_count": "8 flop per complex MAC of: assembly 2 N Pv^2, pp-ladder k Po Pv^2, ring k (ov)^3, "
                      "hh-ladder k Po^2 Pv, coupling N o v^3 + k o^2 v^3 + k o^3 v^2",
        "fp64": {"ms_per_build": ms64, "builds_per_s": 1000.0 / ms64,
                 "tflops_core": flops / (ms64 * 1e-3) / 1e12},
        "speedup_vs_fp64": ms64 / ms,
        "init_ms": h.init_ms,
        "init_wall_s": init_wall,
        "roofline": {"bound": "mfma", "kernel": "ladder term (assembly GEMM + pack + contraction GEMM)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": LADDER_TRAFFIC_BYTES.get(args.precision), "traffic_unit": "bytes per launch",
                     "ms_per_launch": ms_lad, "flop_per_launch": lad_flops,
                     "flop_count": "8 (2 N Pv^2 + k Po Pv^2): every <ab||cd> (a<b, c<d) from two Cholesky sums, "
                                   "plus the contraction",
                     "effective_peak": eff_peak, "frac_effective": achieved / eff_peak,
                     "mfma_exec_frac_counters": MFMA_COUNTERS.get(args.precision, {}).get("exec_frac"),
                     "mfma_busy_frac_counters": MFMA_COUNTERS.get(args.precision, {}).get("busy_frac")},
    }
    if not args.no_eig and args.precision != "fp64":
        # mixed: reduced-precision sweeps to |r| <= 1e-4, then FP64 until the
        # FP64 residual is <= 3e-5 (eigenvalue error <= |r|^2/gap ~ 1e-7 Eh);
        # reference: FP64 throughout to |r| <= 1e-7
        # both solves iterate on the device (captured iteration graphs)
        hm = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision=args.precision, conv_tol=3e-5,
                        graphs=True)
        t0 = time.perf_counter()
        r_mixed = hm.davidson()
        t_mixed = time.perf_counter() - t0
        hm.close()
        h64 = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision="fp64", conv_tol=1e-7, graphs=True)
        t0 = time.perf_counter()
        r64 = h64.davidson(want_vectors=args.certify == "both")
        t64 = time.perf_counter() - t0
        h64.close()
        out["eigen"] = {"omega_fp64": r64["omega"].tolist(), "omega_mixed": r_mixed["omega"].tolist(),
                        "max_abs_diff_Eh": float(np.abs(r64["omega"] - r_mixed["omega"]).max()),
                        "per_root_diff_Eh": np.abs(r64["omega"] - r_mixed["omega"]).tolist(),
                        "solve_s_mixed": t_mixed, "solve_s_fp64": t64, "tol_mixed_fp64_residual": 3e-5,
                        "tol_fp64": 1e-7, "iteration": "device (captured graphs)",
                        "iters_mixed": r_mixed["iters"], "iters_fp64": r64["iters"],
                        "converged": bool(r_mixed["converged"].all() and r64["converged"].all())}
        print(f"[bench] davidson mixed {t_mixed:.1f} s fp64 {t64:.1f} s, max |dw| "
              f"{out['eigen']['max_abs_diff_Eh']:.2e}", file=sys.stderr, flush=True)
        if args.certify != "none" and not args.no_cpu:
            # the gaps: the lowest k + 2 roots (loose mixed solve)
            hw = adc.Handle("EE", P.o, P.v, P.eps, P.L, k + 2, x=P.x, precision=args.precision, conv_tol=1e-4,
                            refine_fp64=False)
            spec = hw.davidson(want_vectors=False)["omega"]
            hw.close()
            X = r_mixed["vectors"].cpu().numpy()
            om = r_mixed["omega"]
            if args.certify == "both":
                X = np.concatenate([X, r64["vectors"].cpu().numpy()])
                om = np.concatenate([om, r64["omega"]])
            print(f"[bench] oracle certificate of {X.shape[0]} Ritz vectors (CPU) ...", file=sys.stderr, flush=True)
            cert, t_setup, t_sigma = certify(P, X, om, spec, [j % k for j in range(X.shape[0])])
            cm = cert[:k]
            out["eigen"]["certificate"] = {
                "method": "oracle FP64 sigma of the GPU Ritz vectors: |omega_gpu - theta| + |r|^2/gap per root",
                "mixed": cm, "max_bound_mixed_Eh": max(c["bound_Eh"] for c in cm),
                "fp64_vs_oracle_theta_of_mixed_Eh": [abs(r64["omega"][j] - cm[j]["theta_oracle"]) for j in range(k)]}
            if args.certify == "both":
                cf = cert[k:]
                out["eigen"]["certificate"]["fp64"] = cf
                out["eigen"]["certificate"]["max_bound_fp64_Eh"] = max(c["bound_Eh"] for c in cf)
            print(f"[bench] certified mixed max error {out['eigen']['certificate']['max_bound_mixed_Eh']:.2e} Eh "
                  f"(oracle sigma {t_sigma:.1f} s)", file=sys.stderr, flush=True)
            # the oracle's sigma of these vectors is a full build (every block,
            # M11 included) of X.shape[0] vectors: k of them make one build
            info = cpu_info()
            out["cpu_baseline"] = {"value": (X.shape[0] / k) / t_sigma, "unit": "sigma builds/s",
                                   "cores": info["blas_threads"] or info["affinity"], "kind": "oracle",
                                   "sample": f"oracle numpy FP64 matrix-free sigma (all blocks, M11 included) of "
                                             f"the {X.shape[0]} certified Ritz vectors = {X.shape[0] / k:g} full "
                                             f"builds of {k} vectors, {t_sigma:.1f} s; integral and amplitude "
                                             f"setup {t_setup:.1f} s excluded",
                                   **info}
    h.close()
    if "cpu_baseline" not in out and not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        X = np.random.default_rng(5).standard_normal((1, h.dim)) + 0j
        _, t_setup, t_sigma = oracle_build(P, X)
        info = cpu_info()
        out["cpu_baseline"] = {"value": (1.0 / k) / t_sigma, "unit": "sigma builds/s",
                               "cores": info["blas_threads"] or info["affinity"], "kind": "oracle",
                               "sample": f"oracle numpy FP64 matrix-free sigma (all blocks, M11 included) of 1 of "
                                         f"{k} vectors, {t_sigma:.1f} s; setup {t_setup:.1f} s excluded", **info}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
