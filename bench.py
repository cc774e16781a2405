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
LADDER_TRAFFIC_BYTES = {"split_bf16": 7.230e9 + 1.511e9}
DTYPE = {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16x3"}


def core_flops(o, v, N, k):
    """Algorithmic (core) flop of one EE sigma build, 8 flop per complex MAC:
    vvvv assembly of the Hermitian upper part 2 N Pv (Pv + 1) / 2 (each
    <ab||cd>, ab <= cd, is two Cholesky sums of N), pp-ladder k Po Pv^2, ring
    k (ov)^3, hh-ladder k Po^2 Pv, first-order coupling k o^2 v^3
    (three-external class stored)."""
    Po, Pv = o * (o - 1) // 2, v * (v - 1) // 2
    assembly = N * Pv * (Pv + 1)
    ladder = k * Po * Pv * Pv
    ring = k * (o * v) ** 3
    hh = k * Po * Po * Pv
    coupling = k * o * o * v ** 3
    return 8.0 * (assembly + ladder + ring + hh + coupling), 8.0 * (assembly + ladder)


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


def cpu_baseline(P, k):
    """The oracle's matrix-free FP64 sigma on the host, one of the k roots, M11
    product and integral setup excluded (they are one-off)."""
    from oracle.adc_terms import Ints, dims, sigma_block
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    ints = Ints(P.eps, P.L, P.o)
    for c in ("vvvv", "ovvv", "vovv", "ovov", "oovv", "vvoo", "ooov", "oooo"):
        ints.g(c)
    ints.amp("t")
    n1, n2 = dims("EE", P.o, P.v)
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((1, n1 + n2)) + 1j * rng.standard_normal((1, n1 + n2))
    t0 = time.perf_counter()
    for blk, od, f in [("12", 1, 1.0), ("12", 2, P.x), ("21", 1, 1.0), ("21", 2, P.x), ("22", 0, 1.0), ("22", 1, P.x)]:
        src = Y[:, :n1] if blk[1] == "1" else Y[:, n1:]
        sigma_block(ints, "EE", blk, od, src)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / (k * dt), "unit": "sigma builds/s", "cores": int(cores), "kind": "oracle",
            "sample": f"1 of {k} trial vectors of one build (numpy FP64 einsum, integrals precomputed, "
                      f"M11 product excluded), {dt:.1f} s"}


def c4_device_gb(kind, o, v, N, k):
    """Rough device memory of one instance of the batched workload, GB:
    (resident, transient).  Resident: L blocks, stored integral classes,
    amplitudes and intermediates, M11, the cached split-bf16 planes.
    Transient (while its lane solves it): Davidson subspace (6k vectors of V and S, three k-blocks), the sigma
    workspace of one pass (unpacked doubles, at most 16 GiB) and the ladder
    batch (4 GiB)."""
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
    return res * 16 / 1e9, tr * 16 / 1e9


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
    t_init = t_build = t_solve = 0.0
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
        t0 = time.perf_counter()
        for j in range(len(idx)):
            B.sigma(j, Ys[j])
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        del Ys
        t0 = time.perf_counter()
        out, rc = B.davidson()
        t_solve += time.perf_counter() - t0
        for j, i in enumerate(idx):
            res[i] = out[j]
        print(f"[c4] wave {w + 1}: solve {time.perf_counter() - t0:.1f} s, rc {rc}", file=sys.stderr, flush=True)
        B.close()
        torch.cuda.empty_cache()
    iters = [res[i]["iters"] for i in range(len(draw))]
    conv = all(bool(res[i]["converged"].all()) for i in range(len(draw)))
    kinds = [d[0] for d in draw]
    out = {"metric": "batched solve of uneven EE/IP/EA instances", "workload": f"{len(draw)} instances of the "
           f"64-instance draw (EE {kinds.count('EE')}, IP {kinds.count('IP')}, EA {kinds.count('EA')}), x=0.5",
           "precision": args.precision, "waves": len(waves), "roots": int(sum(d[4] for d in draw)),
           "init_s": t_init, "all_instance_build_s": t_build, "core_flop_all_instance_build": flop_build,
           "all_instance_build_tflops": flop_build / t_build / 1e12, "solve_s": t_solve,
           "iters_min_max_mean": [min(iters), max(iters), float(np.mean(iters))], "converged": conv,
           "data": "synthetic"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="split_bf16", choices=["fp32", "split_bf16", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-eig", action="store_true")
    ap.add_argument("--only-ladder", action="store_true",
                    help="time only the ladder term (for counter runs)")
    ap.add_argument("--only-sigma", action="store_true",
                    help="time only the sigma build at --precision (for kernel traces)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--c4", type=int, default=0,
                    help="instead: batched solve of the first N instances of the 64-instance draw")
    ap.add_argument("--c4-budget-gb", type=float, default=200.0)
    ap.add_argument("--verbose", action="store_true", help="one line per Davidson iteration on stderr")
    args = ap.parse_args()
    if args.c4:
        run_c4(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on one GPU; "
              f"sharding over several is not built)", file=sys.stderr)
        sys.exit(2)

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
        return
    ms64 = time_calls(lambda: h.sigma(Y, S, precision="fp64"), max(3, args.steps // 2), 1, stream)
    print(f"[bench] fp64 sigma {ms64:.2f} ms/build", file=sys.stderr, flush=True)
    ms_lad = time_calls(lambda: h.sigma_term("ladder", Y, S, precision=args.precision), args.steps, 1, stream)
    print(f"[bench] ladder term {ms_lad:.2f} ms", file=sys.stderr, flush=True)

    flops, lad_flops = core_flops(P.o, P.v, P.n_chol, k)
    peak = PEAK_TFLOPS[args.precision]
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
        "fp64": {"ms_per_build": ms64, "builds_per_s": 1000.0 / ms64,
                 "tflops_core": flops / (ms64 * 1e-3) / 1e12},
        "speedup_vs_fp64": ms64 / ms,
        "init_ms": h.init_ms,
        "init_wall_s": init_wall,
        "roofline": {"bound": "mfma", "kernel": "ladder term (assembly GEMM + pack + contraction GEMM)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": LADDER_TRAFFIC_BYTES.get(args.precision), "traffic_unit": "bytes per launch",
                     "ms_per_launch": ms_lad, "flop_per_launch": lad_flops,
                     "effective_peak": peak / 3.0 if args.precision == "split_bf16" else peak,
                     "frac_effective": achieved / (peak / 3.0 if args.precision == "split_bf16" else peak)},
    }
    if not args.no_eig and args.precision != "fp64":
        # mixed: reduced-precision sweeps to |r| <= 1e-4, then FP64 until the
        # FP64 residual is <= 3e-5 (eigenvalue error <= |r|^2/gap ~ 1e-7 Eh);
        # reference: FP64 throughout to |r| <= 1e-7
        hm = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision=args.precision, conv_tol=3e-5)
        t0 = time.perf_counter()
        r_mixed = hm.davidson(want_vectors=False)
        t_mixed = time.perf_counter() - t0
        hm.close()
        h64 = adc.Handle("EE", P.o, P.v, P.eps, P.L, k, x=P.x, precision="fp64", conv_tol=1e-7)
        t0 = time.perf_counter()
        r64 = h64.davidson(want_vectors=False)
        t64 = time.perf_counter() - t0
        out["eigen"] = {"omega_fp64": r64["omega"].tolist(), "omega_mixed": r_mixed["omega"].tolist(),
                        "max_abs_diff_Eh": float(np.abs(r64["omega"] - r_mixed["omega"]).max()),
                        "per_root_diff_Eh": np.abs(r64["omega"] - r_mixed["omega"]).tolist(),
                        "solve_s_mixed": t_mixed, "solve_s_fp64": t64, "tol_mixed_fp64_residual": 3e-5,
                        "tol_fp64": 1e-7,
                        "iters_mixed": r_mixed["iters"], "iters_fp64": r64["iters"],
                        "converged": bool(r_mixed["converged"].all() and r64["converged"].all())}
        print(f"[bench] davidson mixed {t_mixed:.1f} s fp64 {t64:.1f} s, max |dw| "
              f"{out['eigen']['max_abs_diff_Eh']:.2e}", file=sys.stderr, flush=True)
        h64.close()
    h.close()
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
