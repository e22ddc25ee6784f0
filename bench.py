"""Benchmark: quadrature-pair interactions/s of the Galerkin PMCHWT apply.

One step = one full operator apply y = A x on the sphere workload with 10,242
vertices / 20,480 triangles (k0 = 10, k1 = 10.5, density ratio 1.05): gather,
FP32 pair kernel for the exterior pass (union of boundaries, k0) and the
interior pass (k1), reduction, test-side projection and the FP64 singular
correction.  Inputs are resident in HBM before the timed region.

Also reported: GMRES time-to-solve at 1e-5 on the same problem (plane wave),
the roofline of the pair kernel (HIP events on the library's stream) and the
FP64 CPU oracle timed on a bounded sample of rows on this host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-solve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BEM apply G quad-pair interactions/s + GMRES time-to-solve at 1e-5; p50/p99 latency"
FLOP_PER_PAIR = 140.0          # fused V, K, K', W multitrace pair (per-pair count of the design notes)
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector peak


def pairs_per_apply(prob):
    m_all = prob.n_points
    return float(m_all) ** 2 + sum(float(6 * d.n_triangles) ** 2 for d in prob.domains)


def cpu_baseline(prob, seconds_target=15.0):
    """FP64 oracle rows on this host; scaled to interactions/s of a full apply."""
    import oracle
    from bem_inputs import vectors

    nthreads = os.cpu_count() or 1
    env_threads = os.environ.get("OMP_NUM_THREADS")
    if env_threads:
        nthreads = int(env_threads)
    x = vectors.random_complex(prob.n_unknowns, seed=0)
    nv = sum(d.n_vertices for d in prob.domains)
    # warm up (thread pool, rule tables), calibrate on 16 vertices, then run a
    # sample sized for ~seconds_target
    oracle.pmchwt_rows(prob, vectors.random_rows(nv, 2, seed=10))
    n_v = 16
    t0 = time.perf_counter()
    rows = vectors.random_rows(nv, n_v, seed=11)
    R = oracle.pmchwt_rows(prob, rows)
    _ = R @ x
    dt = time.perf_counter() - t0
    n_v2 = int(np.clip(n_v * seconds_target / max(dt, 1e-3), n_v, 4096))
    rows = vectors.random_rows(nv, n_v2, seed=12)
    t0 = time.perf_counter()
    R = oracle.pmchwt_rows(prob, rows)   # Dirichlet rows of the sampled vertices (all four operators computed)
    _ = R @ x
    dt = time.perf_counter() - t0
    frac = n_v2 / nv
    return {"value": frac * pairs_per_apply(prob) / dt, "unit": "quad-pair interactions/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"FP64 oracle rows of {n_v2} random test vertices of {nv} (V, K, K', W at k0 and k1, "
                      f"6-point far rule + Sauter-Schwab order 6), {dt:.1f} s, scaled by {nv}/{n_v2}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-assembled", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the heuristic launch shapes")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only a 1 GiB elementwise copy (the counter scale) and 3 applies, for HBM counters")
    ap.add_argument("--level", type=int, default=5, help="icosphere level of the sphere workload (5: 10,242 v)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding is a design note, not a code path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1910_01011_amd as bem
    from bem_inputs import configs, vectors

    torch.cuda.set_device(0)
    prob = configs.config2() if args.level == 5 else configs.sphere_problem(args.level, 10.0, 10.5, 1.05)
    t_setup = time.perf_counter()
    P = bem.Problem.from_config(prob, device=True, autotune=not args.no_autotune)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
    y = torch.empty_like(x)
    if args.traffic_probe:
        traffic_probe(P, x, y, torch)
        return
    for _ in range(args.warmup):
        P.apply(x, out=y)
    torch.cuda.synchronize()
    pair_ms = []
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.apply(x, out=y)
        tm = P.timings()       # waits for this apply's events on the library stream
        step_ms.append(tm[0])
        pair_ms.append(tm[1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = pairs_per_apply(prob)
    ms_per_step = 1e3 * wall / args.steps
    value = pairs * args.steps / wall
    pair_avg = float(np.mean(pair_ms))
    achieved = FLOP_PER_PAIR * pairs / (pair_avg * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "quad-pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: on-the-fly PMCHWT apply, icosphere {prob.domains[0].n_vertices} v / "
                               f"{prob.domains[0].n_triangles} t, k0=10, k1=10.5, rho1/rho0=1.05, 6-pt far rule, "
                               f"Sauter-Schwab order 6 singular pass",
                   "pairs_per_apply": pairs, "unknowns": prob.n_unknowns, "setup_s": t_setup,
                   "autotune": not args.no_autotune, "pair_launch_shape": list(P.pair_launch_shape()),
                   "apply_ms_p50": float(np.percentile(step_ms, 50)),
                   "apply_ms_p99": float(np.percentile(step_ms, 99))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": recorded_traffic(),
                     "kernel": "k_pairs", "kernel_ms": pair_avg, "flop_per_pair": FLOP_PER_PAIR},
    }
    if not args.no_solve:
        # GMRES(100) on the on-the-fly operator, plane wave along +z, without and
        # with the OSRC preconditioner (N_Pade = 4, R_eps = 0.1 = radius / 10)
        inc = bem.Incident.plane_waves([[0.0, 0.0, 1.0]])
        b = P.rhs(inc)
        g = {}
        for pname, pc in (("plain", bem.BEM_PRECOND_NONE), ("osrc", bem.BEM_PRECOND_OSRC)):
            for tol in (1e-5, 1e-6):
                torch.cuda.synchronize()
                ts = time.perf_counter()
                u, info = P.solve(b, bem.solve_options(tol=tol, restart=100, max_iter=400, precond=pc, n_pade=4,
                                                       r_eps=0.1, theta=np.pi / 3))
                torch.cuda.synchronize()
                ts = time.perf_counter() - ts
                g[f"{pname}_tol{tol:g}"] = {"time_to_solve_s": ts, "iterations": info[0]["iterations"],
                                            "rel_residual": info[0]["rel_residual"],
                                            "converged": info[0]["converged"]}
        out["gmres"] = g
    if not args.no_assembled:
        del P
        torch.cuda.empty_cache()
        out["assembled"] = assembled_section(prob, bem, vectors, torch, autotune=not args.no_autotune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


COPY_PROBE_BYTES = 1 << 30     # bytes read (and written) by the copy of the traffic probe


def traffic_probe(P, x, y, torch):
    """Kernels for the HBM-counter runs: a plain elementwise copy of known size
    (1 GiB read, 1 GiB written; its FETCH_SIZE / WRITE_SIZE give the counter
    scale) and three applies."""
    a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b
    for _ in range(3):
        P.apply(x, out=y)
    torch.cuda.synchronize()
    print("traffic probe done", flush=True)


def recorded_traffic():
    """HBM bytes per k_pairs launch from the committed counter summary, or None
    when the pair kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_pairs_sphere10242_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1910_01011_amd", "csrc", "k_farfield.hip")
    try:
        fields = {}
        for line in open(path):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("k_farfield.hip sha256") != digest:
            return None
        return float(fields["HBM bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 MFMA
HBM_PEAK_GBPS = 8000.0


def assembled_section(prob, bem, vectors, torch, autotune=True):
    """Assembled mode on the same problem: dense assembly, GEMV (HBM roofline),
    multi-RHS GEMM (MFMA roofline) and time-to-solve of the three precision forms."""
    n = prob.n_unknowns
    res = {"n": n}
    t = time.perf_counter()
    P = bem.Problem.from_config(prob, device=True, mode=bem.BEM_ASSEMBLED_SPLIT_BF16, autotune=autotune)
    torch.cuda.synchronize()
    res["assembly_s"] = time.perf_counter() - t
    x = torch.from_numpy(vectors.random_complex(n, seed=0)).cuda()
    for _ in range(2):
        P.apply(x)
    ts = []
    for _ in range(10):
        P.apply(x)
        ts.append(P.timings()[1])
    ms = float(np.median(ts))
    gbps = 8.0 * n * n / (ms * 1e-3) / 1e9
    res["gemv"] = {"ms": ms, "GBps": gbps, "frac_hbm": gbps / HBM_PEAK_GBPS, "bytes": 8.0 * n * n}
    for R in (64, 256):
        X = torch.from_numpy(vectors.random_complex(n, seed=1, n_rhs=R)).cuda()
        for kern, key, peak, fl in ((bem.BEM_APPLY_MFMA_SPLIT_BF16, "bf16x3", BF16_PEAK_TFLOPS, 24.0),
                                    (bem.BEM_APPLY_MFMA_FP32, "fp32", FP32_MFMA_PEAK_TFLOPS, 8.0)):
            for _ in range(2):
                P.apply(X, kernel=kern)
            ts = []
            for _ in range(5):
                P.apply(X, kernel=kern)
                ts.append(P.timings()[1])
            ms = float(np.median(ts))
            tf = fl * n * n * R / (ms * 1e-3) / 1e12
            res[f"gemm_{key}_R{R}"] = {"ms": ms, "TFLOPs": tf, "frac": tf / peak, "peak": peak}
    # time-to-solve at 1e-5 for one plane wave and for 64 plane waves
    dirs = np.random.default_rng(7).standard_normal((64, 3))
    for R in (1, 64):
        b = P.rhs(bem.Incident.plane_waves(dirs[:R]))
        for name, prec in (("plain_fp32", bem.BEM_PREC_FP32), ("split_bf16_fgmres", bem.BEM_PREC_SPLIT_BF16_FGMRES),
                           ("fp32_mfma_fgmres", bem.BEM_PREC_FP32_MFMA_FGMRES)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            u, info = P.solve(b, bem.solve_options(tol=1e-5, restart=100 if prec == bem.BEM_PREC_FP32 else 30,
                                                   max_iter=400, precision=prec, inner_tol=1e-3))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            res[f"solve_{name}_R{R}"] = {"s": dt, "iterations": int(max(i["iterations"] for i in info)),
                                         "max_rel_residual": float(max(i["rel_residual"] for i in info)),
                                         "all_converged": all(i["converged"] for i in info)}
    return res


if __name__ == "__main__":
    main()
