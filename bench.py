"""Benchmark: quadrature-pair interactions/s of the Galerkin PMCHWT apply.

One step = one full on-the-fly operator apply y = A x on the rib-cage stack
(the paper's ribs + fat layer + liver model problem, synthetic stand-in): a fat
slab, five capsule ribs and a liver box, 53,524 vertices / 107,048 unknowns
meshed at lambda/6, exterior k0 = 2 pi plus one interior pass per domain.  The
apply is gather, the FP32 pair kernel (exterior pass over the union of all
boundaries, interior passes per domain), reduction, test-side projection and
the FP64 singular correction.  Inputs are resident in HBM before the timed
region.

Also on the line: the GMRES time-to-solve of the stack's 256-piston field to a
true (unpreconditioned, on-the-fly operator) relative residual of 1e-5, the
roofline of the pair kernel (HIP events on the library's stream), the FP64 CPU
oracle timed on a bounded sample of rows on this host, and, as sub-objects,
the 10,242-vertex sphere (apply, solves with and without OSRC, assembled
GEMV/GEMM paths) and a bounded kidney serving run (request latency p50/p99,
solves/s, continuous batching).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-solve] [--no-sphere]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BEM apply G quad-pair interactions/s + GMRES time-to-solve at 1e-5; p50/p99 latency"
FLOP_PER_PAIR = 140.0          # fused V, K, K', W multitrace pair (per-pair count of the design notes)
FLOP_PER_PAIR_V = 21.0         # single-layer pair alone: difference, r^2, r, phase, G, one complex multiply-add
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector peak
ACHIEVED_KIND = ("algorithmic: 140 FLOP per quadrature-point pair (difference, r^2, rsq, phase, G, F and 15 "
                 "complex channel multiply-adds) x pairs per launch / mean HIP-event duration of the kernel")


def pairs_per_apply(prob):
    m_all = prob.n_points
    return float(m_all) ** 2 + sum(float(6 * d.n_triangles) ** 2 for d in prob.domains)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, seconds_target=8.0, repeats=3):
    """FP64 oracle rows on this host, scaled to interactions/s of a full apply;
    the median of ``repeats`` timings of the same sample."""
    import oracle
    from bem_inputs import vectors

    nthreads = os.cpu_count() or 1
    env_threads = os.environ.get("OMP_NUM_THREADS")
    if env_threads:
        nthreads = int(env_threads)
    x = vectors.random_complex(prob.n_unknowns, seed=0)
    nv = sum(d.n_vertices for d in prob.domains)
    # warm up (thread pool, rule tables), calibrate on a few vertices, then time
    # a sample sized for about seconds_target, three times
    oracle.pmchwt_rows(prob, vectors.random_rows(nv, 1, seed=10))
    n_v = 2
    t0 = time.perf_counter()
    R = oracle.pmchwt_rows(prob, vectors.random_rows(nv, n_v, seed=11))
    dt = time.perf_counter() - t0
    n_v2 = int(np.clip(n_v * seconds_target / max(dt, 1e-3), n_v, 4096))
    rows = vectors.random_rows(nv, n_v2, seed=12)
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        R = oracle.pmchwt_rows(prob, rows)   # Dirichlet rows of the sampled vertices (all four operators computed)
        _ = R @ x
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    frac = n_v2 / nv
    return {"value": frac * pairs_per_apply(prob) / dt, "unit": "quad-pair interactions/s", "cores": nthreads,
            "kind": "oracle", "cpu_model": cpu_model(), "repeats": repeats,
            "times_s": [round(t, 3) for t in times],
            "sample": f"{prob.name}: FP64 oracle rows of {n_v2} random test vertices of {nv} (V, K, K', W at k0 and "
                      f"each domain's k, 6-point far rule + Sauter-Schwab order 6), median of {repeats} runs "
                      f"{dt:.1f} s, scaled by {nv}/{n_v2}"}


def profile_fields(name, source="k_farfield.hip"):
    """Key-value lines of a committed profile summary, or None when the kernel
    source changed since the counters were taken (SHA-256 recorded there)."""
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_1910_01011_amd", "csrc", source)
    try:
        fields = {}
        for line in open(path):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get(f"{source} sha256") != digest:
            return None
        return fields
    except OSError:
        return None


def recorded_traffic(name, launch_shape):
    """HBM bytes per k_pairs launch from a committed counter summary, or None
    (source changed, or the summary was taken at another launch shape: the
    partial sums written grow with the trial splits)."""
    f = profile_fields(name)
    try:
        key = "HBM bytes per launch ({} {})".format(*launch_shape)
        return float(f[key]) if f and key in f else None
    except (KeyError, ValueError, IndexError):
        return None


def recorded_executed_flop(name):
    """Executed FP32 FLOP per k_pairs launch from a committed VALU-counter
    summary (64 lanes x (ADD + MUL + TRANS + 2 FMA) F32 instructions), or None."""
    f = profile_fields(name)
    try:
        return float(f["executed FP32 FLOP per launch"]) if f else None
    except (KeyError, ValueError):
        return None


def time_applies(P, x, y, steps, warmup, torch):
    """Warm-up applies, then `steps` timed applies: wall time of the whole
    region, and per apply the HIP-event durations of the apply and of the pair
    kernel (recorded on the library's stream)."""
    for _ in range(warmup):
        P.apply(x, out=y)
    torch.cuda.synchronize()
    pair_ms, step_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        P.apply(x, out=y)
        tm = P.timings()       # waits for this apply's events on the library stream
        step_ms.append(tm[0])
        pair_ms.append(tm[1])
    torch.cuda.synchronize()
    return time.perf_counter() - t0, step_ms, pair_ms


def pair_roofline(pairs, pair_ms, traffic_profile, valu_profile, launch_shape):
    k_ms = float(np.mean(pair_ms))
    achieved = FLOP_PER_PAIR * pairs / (k_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": recorded_traffic(traffic_profile, launch_shape),
            "kernel": "k_pairs", "kernel_ms": k_ms, "flop_per_pair": FLOP_PER_PAIR, "achieved_kind": ACHIEVED_KIND}
    ex = recorded_executed_flop(valu_profile)
    if ex is not None:
        t = ex / (k_ms * 1e-3) / 1e12
        roof["executed"] = {"tflops": t, "frac": t / FP32_PEAK_TFLOPS, "flop_per_launch": ex,
                            "flop_per_pair": ex / pairs, "source": f"profiles/{valu_profile}"}
    else:
        roof["executed"] = None
    return roof


def osrc_apply_ms(P, prob, bem, torch, n_pade, r_eps, cg_tol=1e-6, reps=5):
    """Median wall time of one OSRC preconditioner apply (one residual vector,
    inner COCG to cg_tol: the tolerance a GMRES solve to 1e-5 gives them)."""
    from bem_inputs import vectors
    y = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=5)).cuda()
    opts = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=n_pade, r_eps=r_eps, theta=np.pi / 3,
                             osrc_tol=cg_tol)
    P.precondition(y, opts)
    ts = []
    for _ in range(reps):
        _, t = _timed(torch, lambda: P.precondition(y, opts))
        ts.append(1e3 * t)
    return {"apply_ms": float(np.median(ts)), "n_pade": n_pade, "r_eps": r_eps, "cocg_tol": cg_tol}


def ribcage_time_to_solve(P, prob, bem, torch):
    """Time-to-solve of the stack's 256-piston bowl (one field, all pistons at
    unit amplitude) to a true relative residual of 1e-5 of the on-the-fly FP32
    operator: flexible GMRES(10) whose Arnoldi vectors and residual use the
    on-the-fly apply (FP64 accumulation), with inner OSRC-preconditioned
    GMRES(300) to 1e-3 on the hierarchical matrix (ACA, eps 1e-4, leaves of 64,
    eta 2).  OSRC with the paper's parameters relative to the wavelength:
    N_Pade = 4 and R_eps = lambda_0 / 3 (its sphere: 5e-4 m at lambda_0 =
    1.5 mm).  The hierarchical-matrix build is set-up and reported beside the
    solve."""
    from bem_inputs import pistons
    c, n, a = pistons.bowl_array()
    b, t_rhs = _timed(torch, lambda: P.rhs(bem.Incident.pistons(c, n, a, 1.0, np.zeros(len(c), dtype=int))))
    log(f"ribcage right-hand side (256 pistons, 24 monopoles each) {t_rhs:.2f} s")
    hinfo, t_build = _timed(torch, lambda: P.hmatrix_build(eps=1e-4, leaf_vertices=64, eta=2.0))
    log(f"ribcage H-matrix: {hinfo['bytes'] / 1e9:.1f} GB, build {t_build:.1f} s")
    r_eps = (2.0 * np.pi / prob.k0.real) / 3.0
    opts = bem.solve_options(tol=1e-5, restart=10, max_iter=10, precond=bem.BEM_PRECOND_OSRC, n_pade=4, r_eps=r_eps,
                             theta=np.pi / 3, precision=bem.BEM_PREC_HMATRIX_FGMRES, inner_tol=1e-3,
                             inner_restart=300, inner_max_iter=1000)
    (u, info), t = _timed(torch, lambda: P.solve(b, opts))
    log(f"ribcage time-to-solve {t:.1f} s, residual {info[0]['rel_residual']:.2e}")
    return {"tol": 1e-5, "time_to_solve_s": t, "converged": info[0]["converged"],
            "rel_residual": info[0]["rel_residual"], "outer_iterations": info[0]["iterations"],
            "setup_hmatrix_build_s": t_build, "setup_rhs_s": t_rhs,
            "hmatrix": {k: hinfo[k] for k in ("bytes", "dense_bytes", "n_lowrank", "n_dense", "max_rank")},
            "method": "flexible GMRES(10), outer Arnoldi and residual on the on-the-fly FP32 operator; inner "
                      "right-hand side: OSRC-preconditioned GMRES(300) to 1e-3 on the hierarchical matrix "
                      "(ACA eps 1e-4); OSRC N_Pade 4, R_eps lambda_0/3; rel_residual is the true residual of "
                      "the on-the-fly operator", "n_pade": 4, "r_eps": r_eps}


def field_probe(bem, torch):
    """Field evaluation (representation formula off the surface, FP64, with the
    winding-number regions) of the 10,242-vertex sphere's plane-wave solution
    on 200 x 200 points over [-3 R, 3 R]^2 in the plane y = 0: median of three
    evaluations, and the (point, source quadrature point) pairs per second."""
    from bem_inputs import configs as cfg
    prob = cfg.config2()
    P = bem.Problem.from_config(prob)
    inc = bem.Incident.plane_waves([[0.0, 0.0, 1.0]])
    b = P.rhs(inc)
    u, info = P.solve(b, bem.solve_options(tol=1e-5, restart=100, max_iter=500))
    pts = cfg.grid_plane_y0(1.0, 200, 3.0)
    ts = []
    for _ in range(3):
        (field, region), t = _timed(torch, lambda: P.evaluate_field(u, pts, inc))
        ts.append(t)
    P.close()
    # one domain: every point's representation formula runs over all source points
    pairs = float(len(pts)) * sum(6 * d.n_triangles for d in prob.domains)
    t = float(np.median(ts))
    log(f"field evaluation: {len(pts)} points, {t * 1e3:.1f} ms, {pairs / t:.3e} pairs/s")
    return {"workload": prob.name, "points": len(pts), "pairs": pairs, "ms": t * 1e3, "pairs_per_s": pairs / t,
            "near_boundary_points": int(np.count_nonzero(region == -1)), "solve_iterations": info[0]["iterations"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-sphere", action="store_true", help="skip the 10,242-vertex sphere sub-object")
    ap.add_argument("--no-serving", action="store_true", help="skip the bounded kidney serving sub-object")
    ap.add_argument("--no-assembled", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the heuristic launch shapes")
    ap.add_argument("--extra", default="",
                    help="comma list of extra workloads appended to the JSON line: ribcage (OSRC GMRES on the "
                         "fly on the 53.5k-vertex stack), ribcage_assembled (26.9k vertices, 256 right-hand sides), "
                         "serving (kidney request stream), paper_sphere (the paper's 1 cm sphere at 1 MHz, fat and "
                         "rib material, 4-10 elements per wavelength, OSRC GMRES), planning (full matrix capture "
                         "of 256 pistons on the 13.5k-vertex stack, then phase conjugation and rib sparing), hmatrix "
                         "(ACA-compressed operator on the sphere and the 53.5k-vertex stack)")
    ap.add_argument("--serving-requests", type=int, default=8, help="requests per arrival rate in --extra serving")
    ap.add_argument("--serving-rates", default="2,10", help="comma list of arrival rates (1/s) of --extra serving")
    ap.add_argument("--serving-inflight", type=int, default=4, help="requests in flight at most in --extra serving")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only a 1 GiB elementwise copy (the counter scale) and 3 applies, for counter runs")
    ap.add_argument("--probe-workload", default="ribcage", choices=("ribcage", "sphere"),
                    help="workload of --traffic-probe, --osrc-probe and --hmatrix-probe")
    ap.add_argument("--osrc-probe", action="store_true",
                    help="run only five OSRC preconditioner applies of the probe workload (for kernel traces)")
    ap.add_argument("--hmatrix-probe", action="store_true",
                    help="run only the hierarchical-matrix build of the probe workload (eps 1e-4, leaves of 64, "
                         "eta 2) and one compressed apply against the on-the-fly one (for kernel traces)")
    ap.add_argument("--solve-probe", action="store_true",
                    help="run only the rib-cage stack's time-to-solve with its set-up (right-hand side and "
                         "hierarchical-matrix build), for kernel traces")
    ap.add_argument("--field-probe", action="store_true",
                    help="run only the field evaluation of the 10,242-vertex sphere's plane-wave solution on a "
                         "200 x 200 grid in the plane y = 0 (for kernel traces)")
    ap.add_argument("--gemm-reference", action="store_true",
                    help="run only torch.matmul (the vendor GEMM library) on the real-GEMM shapes of the split-BF16 "
                         "apply (BF16 and FP32) and on square shapes, as a reference for the library's kernels")
    ap.add_argument("--assembled-kernels-only", action="store_true",
                    help="assembled section without its solves (GEMV and GEMM launches only, for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding is a design note, not a code path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1910_01011_amd as bem
    from bem_inputs import configs, vectors

    torch.cuda.set_device(0)
    if args.osrc_probe:
        rib = args.probe_workload == "ribcage"
        prob = configs.ribcage(1.0) if rib else configs.config2()
        P = bem.Problem.from_config(prob, device=True, autotune=False)
        res = osrc_apply_ms(P, prob, bem, torch, 8 if rib else 4, 1.5 if rib else 0.1)
        print(json.dumps({"workload": prob.name, "osrc": res}), flush=True)
        return
    if args.gemm_reference:
        print(json.dumps({"gemm_reference": gemm_reference(torch)}), flush=True)
        return
    if args.field_probe:
        print(json.dumps({"field": field_probe(bem, torch)}), flush=True)
        return
    if args.solve_probe:
        prob = configs.ribcage(1.0)
        P = bem.Problem.from_config(prob, device=True, autotune=not args.no_autotune)
        print(json.dumps({"workload": prob.name, "time_to_solve": ribcage_time_to_solve(P, prob, bem, torch)}),
              flush=True)
        return
    if args.hmatrix_probe:
        prob = configs.ribcage(1.0) if args.probe_workload == "ribcage" else configs.config2()
        P = bem.Problem.from_config(prob, device=True, autotune=False)
        x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
        yo = P.apply(x)
        info, t_build = _timed(torch, lambda: P.hmatrix_build(eps=1e-4, leaf_vertices=64, eta=2.0))
        yh = P.apply(x, kernel=bem.BEM_APPLY_HMATRIX)
        ts = []
        for _ in range(10):
            P.apply(x, out=yh, kernel=bem.BEM_APPLY_HMATRIX)
            ts.append(P.timings()[0])
        print(json.dumps({"workload": prob.name, "hmatrix": {"build_s": t_build, "info": info,
                                                             "apply_ms": float(np.median(ts)),
                                                             "rel_diff_to_on_the_fly": float((yh - yo).norm() / yo.norm())}}),
              flush=True)
        return
    if args.traffic_probe:
        prob = configs.ribcage(1.0) if args.probe_workload == "ribcage" else configs.config2()
        P = bem.Problem.from_config(prob, device=True, autotune=not args.no_autotune)
        x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
        traffic_probe(P, x, torch.empty_like(x), torch)
        return
    prob = configs.ribcage(1.0)
    log(f"rib-cage stack: {sum(d.n_vertices for d in prob.domains)} vertices, {prob.n_unknowns} unknowns")
    P, t_setup = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, autotune=not args.no_autotune))
    log(f"set-up {t_setup:.1f} s, pair launch shape {P.pair_launch_shape()}")
    x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
    y = torch.empty_like(x)
    wall, step_ms, pair_ms = time_applies(P, x, y, args.steps, args.warmup, torch)
    pairs = pairs_per_apply(prob)
    log(f"ribcage apply {1e3 * wall / args.steps:.1f} ms per step")
    out = {
        "metric": METRIC,
        "value": pairs * args.steps / wall,
        "unit": "quad-pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: rib-cage stack (fat slab, five capsule ribs, liver box; 7 domains, "
                               f"{sum(d.n_vertices for d in prob.domains)} v / {sum(d.n_triangles for d in prob.domains)} t "
                               f"at lambda/6), on-the-fly PMCHWT apply, k0 = 2 pi, speed ratios 0.96 / 1.87 / 1.03, "
                               f"density ratios 0.95 / 1.9 / 1.07, 6-pt far rule, Sauter-Schwab order 6 singular pass",
                   "pairs_per_apply": pairs, "unknowns": prob.n_unknowns, "setup_s": t_setup,
                   "autotune": not args.no_autotune, "pair_launch_shape": list(P.pair_launch_shape()),
                   "apply_ms_p50": float(np.percentile(step_ms, 50)),
                   "apply_ms_p99": float(np.percentile(step_ms, 99))},
        "roofline": pair_roofline(pairs, pair_ms, "k_pairs_ribcage53524_hbm_traffic.md",
                                  "k_pairs_ribcage53524_valu.md", P.pair_launch_shape()),
    }
    if not args.no_solve:
        out["osrc"] = osrc_apply_ms(P, prob, bem, torch, 8, 1.5)
        log(f"ribcage OSRC apply {out['osrc']['apply_ms']:.1f} ms")
        out["time_to_solve"] = ribcage_time_to_solve(P, prob, bem, torch)
    P.close()
    P = None
    torch.cuda.empty_cache()
    if not args.no_sphere:
        out["sphere10242"] = sphere_section(args, bem, torch)
    extras = [e for e in args.extra.split(",") if e]
    if extras:
        os.environ.setdefault("BEM_PROGRESS", "50")   # solver progress lines on stderr
    for e in extras:
        log(f"extra workload {e}")
        if e == "ribcage":
            out["ribcage"] = ribcage_section(bem, torch, not args.no_autotune)
        elif e == "ribcage_assembled":
            out["ribcage_assembled"] = ribcage_assembled_section(bem, torch, not args.no_autotune)
        elif e == "serving":
            out["serving"] = serving_section(bem, torch, args.serving_requests,
                                             tuple(float(r) for r in args.serving_rates.split(",") if r),
                                             args.serving_inflight)
        elif e == "paper_sphere":
            out["paper_sphere"] = paper_sphere_section(bem, torch)
        elif e == "planning":
            out["planning"] = planning_section(bem, torch, not args.no_autotune)
        elif e == "hmatrix":
            out["hmatrix"] = hmatrix_section(bem, torch, not args.no_autotune)
        else:
            raise SystemExit(f"unknown extra workload {e}")
        torch.cuda.empty_cache()
    if not args.no_serving and "serving" not in extras:
        # a bounded serving run: 8 kidney requests arriving at 1/s, at most 4 in
        # flight, continuous batching (request latency p50/p99, solves/s)
        log("serving (bounded)")
        out["serving"] = serving_section(bem, torch, 8, (1.0,), 4)
    if not args.no_solve and not args.no_sphere:
        out["config1"] = config1_section(bem, torch, oracle_leg=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


def sphere_section(args, bem, torch):
    """The 10,242-vertex sphere (k0 = 10, k1 = 10.5, density ratio 1.05): the
    on-the-fly apply with its pair-kernel roofline, the single-layer operator
    alone, GMRES to 1e-5 and 1e-6 without and with OSRC (right- and
    left-preconditioned), and the assembled paths."""
    from bem_inputs import configs, vectors
    prob = configs.config2()
    P, t_setup = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, autotune=not args.no_autotune))
    x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
    y = torch.empty_like(x)
    wall, step_ms, pair_ms = time_applies(P, x, y, args.steps, args.warmup, torch)
    pairs = pairs_per_apply(prob)
    out = {"workload": f"{prob.name}: on-the-fly PMCHWT apply, icosphere {prob.domains[0].n_vertices} v / "
                       f"{prob.domains[0].n_triangles} t, k0=10, k1=10.5, rho1/rho0=1.05",
           "value": pairs * args.steps / wall, "unit": "quad-pair interactions/s",
           "ms_per_step": 1e3 * wall / args.steps, "pairs_per_apply": pairs, "unknowns": prob.n_unknowns,
           "setup_s": t_setup, "pair_launch_shape": list(P.pair_launch_shape()),
           "apply_ms_p50": float(np.percentile(step_ms, 50)), "apply_ms_p99": float(np.percentile(step_ms, 99)),
           "roofline": pair_roofline(pairs, pair_ms, "k_pairs_sphere10242_hbm_traffic.md", "k_pairs_sphere10242_valu.md",
                                     P.pair_launch_shape())}
    log(f"sphere apply {out['ms_per_step']:.2f} ms")
    out["single_layer"] = single_layer_section(P, prob, torch, args.steps, args.warmup)
    if not args.no_solve:
        # GMRES(100) on the on-the-fly operator, plane wave along +z, without and
        # with the OSRC preconditioner (N_Pade = 4, R_eps = 0.1 = radius / 10):
        # right-preconditioned (stops on the true residual) and the paper's
        # left form (stops on the preconditioned residual)
        inc = bem.Incident.plane_waves([[0.0, 0.0, 1.0]])
        b = P.rhs(inc)
        g = {}
        for pname, pc in (("plain", bem.BEM_PRECOND_NONE), ("osrc", bem.BEM_PRECOND_OSRC),
                          ("osrc_left", bem.BEM_PRECOND_OSRC_LEFT)):
            for tol in (1e-5, 1e-6):
                (u, info), ts = _timed(torch, lambda: P.solve(b, bem.solve_options(
                    tol=tol, restart=100, max_iter=400, precond=pc, n_pade=4, r_eps=0.1, theta=np.pi / 3)))
                g[f"{pname}_tol{tol:g}"] = {"time_to_solve_s": ts, "iterations": info[0]["iterations"],
                                            "rel_residual": info[0]["rel_residual"],
                                            "converged": info[0]["converged"]}
        out["gmres"] = g
        out["osrc"] = osrc_apply_ms(P, prob, bem, torch, 4, 0.1)
    P.close()
    P = None
    torch.cuda.empty_cache()
    if not args.no_assembled:
        out["assembled"] = assembled_section(prob, bem, vectors, torch, autotune=not args.no_autotune,
                                             solves=not args.assembled_kernels_only)
    return out


def single_layer_section(P, prob, torch, steps, warmup):
    """The single-layer operator alone, y = V_k0 x on the sphere (exterior pass
    only, M^2 pairs): the one-channel pair kernel, about 21 FLOP and three
    transcendentals per pair, for comparison with the fused multitrace kernel."""
    from bem_inputs import vectors
    nv = sum(d.n_vertices for d in prob.domains)
    x = torch.from_numpy(vectors.random_complex(nv, seed=3)).cuda()
    y = torch.empty_like(x)
    for _ in range(max(1, warmup)):
        P.apply_single_layer(x, out=y)
    torch.cuda.synchronize()
    step_ms, pair_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        P.apply_single_layer(x, out=y)
        tm = P.timings()
        step_ms.append(tm[0])
        pair_ms.append(tm[1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = float(prob.n_points) ** 2
    k_ms = float(np.mean(pair_ms))
    achieved = FLOP_PER_PAIR_V * pairs / (k_ms * 1e-3) / 1e12
    return {"pairs_per_apply": pairs, "value": pairs * steps / wall, "unit": "quad-pair interactions/s",
            "apply_ms_p50": float(np.percentile(step_ms, 50)), "apply_ms_p99": float(np.percentile(step_ms, 99)),
            "kernel": "k_pairs_v", "kernel_ms": k_ms, "kernel_pairs_per_s": pairs / (k_ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "flop_per_pair": FLOP_PER_PAIR_V}}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def config1_section(bem, torch, oracle_leg):
    """The 642-vertex sphere (k0 = 2, k1 = 2.2, plane wave): GPU set-up and
    GMRES(100) to 1e-8, and, in the CPU-baseline leg, the oracle's dense FP64
    assembly and LU on the host cores with the GPU solution's error against it."""
    from bem_inputs import configs
    prob = configs.config1()
    P, t_setup = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, autotune=False))
    b = P.rhs(bem.Incident.plane_waves([[0.0, 0.0, 1.0]]))
    (u, info), t_solve = _timed(torch, lambda: P.solve(b, bem.solve_options(tol=1e-8, restart=100, max_iter=500)))
    u = u[0].cpu().numpy()
    P.close()
    out = {"unknowns": prob.n_unknowns, "gpu_setup_s": t_setup, "gpu_solve_s": t_solve,
           "iterations": info[0]["iterations"], "rel_residual": info[0]["rel_residual"]}
    if oracle_leg:
        import oracle
        t0 = time.perf_counter()
        A = oracle.pmchwt_matrix(prob)
        p, dp = oracle.plane_wave(prob.k0)
        rhs = oracle.rhs(prob, p, dp)
        t1 = time.perf_counter()
        u_ref = oracle.solve_lu(A, rhs)
        t2 = time.perf_counter()
        out["oracle"] = {"assembly_s": t1 - t0, "lu_s": t2 - t1, "cores": int(os.environ.get("OMP_NUM_THREADS") or
                                                                            os.cpu_count() or 1)}
        out["gpu_vs_lu_rel_error"] = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    return out


def ribcage_section(bem, torch, autotune):
    """Rib-cage stack at h = lambda/6 (53,524 vertices, 7 domains): on-the-fly
    apply rate and the OSRC-preconditioned GMRES(100) solve of the 256-piston
    bowl as one field (N_Pade = 8, R_eps = 1.5) to 1e-5."""
    from bem_inputs import configs, pistons
    prob = configs.ribcage(1.0)
    P, t_setup = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, autotune=autotune))
    pairs = pairs_per_apply(prob)
    x = torch.from_numpy(np.random.default_rng(0).standard_normal(prob.n_unknowns) + 0j).cuda()
    y = torch.empty_like(x)
    P.apply(x, out=y)
    ts = []
    for _ in range(3):
        P.apply(x, out=y)
        ts.append(P.timings()[0])
    ms = float(np.median(ts))
    log(f"ribcage apply {ms:.1f} ms")
    c, n, a = pistons.bowl_array()
    inc = bem.Incident.pistons(c, n, a, 1.0, np.zeros(len(c), dtype=int))
    b = P.rhs(inc)
    (u, info), t_solve = _timed(torch, lambda: P.solve(b, bem.solve_options(
        tol=1e-5, restart=100, max_iter=1000, precond=bem.BEM_PRECOND_OSRC, n_pade=8, r_eps=1.5, theta=np.pi / 3)))
    log(f"ribcage OSRC solve {t_solve:.1f} s, {info[0]['iterations']} iterations")
    res = {"vertices": sum(d.n_vertices for d in prob.domains), "unknowns": prob.n_unknowns,
           "domains": len(prob.domains), "setup_s": t_setup, "pair_launch_shape": list(P.pair_launch_shape()),
           "pairs_per_apply": pairs, "apply_ms": ms, "pairs_per_s": pairs / (ms * 1e-3),
           "osrc_solve": {"time_to_solve_s": t_solve, "iterations": info[0]["iterations"],
                          "rel_residual": info[0]["rel_residual"], "converged": info[0]["converged"],
                          "s_per_iteration": t_solve / max(1, info[0]["iterations"])}}
    P.close()
    return res


def gemm_reference(torch):
    """torch.matmul (hipBLASLt / rocBLAS underneath) on the real GEMM of the
    split-BF16 apply at R = 256 (n x 2n times 2n x 2R, one term of the three)
    for the 53,848- and 20,484-unknown matrices, and on square shapes: the rate
    the vendor library reaches on this chip, beside the library's kernels.
    Random operands; median of 5 timed launches (HIP events)."""
    out = {}
    torch.backends.cuda.matmul.allow_tf32 = False
    for (M, K, N) in ((53848, 107712, 512), (20484, 40968, 512), (16384, 16384, 16384), (8192, 8192, 8192)):
        for dt, peak in ((torch.bfloat16, BF16_PEAK_TFLOPS), (torch.float32, FP32_MFMA_PEAK_TFLOPS)):
            if dt == torch.float32 and M * K > 3e9:
                continue
            A = torch.randn(M, K, device="cuda").to(dt)
            B = torch.randn(K, N, device="cuda").to(dt)
            C = A @ B
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                C = A @ B
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            tf = 2.0 * M * K * N / (ms * 1e-3) / 1e12
            key = f"{str(dt).split('.')[-1]}_{M}x{K}x{N}"
            out[key] = {"ms": ms, "TFLOPs": tf, "frac": tf / peak, "peak": peak}
            log(f"torch.matmul {key}: {ms:.3f} ms, {tf:.0f} TFLOP/s, {tf / peak:.3f} of peak")
            del A, B, C
            torch.cuda.empty_cache()
    return out


def ribcage_assembled_section(bem, torch, autotune):
    """Rib-cage stack at h * sqrt(2) (26,924 vertices): assembled split-BF16,
    one right-hand side per piston (R = 256): GEMM rates and time-to-solve of
    split-BF16 FGMRES (to 1e-6), FP32-MFMA FGMRES and plain FP32 GMRES (GEMV)."""
    from bem_inputs import configs, pistons
    prob = configs.ribcage(2.0 ** 0.5)
    n = prob.n_unknowns
    P, t_asm = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, mode=bem.BEM_ASSEMBLED_SPLIT_BF16,
                                                             autotune=autotune))
    log(f"ribcage assembled: n = {n}, assembly {t_asm:.1f} s")
    res = {"vertices": sum(d.n_vertices for d in prob.domains), "unknowns": n, "assembly_s": t_asm}
    X = torch.from_numpy(np.random.default_rng(1).standard_normal((256, n)) + 0j).cuda()
    for kern, key, peak, fl in ((bem.BEM_APPLY_MFMA_SPLIT_BF16, "bf16x3", BF16_PEAK_TFLOPS, 24.0),
                                (bem.BEM_APPLY_MFMA_SPLIT_BF16_W4, "bf16x3_w4", BF16_PEAK_TFLOPS, 24.0),
                                (bem.BEM_APPLY_MFMA_SPLIT_BF16_W8, "bf16x3_w8", BF16_PEAK_TFLOPS, 24.0),
                                (bem.BEM_APPLY_MFMA_FP32, "fp32", FP32_MFMA_PEAK_TFLOPS, 8.0)):
        P.apply(X, kernel=kern)
        ts = []
        for _ in range(3):
            P.apply(X, kernel=kern)
            ts.append(P.timings()[1])
        ms = float(np.median(ts))
        tf = fl * n * n * 256 / (ms * 1e-3) / 1e12
        res[f"gemm_{key}_R256"] = {"ms": ms, "TFLOPs": tf, "frac": tf / peak, "peak": peak}
        log(f"GEMM {key} R=256 {ms:.2f} ms {tf:.0f} TF")
    del X
    c, nn, a = pistons.bowl_array()
    b = P.rhs(bem.Incident.pistons(c, nn, a, 1.0, np.arange(len(c))))
    # flexible forms: all 256 right-hand sides in one block, outer FP64 residual
    # to 1e-6; inner cycles of 200 (the stack needs hundreds of Krylov steps;
    # 200 saves about a tenth of the time against 100)
    for name, prec in (("split_bf16_fgmres", bem.BEM_PREC_SPLIT_BF16_FGMRES),
                       ("fp32_mfma_fgmres", bem.BEM_PREC_FP32_MFMA_FGMRES)):
        (u, info), t = _timed(torch, lambda: P.solve(b, bem.solve_options(
            tol=1e-6, restart=10, max_iter=8, precision=prec, inner_tol=1e-3, inner_restart=200,
            inner_max_iter=1500)))
        res[f"solve_{name}_R256"] = {"tol": 1e-6, "s": t, "outer_iterations_max": int(max(i["iterations"] for i in info)),
                                     "max_rel_residual": float(max(i["rel_residual"] for i in info)),
                                     "all_converged": all(i["converged"] for i in info)}
        log(f"solve {name}: {t:.2f} s")
    # plain FP32 GMRES(100), one GEMV per right-hand side and step: a sample of
    # 8 right-hand sides with a 1000-step budget (time per right-hand side)
    (u, info), t = _timed(torch, lambda: P.solve(b[:8], bem.solve_options(tol=1e-6, restart=100, max_iter=1000,
                                                                          precision=bem.BEM_PREC_FP32)))
    res["solve_plain_fp32_gemv_sample8"] = {"tol": 1e-6, "s": t, "s_per_rhs": t / 8, "iterations_max": int(max(i["iterations"] for i in info)),
                                            "max_rel_residual": float(max(i["rel_residual"] for i in info)),
                                            "all_converged": all(i["converged"] for i in info)}
    log(f"solve plain fp32 (8 rhs): {t:.2f} s")
    P.close()
    return res


def planning_section(bem, torch, autotune):
    """Full matrix capture and excitation planning on the rib-cage stack at
    h * 2 (13.5k vertices): 256 pistons solved as one block (assembled split
    BF16, FGMRES to 1e-5), the total field of every element at the focus and at
    20 points 0.5 below the four central ribs, then phase conjugation and the
    sparing excitation (peak rib-side pressure at most 0.3 of the focal one)."""
    from bem_inputs import configs, pistons
    from paper_1910_01011_amd import planning
    prob = configs.ribcage(2.0)
    P, t_asm = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, mode=bem.BEM_ASSEMBLED_SPLIT_BF16,
                                                             autotune=autotune))
    c, nn, a = pistons.bowl_array()
    spare = np.array([[x, y, -5.4] for x in (-4.5, -1.5, 1.5, 4.5) for y in (-2.0, -1.0, 0.0, 1.0, 2.0)])
    opts = bem.solve_options(tol=1e-5, restart=10, max_iter=8, precision=bem.BEM_PREC_SPLIT_BF16_FGMRES,
                             inner_tol=1e-3, inner_restart=200, inner_max_iter=1500)
    res = planning.plan(P, c, nn, a, np.zeros(3), spare, 0.3, opts)
    P.close()
    info = res["solve_info"]
    out = {"vertices": sum(d.n_vertices for d in prob.domains), "unknowns": prob.n_unknowns, "elements": len(c),
           "assembly_s": t_asm, "capture_s": res["capture_s"], "solve_s": res["solve_s"], "field_s": res["field_s"],
           "optimise_s": res["optimise_s"],
           "all_converged": all(i["converged"] for i in info),
           "max_rel_residual": float(max(i["rel_residual"] for i in info)),
           "phase_conjugation": {k: v for k, v in res["phase_conjugation"].items() if k != "a"},
           "sparing": {k: v for k, v in res["sparing"].items() if k != "a"}}
    log(f"planning: capture {res['capture_s']:.1f} s, ratio pc {out['phase_conjugation']['ratio']:.3f} "
        f"sparing {out['sparing']['ratio']:.3f}")
    return out


def hmatrix_section(bem, torch, autotune):
    """Hierarchical matrix (ACA, eps 1e-4, leaves of 64 vertices, eta 2): on the
    10,242-vertex sphere against the dense complex64 matrix (storage, apply
    time, difference, GMRES to 1e-5), and on the 53.5k-vertex rib-cage stack
    against the on-the-fly operator (OSRC GMRES to 1e-5 with the compressed
    operator; the on-the-fly residual of its solution)."""
    from bem_inputs import configs, pistons, vectors
    out = {}
    prob = configs.config2()
    P = bem.Problem.from_config(prob, device=True, mode=bem.BEM_ASSEMBLED_FP32, autotune=autotune)
    x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
    yd = P.apply(x, kernel=bem.BEM_APPLY_GEMV)
    info = P.hmatrix_build(eps=1e-4, leaf_vertices=64, eta=2.0)
    yh = P.apply(x, kernel=bem.BEM_APPLY_HMATRIX)
    ts_h, ts_d = [], []
    for _ in range(10):
        P.apply(x, out=yh, kernel=bem.BEM_APPLY_HMATRIX)
        ts_h.append(P.timings()[0])
        P.apply(x, out=yd, kernel=bem.BEM_APPLY_GEMV)
        ts_d.append(P.timings()[0])
    b = P.rhs(bem.Incident.plane_waves([[0.0, 0.0, 1.0]]))
    (ud, i_d), t_d = _timed(torch, lambda: P.solve(b, bem.solve_options(tol=1e-5, restart=100, max_iter=400)))
    (uh, i_h), t_h = _timed(torch, lambda: P.solve(b, bem.solve_options(tol=1e-5, restart=100, max_iter=400,
                                                                        precision=bem.BEM_PREC_HMATRIX)))
    r = P.apply(uh[0].contiguous(), kernel=bem.BEM_APPLY_GEMV) - b[0]
    out["sphere10242"] = {"info": info, "apply_ms": float(np.median(ts_h)), "gemv_ms": float(np.median(ts_d)),
                          "rel_diff_to_dense": float((yh - yd).norm() / yd.norm()),
                          "gmres_dense_s": t_d, "gmres_hmatrix_s": t_h, "iterations": [i_d[0]["iterations"],
                                                                                          i_h[0]["iterations"]],
                          "dense_residual_of_h_solution": float(r.norm() / b[0].norm())}
    log(f"hmatrix sphere: {info['bytes'] / 1e6:.0f} MB of {info['dense_bytes'] / 1e6:.0f} MB, "
        f"apply {np.median(ts_h):.3f} ms vs GEMV {np.median(ts_d):.3f} ms")
    P.close()
    torch.cuda.empty_cache()
    prob = configs.ribcage(1.0)
    P, t_setup = _timed(torch, lambda: bem.Problem.from_config(prob, device=True, autotune=autotune))
    x = torch.from_numpy(vectors.random_complex(prob.n_unknowns, seed=0)).cuda()
    yo = P.apply(x)
    info, t_build = _timed(torch, lambda: P.hmatrix_build(eps=1e-4, leaf_vertices=64, eta=2.0))
    yh = P.apply(x, kernel=bem.BEM_APPLY_HMATRIX)
    ts = []
    for _ in range(5):
        P.apply(x, out=yh, kernel=bem.BEM_APPLY_HMATRIX)
        ts.append(P.timings()[0])
    c, nn, a = pistons.bowl_array()
    b = P.rhs(bem.Incident.pistons(c, nn, a, 1.0, np.zeros(len(c), dtype=int)))
    opts = bem.solve_options(tol=1e-5, restart=100, max_iter=1000, precond=bem.BEM_PRECOND_OSRC, n_pade=8, r_eps=1.5,
                             theta=np.pi / 3, precision=bem.BEM_PREC_HMATRIX)
    (u, info_s), t_solve = _timed(torch, lambda: P.solve(b, opts))
    r = P.apply(u[0].contiguous()) - b[0]
    # flexible form: outer residual on the on-the-fly operator, inner OSRC GMRES
    # on the compressed one
    fopts = bem.solve_options(tol=1e-5, restart=10, max_iter=10, precond=bem.BEM_PRECOND_OSRC, n_pade=8, r_eps=1.5,
                              theta=np.pi / 3, precision=bem.BEM_PREC_HMATRIX_FGMRES, inner_tol=1e-3,
                              inner_restart=200, inner_max_iter=1000)
    (uf, info_f), t_f = _timed(torch, lambda: P.solve(b, fopts))
    out["ribcage53524"] = {"info": info, "setup_s": t_setup, "build_s": t_build, "apply_ms": float(np.median(ts)),
                           "rel_diff_to_on_the_fly": float((yh - yo).norm() / yo.norm()),
                           "osrc_gmres_hmatrix": {"time_to_solve_s": t_solve, **info_s[0]},
                           "on_the_fly_residual_of_solution": float(r.norm() / b[0].norm()),
                           "osrc_fgmres_hmatrix_inner": {"time_to_solve_s": t_f, **info_f[0],
                                                         "note": "rel_residual is the on-the-fly operator's"}}
    log(f"hmatrix ribcage: {info['bytes'] / 1e9:.1f} GB of {info['dense_bytes'] / 1e9:.1f} GB, build {t_build:.1f} s, "
        f"apply {np.median(ts):.2f} ms, OSRC GMRES {t_solve:.1f} s, {info_s[0]['iterations']} iterations; "
        f"FGMRES {t_f:.1f} s, residual {info_f[0]['rel_residual']:.2e}")
    P.close()
    return out


def serving_section(bem, torch, n_requests, rates=(2.0, 10.0), max_inflight=4):
    """Kidney + fat-shell request stream: Poisson arrivals at each rate, 2k-40k
    vertices, 1-64 pistons per request, continuous batching of the requests in
    flight; p50/p99 latency (arrival to result on the host), solves/s and the
    batch's launch statistics."""
    from bem_inputs import configs
    from paper_1910_01011_amd import serving
    free, _ = torch.cuda.mem_get_info()
    out = {}
    for rate in rates:
        items = configs.serving_stream(rate, n_requests, 5000 + int(round(100 * rate)),
                                       6000 + int(round(100 * rate)))
        reqs = serving.requests_from_stream(items, free)
        srv = serving.Server(max_inflight=max_inflight, on_result=lambda r, rate=rate: log(
            f"serving rate {rate:g}: request {r.rid} done, latency {r.latency:.2f} s"))
        res = srv.run(reqs)
        summ = serving.summarize(res)
        summ["batch"] = srv.last_batch_stats
        summ["vertices"] = [int(sum(d.n_vertices for d in r.domains)) for r in reqs]
        summ["modes"] = [int(r.mode) for r in reqs]
        summ["rhs_per_request"] = [int(r.incident.n_fields) for r in reqs]
        summ["max_inflight"] = max_inflight
        out[f"rate_{rate:g}_per_s"] = summ
        log(f"serving rate {rate}: p50 {summ['p50_latency_s']:.2f} s p99 {summ['p99_latency_s']:.2f} s, "
            f"{summ['requests_per_s']:.2f} requests/s, batch {srv.last_batch_stats}")
    return out



def paper_sphere_section(bem, torch):
    """The paper's single-sphere model problem: 1 cm sphere at 1 MHz in water,
    fat, the table's rib material or the cortical-like bone of impedance ratio
    5.2 (attenuating media), plane wave, OSRC
    (N_Pade = 4, R_eps = 5e-4 m) GMRES(100) to 1e-5; iterations and time per
    iteration against mesh density (the field error against the series
    solution is checked in the GPU tests)."""
    from bem_inputs import configs
    out = {}
    for material in ("fat", "ribs", "cortical"):
        for epw in (4, 6, 8, 10):
            prob = configs.paper_sphere(material, epw)
            (P, t_setup) = _timed(torch, lambda: bem.Problem.from_config(prob, device=True))
            b = P.rhs(bem.Incident.plane_waves([[0.0, 0.0, 1.0]]))
            (u, info), t = _timed(torch, lambda: P.solve(b, bem.solve_options(
                tol=1e-5, restart=100, max_iter=400, precond=bem.BEM_PRECOND_OSRC, n_pade=4,
                r_eps=prob.meta["r_eps"], theta=np.pi / 3)))
            it = info[0]["iterations"]
            out[f"{material}_e{epw}"] = {"vertices": prob.domains[0].n_vertices, "setup_s": t_setup,
                                         "iterations": it, "time_to_solve_s": t,
                                         "s_per_iteration": t / max(1, it), "rel_residual": info[0]["rel_residual"],
                                         "converged": info[0]["converged"]}
            log(f"paper sphere {material} e={epw}: {prob.domains[0].n_vertices} v, {it} it, {t:.2f} s")
            P.close()
    return out

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


BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 MFMA
HBM_PEAK_GBPS = 8000.0


def assembled_section(prob, bem, vectors, torch, autotune=True, solves=True):
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
    # the PMCHWT matrix is complex-symmetric up to a row swap and a sign, so
    # 4 n^2 bytes are its unique entries: the rate against that minimum too
    res["gemv"] = {"ms": ms, "GBps": gbps, "frac_hbm": gbps / HBM_PEAK_GBPS, "bytes": 8.0 * n * n,
                   "unique_bytes": 4.0 * n * n, "unique_GBps": gbps / 2, "frac_hbm_unique": gbps / 2 / HBM_PEAK_GBPS}
    for R in (64, 256):
        X = torch.from_numpy(vectors.random_complex(n, seed=1, n_rhs=R)).cuda()
        for kern, key, peak, fl in ((bem.BEM_APPLY_MFMA_SPLIT_BF16, "bf16x3", BF16_PEAK_TFLOPS, 24.0),
                                    (bem.BEM_APPLY_MFMA_SPLIT_BF16_W4, "bf16x3_w4", BF16_PEAK_TFLOPS, 24.0),
                                    (bem.BEM_APPLY_MFMA_SPLIT_BF16_W8, "bf16x3_w8", BF16_PEAK_TFLOPS, 24.0),
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
            if R == 64:
                # one 128-column block of X': the matrix (BF16 hi/lo planes or the
                # FP32 real view, 8 n^2 bytes either way) is streamed once, so
                # this size is bound by HBM
                gbs = 8.0 * n * n / (ms * 1e-3) / 1e9
                res[f"gemm_{key}_R{R}"].update({"matrix_bytes": 8.0 * n * n, "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBPS})
    if not solves:
        return res
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
