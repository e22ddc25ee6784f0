"""Serving loop: continuous batching of solve requests on one GPU.

Requests (a transmission problem, an incident field with one or more right-
hand sides, solver options) arrive over time.  The loop admits a waiting
request as soon as a slot is free and its device footprint
(``bem_footprint_bytes``: geometry, singular correction, dense matrix in the
assembled modes, Krylov bases) fits in the HBM budget next to the requests
already running.  Every admitted request runs on its own HIP stream in a
worker thread: set-up, right-hand side and GMRES stay on the device (operators
and Krylov state are device resident; device memory is stream-ordered; the C
calls release the Python lock).  Its problem is attached to the server's
``bem_batch``: the operator applies of all requests inside a solve are
gathered step by step and launched together (the on-the-fly pair kernels of
all requests as one grouped launch over their ragged work lists).  Finished
requests free their memory, which admits the next ones.

Each request's computation is its own (own problem handle and stream, the same
per-request work items, launch shapes and summation orders whatever the mix,
no reductions across requests), so its result is bitwise the same alone and in
a mix.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (BEM_OTF, BEM_PREC_FP32, Batch, Incident, Problem, bem_assemble_opts, _L, _domains, _check,
               solve_options)
import ctypes


@dataclass
class Request:
    rid: int
    domains: list
    k0: complex
    incident: Incident
    rho0: float = 1.0
    mode: int = BEM_OTF
    precision: int = BEM_PREC_FP32
    tol: float = 1e-5
    restart: int = 100
    max_iter: int = 400
    arrival: float = 0.0        # seconds after the start of the stream


@dataclass
class Result:
    rid: int
    u: np.ndarray
    info: list
    arrival: float
    admitted: float
    finished: float
    footprint: int
    n_rhs: int
    extra: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def choose_mode(n_vertices: int, n_rhs: int, free_bytes: int):
    """Operator mode and solver precision of a request.

    On the fly (FP32 GMRES) only when the dense complex64 matrix (8 (2 N_V)^2
    bytes) would take more than a quarter of the free HBM: an on-the-fly apply
    re-evaluates every quadrature pair, which costs far more than reading the
    dense matrix once the matrix is built.  Otherwise assembled: FP32 GMRES with
    one GEMV per right-hand side for one or two right-hand sides, else
    split-BF16 block GMRES inside FP64-residual FGMRES (one GEMM per step for
    the whole block).
    """
    from . import BEM_ASSEMBLED_FP32, BEM_ASSEMBLED_SPLIT_BF16, BEM_PREC_SPLIT_BF16_FGMRES
    if 32 * n_vertices ** 2 > 0.25 * free_bytes:
        return BEM_OTF, BEM_PREC_FP32
    if n_rhs <= 2:
        return BEM_ASSEMBLED_FP32, BEM_PREC_FP32
    return BEM_ASSEMBLED_SPLIT_BF16, BEM_PREC_SPLIT_BF16_FGMRES


def requests_from_stream(items, free_bytes: int, tol: float = 1e-5) -> list[Request]:
    """Requests from generated stream items (problem, piston geometry, arrival):
    one right-hand side per piston, mode from ``choose_mode``."""
    out = []
    for rid, it in enumerate(items):
        prob = it["problem"]
        c, n = it["piston_centres"], it["piston_normals"]
        R = len(c)
        inc = Incident.pistons(c, n, it["piston_radius"], 1.0, np.arange(R))
        mode, prec = choose_mode(sum(d.n_vertices for d in prob.domains), R, free_bytes)
        flexible = prec != BEM_PREC_FP32
        out.append(Request(rid, prob.domains, prob.k0, inc, rho0=prob.rho0, mode=mode, precision=prec, tol=tol,
                           restart=30 if flexible else 100, max_iter=400, arrival=it["arrival"]))
    return out


def footprint(req: Request) -> int:
    arr, keep = _domains(req.domains)
    opts = bem_assemble_opts()
    opts.mode = req.mode
    out = ctypes.c_uint64(0)
    _check(_L.bem_footprint_bytes(arr, len(req.domains), ctypes.byref(opts), req.incident.n_fields,
                                  req.restart, ctypes.byref(out)))
    return int(out.value)


def run_request(req: Request, t0: float, admitted: float, fp: int, batch: Batch | None = None) -> Result:
    """Set up, build the right-hand sides and solve one request on its own
    stream; with a batch, the solve's operator applies go through it."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ta = time.perf_counter()
        P = Problem(req.domains, req.k0, req.rho0, device=True, mode=req.mode, stream=stream.cuda_stream)
        if batch is not None:
            batch.attach(P)
        b = P.rhs(req.incident)
        stream.synchronize()
        tb = time.perf_counter()
        u, info = P.solve(b, solve_options(tol=req.tol, restart=req.restart, max_iter=req.max_iter,
                                           precision=req.precision))
        u_host = u.cpu().numpy()
        stream.synchronize()
        tc = time.perf_counter()
        P.close()
    extra = {"setup_s": tb - ta, "solve_s": tc - tb, "iterations": int(max(i["iterations"] for i in info))}
    return Result(req.rid, u_host, info, req.arrival, admitted, time.perf_counter() - t0, fp,
                  req.incident.n_fields, extra)


class Server:
    """Admission by HBM footprint, bounded concurrency, one stream per request,
    operator applies batched across the requests in flight (``batching``)."""

    def __init__(self, hbm_budget_bytes: int | None = None, max_inflight: int = 4, headroom_bytes: int = 16 << 30,
                 batching: bool = True, batch_window_s: float | None = None, on_result=None):
        if hbm_budget_bytes is None:
            free, _total = torch.cuda.mem_get_info()
            hbm_budget_bytes = max(0, free - headroom_bytes)
        self.budget = int(hbm_budget_bytes)
        self.max_inflight = int(max_inflight)
        self.batching = bool(batching)
        self.batch_window_s = batch_window_s
        self.on_result = on_result   # called with each Result as it completes (progress reporting)
        self.last_batch_stats: dict = {}

    def run(self, requests: list[Request]) -> list[Result]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        fps = {r.rid: footprint(r) for r in reqs}
        for r in reqs:
            if fps[r.rid] > self.budget:
                raise MemoryError(f"request {r.rid} needs {fps[r.rid]} bytes, over the budget {self.budget}")
        results: list[Result] = []
        lock = threading.Lock()
        done_evt = threading.Event()
        inflight: dict[int, int] = {}
        used = [0]

        errors: list[BaseException] = []

        def finished(fut, rid):
            with lock:
                used[0] -= inflight.pop(rid)
                exc = fut.exception()
                if exc is not None:
                    errors.append(exc)
                else:
                    results.append(fut.result())
            if exc is None and self.on_result is not None:
                self.on_result(fut.result())
            done_evt.set()

        batch = Batch(torch.cuda.current_device()) if self.batching else None
        if batch is not None and self.batch_window_s is not None:
            batch.set_window(self.batch_window_s)
        t0 = time.perf_counter()
        pending: list[Request] = []
        nxt = 0
        with ThreadPoolExecutor(max_workers=self.max_inflight) as pool:
            while nxt < len(reqs) or pending or inflight:
                now = time.perf_counter() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                # first-come first-served admission while slots and memory allow
                with lock:
                    while pending and len(inflight) < self.max_inflight and used[0] + fps[pending[0].rid] <= self.budget:
                        r = pending.pop(0)
                        inflight[r.rid] = fps[r.rid]
                        used[0] += fps[r.rid]
                        fut = pool.submit(run_request, r, t0, time.perf_counter() - t0, fps[r.rid], batch)
                        fut.add_done_callback(lambda f, rid=r.rid: finished(f, rid))
                # sleep until the next arrival or a completion
                wait = 0.05
                if nxt < len(reqs):
                    wait = max(0.0, min(wait, reqs[nxt].arrival - (time.perf_counter() - t0)))
                done_evt.wait(timeout=wait)
                done_evt.clear()
                if errors:
                    break
        if batch is not None:
            self.last_batch_stats = batch.stats()
            batch.close()
        if errors:
            raise errors[0]
        return sorted(results, key=lambda r: r.rid)


def summarize(results: list[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    makespan = max(r.finished for r in results) - min(r.arrival for r in results)
    n_rhs = sum(r.n_rhs for r in results)
    return {"requests": len(results), "rhs": n_rhs, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "makespan_s": float(makespan), "requests_per_s": len(results) / makespan,
            "solves_per_s": n_rhs / makespan,
            "all_converged": all(all(i["converged"] for i in r.info) for r in results),
            "setup_s": [round(r.extra.get("setup_s", 0.0), 3) for r in results],
            "solve_s": [round(r.extra.get("solve_s", 0.0), 3) for r in results],
            "iterations": [r.extra.get("iterations", 0) for r in results],
            "queue_s": [round(r.admitted - r.arrival, 3) for r in results]}
