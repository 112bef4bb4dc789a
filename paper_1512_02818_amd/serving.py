"""Load driver of the serving loop: replays a seeded Poisson stream of
node-solve requests (workloads.serving_stream) against a pdd.Server at
their arrival times, then reports the server's counters and latency
percentiles. Every solve runs in the native server thread and the HIP
kernels; this module only creates problems and grids and submits.

    python -m paper_1512_02818_amd.serving --rate 200 --duration 5 --drain 20
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import pdd
from . import workloads as W


class Fixtures:
    """Device problems and u_prev / residual grids of a request stream (one
    grid pair per problem and grid size, shared by its requests)."""

    def __init__(self, ctx, problems, requests, precision="fp32"):
        import torch
        self.problems = [pdd.Problem(ctx, pd) for pd in problems]
        self.grids = {}
        dt = np.float32 if precision == "fp32" else np.float64
        for r in requests:
            key = (r["problem"], r["grid_n"])
            if r["cv"] and key not in self.grids:
                gu, gr, _ = W.correction_grids(problems[r["problem"]], n=r["grid_n"], seed=r["problem"] + 1,
                                               dtype=dt)
                self.grids[key] = (gu, torch.as_tensor(gu["data"]).cuda().contiguous(),
                                   gr, torch.as_tensor(gr["data"]).cuda().contiguous())
        torch.cuda.synchronize()

    def submit(self, server, r, precision="fp32"):
        kw = {}
        if r["cv"]:
            gu, tu, gr, tr = self.grids[(r["problem"], r["grid_n"])]
            kw = dict(u_prev=gu, u_prev_t=tu, resid=gr, resid_t=tr)
        return server.submit(self.problems[r["problem"]], r["nodes"], r["dt"], r["target_se"],
                             precision=precision, stream_id=r["stream_id"], tag=r["stream_id"], **kw)

    def close(self):
        for p in self.problems:
            p.close()


def run_stream(ctx, problems, requests, drain_s=20.0, server_opts=None, precision="fp32",
               fixtures=None, log=None):
    """Submits `requests` at their arrival times (seconds from the start),
    waits up to drain_s after the last arrival, then stops the server
    (cancelling what is left). Returns (report dict, {stream_id: completion})."""
    fx = fixtures or Fixtures(ctx, problems, requests, precision)
    server = pdd.Server(ctx, **(server_opts or {}))
    shed = 0
    by_id = {}
    t0 = time.perf_counter()
    for r in requests:
        delay = r["t"] - (time.perf_counter() - t0)
        if delay > 0:
            server.poll(wait_ms=0)
            time.sleep(delay)
        try:
            by_id[fx.submit(server, r, precision)] = r["stream_id"]
        except pdd.PDDError as e:
            if e.status not in (-5, -2):  # shed by the queue limit or the memory budget
                raise
            shed += 1
    t_last = time.perf_counter()
    deadline = t_last + drain_s
    t_log = t_last
    while server.pending and time.perf_counter() < deadline:
        server.poll(wait_ms=50)
        if log and time.perf_counter() - t_log > 2.0:
            t_log = time.perf_counter()
            log(f"completed {len(server.results)} / {len(by_id)}")
    rep = server.report()
    rep["offered_requests"] = len(requests)
    rep["offered_rate_per_s"] = len(requests) / max(requests[-1]["t"], 1e-9) if requests else 0.0
    rep["shed_at_submit"] = shed
    rep["cancelled"] = len(server.pending)
    rep["arrival_window_s"] = t_last - t0
    rep["drain_s"] = time.perf_counter() - t_last
    done = {by_id[i]: c for i, c in server.results.items()}
    server.close()
    if fixtures is None:
        fx.close()
    return rep, done


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--drain", type=float, default=20.0)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--cv-frac", type=float, default=0.3)
    ap.add_argument("--tols", default="1e-2,3e-3,1e-3")
    ap.add_argument("--epoch-paths", type=int, default=1 << 24)
    ap.add_argument("--chunk-paths", type=int, default=1 << 22)
    ap.add_argument("--pipeline", type=int, default=0, help="epochs in flight at once (0 = the library's 2)")
    args = ap.parse_args(argv)
    problems, reqs = W.serving_stream(seed=args.seed, rate=args.rate, duration=args.duration,
                                      cv_frac=args.cv_frac,
                                      tols=tuple(float(t) for t in args.tols.split(",")))
    ctx = pdd.Context(0)
    rep, _ = run_stream(ctx, problems, reqs, drain_s=args.drain,
                        server_opts=dict(epoch_paths=args.epoch_paths, chunk_paths=args.chunk_paths,
                                         pipeline=args.pipeline),
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(rep), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
