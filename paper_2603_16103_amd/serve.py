"""Continuous-batching simplification server on one GPU.

Requests (a scene in the stored 3DGS form, a target ratio, k and a draw
seed) arrive at any time.  The server admits a request when its splats fit
in the HBM budget, copies its input to the device on a copy stream (so the
copy overlaps the passes of the jobs already running), and submits it to a
``nanogs.Batch``: the job joins the working set at the next pass boundary,
every pass runs all live jobs with one launch per stage, and a job leaves
the working set as soon as it reaches its target.  Finished results are
copied back on the copy stream; a request's latency is the time from its
arrival to the end of that copy.

``PlainServer`` runs the same trace one job at a time through
``nanogs_simplify`` (the baseline the batched server is compared with).

Admission by footprint: the working set holds at most ``rows`` splats, and
each admitted job also holds its device input and output buffers; ``rows``
is the largest count for which the engine workspace plus those buffers fit
in the budget.

Command line: ``python -m paper_2603_16103_amd.serve --duration 120 --rate 20``
replays a Poisson trace (scene sizes log-uniform in [1e4, 4e6], targets from
{0.5, 0.1, 0.01}, k from {16, 24}) through both servers and prints one JSON
line with throughput and p50/p99 latency of each.  By default every request
carries its own scene, drawn on the device from seed 20000 + request id when
it is admitted (synth.gen_scene_device; the draw takes the place of the
host-to-device copy of a client's upload); ``--scenes pool`` instead reuses a
pool of host scenes copied in over PCIe.  The HBM budget defaults to the
device's free memory minus a 16 GiB reserve.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass, field

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2603_16103_amd import nanogs as ng  # noqa: E402
from paper_2603_16103_amd.synth import gen_scene, gen_scene_device, serving_trace  # noqa: E402

IO_BYTES_PER_SPLAT = 4 * (3 + 3 + 4 + 1 + 48)  # stored form, one copy


@dataclass
class Request:
    rid: int
    t_arrival: float     # seconds from the start of the replay
    scene: object        # synth.Scene (host, float32), or None: drawn on the device
    target: int
    k: int
    seed: int
    scene_seed: int = -1  # device-drawn scene: its seed
    size: int = 0         # device-drawn scene: its splat count
    # filled by the server
    t_admit: float = -1.0
    t_done: float = -1.0
    n_out: int = 0
    result: tuple = field(default=None, repr=False)  # host arrays when kept

    @property
    def n(self) -> int:
        return self.scene.n if self.scene is not None else self.size


def _pin(a: np.ndarray):
    import torch
    t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
    t.numpy()[...] = a
    return t


class _HostScene:
    """A scene's stored-form arrays in page-locked host memory."""

    def __init__(self, scene):
        self.n = scene.n
        self.arrays = [_pin(np.ascontiguousarray(x)) for x in
                       (scene.pos, scene.log_scale, scene.rot, scene.opacity, scene.sh)]


def max_engine_rows(max_k: int) -> int:
    """Largest working set the library accepts for kNN size max_k: the round
    engine keeps two int32 adjacency entries per edge and at most
    rows * max_k edges per pass, so 2 * rows * max_k < 2^31."""
    return ((1 << 31) - 2) // (2 * max_k)


def rows_for_budget(hbm_budget: int, max_k: int, max_jobs: int) -> int:
    """Largest working-set size whose workspace plus the input/output
    buffers of that many admitted splats fit in hbm_budget bytes, clamped to
    the largest working set the library accepts."""
    probe = 1 << 20
    per_row = ng.batch_workspace_bytes(probe, max_k, max_jobs) / probe + 2 * IO_BYTES_PER_SPLAT
    rows = min(int(hbm_budget / per_row), max_engine_rows(max_k))
    while rows > 2 and (ng.batch_workspace_bytes(rows, max_k, max_jobs)
                        + 2 * IO_BYTES_PER_SPLAT * rows > hbm_budget):
        rows = int(rows * 0.98)
    return max(rows, 2)


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


class BatchServer:
    """Continuous batching over one nanogs.Batch (see the module doc)."""

    def __init__(self, hbm_budget: int, max_k: int = 24, max_jobs: int = 64,
                 opts=None, keep_results: bool = False):
        import torch
        self.torch = torch
        self.rows = rows_for_budget(hbm_budget, max_k, max_jobs)
        self.max_k = max_k
        self.batch = ng.Batch(self.rows, max_k, max_jobs, opts)
        self.compute = torch.cuda.current_stream()
        self.copy = torch.cuda.Stream()
        self.keep_results = keep_results
        self.rows_admitted = 0
        self.max_rows_seen = 0
        self.steps = 0
        self.rejected = 0

    def _admit(self, req: Request, host: _HostScene, t0: float):
        torch = self.torch
        g = ng.GaussianTensors.empty(req.n)
        out = ng.GaussianTensors.empty(req.n)
        dev = (g.pos, g.log_scale, g.rot, g.opacity, g.sh)
        with torch.cuda.stream(self.copy):
            if host is None:
                gen_scene_device(req.n, req.scene_seed, out=dev, stream=self.copy)
            else:
                for d, h in zip(dev, host.arrays):
                    d.copy_(h, non_blocking=True)
        for d in dev:
            d.record_stream(self.copy)
        ev = torch.cuda.Event()
        ev.record(self.copy)
        self.compute.wait_event(ev)  # the job's set-up runs after its copy
        jid = self.batch.submit(g, req.target, k=req.k, seed=req.seed, out=out)
        req.t_admit = time.perf_counter() - t0
        self.rows_admitted += req.n
        return jid, out

    def _collect(self, jid: int, req: Request, out):
        torch = self.torch
        _, n_out, _ = self.batch.job(jid)
        req.n_out = n_out
        res = out.slice(n_out)
        self.copy.wait_stream(self.compute)
        with torch.cuda.stream(self.copy):
            host = [torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
                    for x in (res.pos, res.log_scale, res.rot, res.opacity, res.sh)]
            for h, x in zip(host, (res.pos, res.log_scale, res.rot, res.opacity, res.sh)):
                h.copy_(x, non_blocking=True)
        for x in (out.pos, out.log_scale, out.rot, out.opacity, out.sh):
            x.record_stream(self.copy)
        ev = torch.cuda.Event()
        ev.record(self.copy)
        return ev, host

    def serve(self, requests, hosts, log=None):
        """Replays `requests` (sorted by arrival) in real time; returns the
        report dict.  hosts[i] is the _HostScene of requests[i]."""
        t0 = time.perf_counter()
        pending = []       # arrived, not admitted (FIFO)
        running = {}       # jid -> (req, out)
        draining = []      # (event, req, host arrays)
        nxt = 0
        done = 0
        total = len(requests)
        while done < total:
            now = time.perf_counter() - t0
            while nxt < total and requests[nxt].t_arrival <= now:
                if requests[nxt].n > self.rows:  # can never fit: rejected
                    requests[nxt].t_done = -1.0
                    self.rejected += 1
                    done += 1
                else:
                    pending.append(nxt)
                nxt += 1
            # admission by footprint, first come first served
            while pending and self.rows_admitted + requests[pending[0]].n <= self.rows:
                i = pending.pop(0)
                jid, out = self._admit(requests[i], hosts[i], t0)
                running[jid] = (requests[i], out)
            if running:
                self.batch.step()
                self.steps += 1
                self.max_rows_seen = max(self.max_rows_seen, self.batch.rows_in_use())
                for jid in list(running):
                    state = self.batch.job(jid)[0]
                    if state == ng.JOB_DONE or state < 0:
                        req, out = running.pop(jid)
                        self.rows_admitted -= req.n
                        if state < 0:
                            raise ng.NanoGSError(-state, f"request {req.rid} failed")
                        ev, host = self._collect(jid, req, out)
                        draining.append((ev, req, host))
                        self.batch.release(jid)
            elif not draining and nxt < total:
                time.sleep(max(0.0, min(0.01, requests[nxt].t_arrival - now)))
            still = []
            for ev, req, host in draining:
                if ev.query():
                    req.t_done = time.perf_counter() - t0
                    if self.keep_results:
                        req.result = tuple(h.numpy() for h in host)
                    done += 1
                    if log and done % 50 == 0:
                        log(f"batched: {done}/{total} done")
                else:
                    still.append((ev, req, host))
            draining = still
            if not running and draining:
                draining[0][0].synchronize()
        return report(requests, "batched", extra={"rows": self.rows, "steps": self.steps,
                                                  "max_rows_in_use": self.max_rows_seen,
                                                  "rejected": self.rejected})


class PlainServer:
    """The same trace, one job at a time through nanogs_simplify."""

    def __init__(self, max_n: int, max_k: int = 24, opts=None, keep_results: bool = False):
        import torch
        self.torch = torch
        self.sims = {}
        self.max_n = max_n
        self.opts = opts
        self.keep_results = keep_results

    def _sim(self, k):
        if k not in self.sims:
            self.sims[k] = ng.Simplifier(self.max_n, k, self.opts)
        return self.sims[k]

    def serve(self, requests, hosts, log=None):
        torch = self.torch
        t0 = time.perf_counter()
        for i, req in enumerate(requests):
            now = time.perf_counter() - t0
            if req.t_arrival > now:
                time.sleep(req.t_arrival - now)
            req.t_admit = time.perf_counter() - t0
            g = ng.GaussianTensors.empty(req.n)
            dev = (g.pos, g.log_scale, g.rot, g.opacity, g.sh)
            if hosts[i] is None:
                gen_scene_device(req.n, req.scene_seed, out=dev)
            else:
                for d, h in zip(dev, hosts[i].arrays):
                    d.copy_(h, non_blocking=True)
            out = ng.GaussianTensors.empty(req.n)
            sim = self._sim(req.k)
            sim.opts.seed = req.seed
            n_out = sim(g, req.target, out)
            res = out.slice(n_out)
            host = [x.cpu() for x in (res.pos, res.log_scale, res.rot, res.opacity, res.sh)]
            torch.cuda.synchronize()
            req.n_out = n_out
            req.t_done = time.perf_counter() - t0
            if self.keep_results:
                req.result = tuple(h.numpy() for h in host)
            if log and (i + 1) % 50 == 0:
                log(f"plain: {i + 1}/{len(requests)} done")
        return report(requests, "plain")


def report(requests, name, extra=None):
    served = [r for r in requests if r.t_done >= 0]
    lat = [r.t_done - r.t_arrival for r in served]
    p50, p99 = _percentiles(lat)
    first = min(r.t_arrival for r in requests)
    last = max([r.t_done for r in served] + [first])
    n_in = sum(r.n for r in served)
    out = {"server": name, "requests": len(requests), "served": len(served), "splats_in": n_in,
           "span_s": round(last - first, 3),
           "throughput_splats_per_s": round(n_in / max(last - first, 1e-9), 1),
           "latency_p50_s": round(p50, 4) if p50 is not None else None,
           "latency_p99_s": round(p99, 4) if p99 is not None else None}
    if extra:
        out.update(extra)
    return out


def make_trace(rate: float, duration: float, seed: int, lo: float, hi: float,
               pool_size: int, ks=(16, 24), ratios=(0.5, 0.1, 0.01)):
    """Poisson arrivals with log-uniform sizes; scenes come from a pool of
    `pool_size` generated scenes whose sizes follow the same distribution
    (a request takes the pool scene nearest to its drawn size), so a long
    trace does not need one generated scene per request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pool_n = sorted(int(round(math.exp(x))) for x in
                    rng.uniform(math.log(lo), math.log(hi), pool_size))
    pool = [gen_scene(n, 30000 + i, n_planes=int(rng.integers(2, 9)),
                      n_spheres=int(rng.integers(0, 5))) for i, n in enumerate(pool_n)]
    reqs, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        j = int(np.argmin([abs(p - n) for p in pool_n]))
        ratio = float(rng.choice(list(ratios)))
        k = int(rng.choice(list(ks)))
        sc = pool[j]
        reqs.append(Request(rid, t, sc, max(int(math.ceil(ratio * sc.n)), 1), k,
                            seed=1000003 * rid + 7))
        rid += 1
    return reqs, pool


def make_device_trace(rate: float, duration: float, seed: int):
    """Poisson arrivals of synth.serving_trace, each request with its own
    scene (seed 20000 + request id) drawn on the device at admission."""
    reqs = []
    for rid, (t, n, sseed, ratio, k) in enumerate(serving_trace(rate, duration, seed)):
        reqs.append(Request(rid, t, None, max(int(math.ceil(ratio * n)), 1), k,
                            seed=1000003 * rid + 7, scene_seed=sseed, size=n))
    return reqs


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--lo", type=float, default=1e4)
    ap.add_argument("--hi", type=float, default=4e6)
    ap.add_argument("--pool", type=int, default=16)
    ap.add_argument("--hbm-gb", type=float, default=0.0,
                    help="HBM budget in GiB (0: free device memory minus --reserve-gb)")
    ap.add_argument("--reserve-gb", type=float, default=16.0)
    ap.add_argument("--scenes", choices=("device", "pool"), default="device")
    ap.add_argument("--max-jobs", type=int, default=64)
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()

    import torch
    torch.cuda.set_device(0)
    ng.load()

    def eprint(*a):
        print(*a, file=sys.stderr, flush=True)

    free, total_mem = torch.cuda.mem_get_info()
    budget = int(args.hbm_gb * 2**30) if args.hbm_gb > 0 else int(free - args.reserve_gb * 2**30)
    if args.scenes == "pool":
        eprint("generating the scene pool")
        reqs, pool = make_trace(args.rate, args.duration, args.seed, args.lo, args.hi, args.pool)
        host_of = {id(sc): _HostScene(sc) for sc in pool}
        hosts = [host_of[id(r.scene)] for r in reqs]
    else:
        reqs = make_device_trace(args.rate, args.duration, args.seed)
        hosts = [None] * len(reqs)
    eprint(f"{len(reqs)} requests, {sum(r.n for r in reqs)} splats, budget {budget / 2**30:.1f} GiB")
    srv = BatchServer(budget, max_k=24, max_jobs=args.max_jobs)
    # warm-up pass of the kernels, not timed
    w = ng.Batch(200000, 24, 4)
    w.submit(ng.GaussianTensors.from_scene(gen_scene(50000, 1)), 1000, k=24)
    w.run()
    w.close()
    gen_scene_device(1000, 1)
    res = {"batched": srv.serve(reqs, hosts, log=eprint)}
    srv.batch.close()
    srv_rows = srv.rows
    del srv
    torch.cuda.empty_cache()
    if not args.no_plain:
        for r in reqs:
            r.t_done = -1.0
        plain = PlainServer(max(r.n for r in reqs), 24)
        res["plain"] = plain.serve(reqs, hosts, log=eprint)
    res["trace"] = {"rate_per_s": args.rate, "duration_s": args.duration,
                    "sizes": [args.lo, args.hi] if args.scenes == "pool" else [1e4, 4e6],
                    "ratios": [0.5, 0.1, 0.01], "k": [16, 24],
                    "scenes": (f"pool of {args.pool} host scenes" if args.scenes == "pool" else
                               "one per request, drawn on the device from seed 20000 + id"),
                    "hbm_budget_gib": round(budget / 2**30, 2),
                    "device_free_gib": round(free / 2**30, 2),
                    "device_total_gib": round(total_mem / 2**30, 2),
                    "working_set_rows": srv_rows,
                    "working_set_row_limit": max_engine_rows(24)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
