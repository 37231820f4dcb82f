"""Continuous-batching serving loop for RT-TDA propagation requests on one GPU.

Requests (o, v, N_Q, pulse, steps) arrive over time.  The library's serving pool (rttda_pool_*)
does the batching: it admits a request when its HBM footprint (factor tensors + library
workspace + state + trace) fits the remaining budget, advances every admitted request in chunks
of RK4 steps, each on its own HIP stream so that the work of different requests overlaps on the
device, and returns a request's budget when it is released.  This module keeps the arrival
queue (first come, first served, with later requests filling memory that earlier ones do not
fit), creates each request's context and device tensors, and records latencies.

Each request's result does not depend on what else is resident: the kernels use no atomics
and no cross-request state, so a request's trace in a mix is bitwise the trace it gets alone.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import inputs as I
from . import rttda

AU_FS = 0.02418884326585747
RK4_LIMIT = 2.5


def request_flops(shape: I.Shape, n_steps: int) -> float:
    ov = shape.o * shape.v
    return n_steps * 4.0 * (8.0 * shape.nq * ov + 4.0 * shape.nq * ov * (shape.o + shape.v))


def padded_sizes(o: int, v: int):
    """Orbital counts a request is served at: v up to a multiple of 8 and o up to an even count (a
    multiple of 8 from 121 on), the sizes the direct-to-LDS and large-o GEMM exchange kernels take.
    The added orbitals carry zero factors and zero dipoles, so their amplitudes stay exactly zero
    and the request's own amplitudes follow the same equations (only zero terms join the sums)."""
    vp = (v + 7) // 8 * 8
    op = (o + 7) // 8 * 8 if o > 120 else (o + 1) // 2 * 2
    return op, vp


def padded_tensors(shape: I.Shape, t: dict, device: str):
    """The request's tensors embedded in the padded sizes (zero factors and dipoles for the added
    orbitals; their energies repeat the highest occupied and lowest virtual level, so the gaps of A
    stay within the request's own range)."""
    import torch

    o, v = shape.o, shape.v
    op, vp = padded_sizes(o, v)
    if (op, vp) == (o, v):
        return t
    out = {}
    out["e_occ"] = torch.cat([t["e_occ"], t["e_occ"][-1:].expand(op - o)]).contiguous()
    out["e_virt"] = torch.cat([t["e_virt"][:1].expand(vp - v), t["e_virt"]]).contiguous()
    # (added virtuals go first so that e_virt stays sorted; the factor and dipole columns follow)
    nq = shape.nq
    dt = t["b_ov"].dtype
    b_ov = torch.zeros((nq, op, vp), dtype=dt, device=device)
    b_ov[:, :o, vp - v:] = t["b_ov"]
    b_oo = torch.zeros((nq, op, op), dtype=dt, device=device)
    b_oo[:, :o, :o] = t["b_oo"]
    b_vv = torch.zeros((nq, vp, vp), dtype=dt, device=device)
    b_vv[:, vp - v:, vp - v:] = t["b_vv"]
    n, npd = o + v, op + vp
    mu = torch.zeros((3, npd, npd), dtype=t["mu"].dtype, device=device)
    idx = torch.cat([torch.arange(o), op + (vp - v) + torch.arange(v)]).to(device)
    mu[:, idx[:, None], idx[None, :]] = t["mu"]
    out.update(b_ov=b_ov, b_oo=b_oo, b_vv=b_vv, mu=mu)
    return out


def footprint(shape: I.Shape, n_steps: int, precision: str) -> int:
    """HBM bytes a resident request holds (at its padded sizes)."""
    o, v = padded_sizes(shape.o, shape.v)
    nq = shape.nq
    bsz = 4 if precision == "fp32" else 2
    factors = nq * (o * v + o * o + v * v) * bsz
    other = (o + v) * 8 + 3 * (o + v) ** 2 * 8
    state = 2 * o * v * 8 + 16
    trace = (n_steps + 1) * 8
    ws = rttda.workspace_bytes(o, v, nq, precision, 1) + 512
    return int(factors + other + state + trace + ws)


@dataclass
class Slot:
    req: I.Request
    ctx: rttda.Context
    dev: rttda.DeviceProblem
    c0: object
    c: object
    trace: object
    stream: object
    bytes: int
    t_admit: float
    pool_slot: int = -1


@dataclass
class Result:
    rid: int
    o: int
    n_steps: int
    arrival: float
    admitted: float
    finished: float
    trace: Optional[np.ndarray] = None
    refused: str = ""  # why the request was not propagated (empty when it was)

    @property
    def latency(self):
        return self.finished - self.arrival

    @property
    def wait(self):
        return self.admitted - self.arrival


class Server:
    def __init__(self, budget_bytes: int, chunk_steps: int = 128, precision: str = "mixed", device: str = "cuda:0",
                 keep_traces: bool = True, max_active: int = 64, progress=None, stability_steps: int = 20):
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_steps)
        self.precision = precision
        self.device = device
        self.keep_traces = keep_traces
        self.max_active = max_active
        self.progress = progress  # called with a line of text when a request retires, or None
        # Lanczos steps of the time-step check at admission (0: no check).  RK4 is stable for
        # |lambda dt| <= 2.8 on the imaginary axis; a request whose bound on rho(A) dt exceeds 2.5
        # is refused before it takes a pool slot.
        self.stability_steps = int(stability_steps)
        self.pool = rttda.Pool(self.budget)
        self.peak_used = 0
        self.active: List[Slot] = []
        self.queue: deque = deque()
        self.results: Dict[int, Result] = {}

    @property
    def used(self) -> int:
        return self.pool.usage()[0]

    # ------------------------------------------------------------------------------------
    def _admit(self, req: I.Request, now: float) -> Optional[Slot]:
        import torch

        nb = footprint(req.shape, req.n_steps, self.precision)
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            t = I.make_device_tensors(req.shape, req.seed, device=self.device)
            op, vp = padded_sizes(req.shape.o, req.shape.v)
            shp = I.Shape(op, vp, req.shape.nq, req.shape.b_scale, storage=req.shape.storage)
            dev = rttda.DeviceProblem.from_tensors(shp, padded_tensors(req.shape, t, self.device), self.precision)
            ctx = rttda.Context(dev, max_rhs=1, stream=stream, sync_streams=False)
            c0, c = rttda.ground_state(1, op, vp, device=self.device)
            trace = torch.empty((req.n_steps + 1, 1), dtype=torch.float64, device=self.device)
        if self.stability_steps > 0:
            _, bound = ctx.spectral_radius(self.stability_steps)
            if bound * req.dt > RK4_LIMIT:
                ctx.close()
                why = f"rho(A) dt <= {bound * req.dt:.3f} exceeds the RK4 stability limit {RK4_LIMIT}"
                self.results[req.rid] = Result(req.rid, req.shape.o, req.n_steps, req.arrival, now, now, None, why)
                if self.progress is not None:
                    self.progress(f"request {req.rid} refused: {why}")
                return None
        slot = Slot(req, ctx, dev, c0, c, trace, stream, nb, now)
        slot.pool_slot = self.pool.admit(ctx, [req.pulse], req.dt, req.n_steps, c0, c, trace, footprint=nb)
        self.peak_used = max(self.peak_used, self.used)
        if self.progress is not None:
            self.progress(f"request {req.rid} (o={req.shape.o}, {req.n_steps} steps, {nb / 2 ** 30:.2f} GiB) admitted "
                          f"at {now:.2f} s")
        return slot

    def _retire(self, s: Slot, now: float):
        bad = self.pool.result(s.pool_slot)  # the guard over all the request's chunks
        self.pool.release(s.pool_slot)
        tr = s.trace.cpu().numpy()[:, 0] if self.keep_traces else None
        if bad != -1:
            raise rttda.RttdaError(rttda.E_UNSTABLE, f"request {s.req.rid}: norm guard at step {bad}")
        s.ctx.close()
        self.results[s.req.rid] = Result(s.req.rid, s.req.shape.o, s.req.n_steps, s.req.arrival, s.t_admit, now, tr)
        if self.progress is not None:
            self.progress(f"request {s.req.rid} (o={s.req.shape.o}, {s.req.n_steps} steps) done at {now:.2f} s")

    # ------------------------------------------------------------------------------------
    def run(self, requests: List[I.Request], time_scale: float = 1.0, realtime: bool = True) -> dict:
        """Serve `requests` (arrival times scaled by time_scale); returns statistics."""
        import torch

        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in requests:
            if footprint(r.shape, r.n_steps, self.precision) > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        max_concurrent = 0
        last_note = 0.0
        while pending or self.queue or self.active:
            now = clock()
            if self.progress is not None and now - last_note > 15.0:
                last_note = now
                self.progress(f"t={now:.0f} s: {len(self.active)} resident, {len(self.queue)} queued, "
                              f"{len(self.results)} done, {self.used / 2 ** 30:.1f} GiB in use")
            while pending and (not realtime or pending[0].arrival * time_scale <= now):
                self.queue.append(pending.popleft())
            # retire finished requests
            for s in list(self.active):
                if self.pool.poll(s.pool_slot)[1]:
                    self.active.remove(s)
                    self._retire(s, clock())
            # admit in arrival order while memory and slots allow (later requests may backfill)
            for r in list(self.queue):
                if len(self.active) >= self.max_active:
                    break
                if self.used + footprint(r.shape, r.n_steps, self.precision) <= self.budget:
                    self.queue.remove(r)
                    s = self._admit(r, clock())
                    if s is not None:
                        self.active.append(s)
            max_concurrent = max(max_concurrent, len(self.active))
            # next chunk of every resident request whose previous chunk has finished
            issued = self.pool.step(self.chunk) if self.active else 0
            if not issued:
                if self.active:
                    time.sleep(2e-4)
                elif pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival * time_scale - clock())))
        makespan = clock()
        torch.cuda.synchronize()
        served = [r for r in requests if not self.results[r.rid].refused]
        res = [self.results[r.rid] for r in served]
        lat = np.array([x.latency for x in res]) if res else np.zeros(1)
        wait = np.array([x.wait for x in res]) if res else np.zeros(1)
        flops = sum(request_flops(r.shape, r.n_steps) for r in served)
        fs = sum(r.n_steps * r.dt * AU_FS for r in served)
        return {
            "requests": len(requests),
            "refused": len(requests) - len(served),
            "makespan_s": makespan,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_wait_s": float(np.percentile(wait, 50)),
            "max_concurrent": max_concurrent,
            "peak_hbm_bytes": self.peak_used,
            "budget_bytes": self.budget,
            "aggregate_fs_per_hour": fs / (makespan / 3600.0),
            "sigma_gflops": flops / makespan / 1e9,
        }


def _scaled_requests(n: int, seed: int, o_max: int, steps_scale: float, rate: float):
    reqs = I.serving_requests(n, rate=rate, seed=seed, o_min=10, o_max=o_max)
    for r in reqs:
        r.n_steps = max(20, int(round(r.n_steps * steps_scale)))
        if r.pulse.kind == I.PULSE_GAUSS:
            r.pulse.t0 = 0.5 * r.n_steps * r.dt
            r.pulse.fwhm = min(400.0, 0.25 * r.n_steps * r.dt)
    return reqs


def main(argv=None):
    """Capacity-scaled serving run: a burst (all arrivals at t = 0) measures the capacity of the
    request mix; a Poisson stream at `load` x that capacity then gives steady-state latencies."""
    import argparse
    import json

    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--o-max", type=int, default=48)
    ap.add_argument("--steps-scale", type=float, default=0.1, help="scale of the 500..8000 step counts")
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--seed", type=int, default=I.SEED_BASE + 5)
    ap.add_argument("--verbose", action="store_true", help="a line on stderr per retired request")
    ap.add_argument("--max-active", type=int, default=64,
                    help="most requests resident at once (besides the HBM budget): the compute the mix shares")
    a = ap.parse_args(argv)
    budget = int(a.budget_gib * (1 << 30))
    burst = _scaled_requests(a.requests, a.seed, a.o_max, a.steps_scale, rate=1e9)
    import sys

    say = (lambda m: print(m, file=sys.stderr, flush=True)) if a.verbose else None
    srv = Server(budget, chunk_steps=a.chunk, precision="mixed", keep_traces=False, progress=say,
                 max_active=a.max_active)
    b = srv.run(burst, realtime=False)
    capacity = a.requests / b["makespan_s"]
    rate = a.load * capacity
    stream = _scaled_requests(a.requests, a.seed, a.o_max, a.steps_scale, rate=rate)
    srv2 = Server(budget, chunk_steps=a.chunk, precision="mixed", keep_traces=False, progress=say,
                  max_active=a.max_active)
    p = srv2.run(stream, realtime=True)
    torch.cuda.synchronize()
    print(json.dumps({"mix": {"requests": a.requests, "o": [10, a.o_max], "v": "7.5 o", "n_aux": "20 o",
                              "steps": [int(500 * a.steps_scale), int(8000 * a.steps_scale)],
                              "pulses": "50% delta kick, 50% Gaussian-sine", "precision": "mixed",
                              "max_active": a.max_active, "chunk_steps": a.chunk, "budget_gib": a.budget_gib},
                      "burst": b, "capacity_req_per_s": capacity, "poisson_rate_req_per_s": rate, "poisson": p}))


if __name__ == "__main__":
    main()
