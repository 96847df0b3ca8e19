"""Request loop for many independent solves on one GPU (continuous batching).

Requests arrive over time (a seeded Poisson process), are admitted as slots
and HBM budget free up (admission by device footprint), keep their state
resident on the device, and share launches with whatever else is running
(:class:`paper_1208_4772_amd.dg.Batch`).  A request that arrives while others
are on the GPU joins at the next chunk boundary.  Latency is measured from
arrival to completion, so queueing is included.

The host side here only orders requests and calls the C ABI; every step of
every solve runs in the library's kernels.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

import meshgen

from . import dg

# Element counts of the two O-grids at scale 1 (the scale factor sets K).
_DEFAULT_K = {"cylinder": 20000, "airfoil": 120000}


@dataclass
class Request:
    rid: int
    kind: str
    K_target: int
    P: int
    mach: float
    steps: int
    arrival: float            # seconds after the start of the run
    av: bool | None = None    # artificial viscosity; None takes the case's default
    case: object = None       # meshgen Case, built before the run (the request payload)
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    status: int = 0
    t_sim: float = math.nan
    steps_run: int = 0           # steps the solve actually ran (fewer if it stopped)
    final_state: object = None   # host copy of the result when the server keeps states
    error: str = ""

    @property
    def dofs(self):
        return self.case.dofs() if self.case is not None else 0

    @property
    def latency(self):
        return self.finished - self.arrival


def make_requests(n=64, mean_gap=0.05, seed=64, K_range=(2000, 60000), steps_range=(500, 3000),
                  P_choices=(1, 2, 3, 4, 5), mach_range=(0.3, 0.85), av=None, build=True):
    """The seeded request mix: case in {cylinder, airfoil}, element count
    uniform in K_range, order uniform over P_choices, Mach uniform in
    mach_range, step count uniform in steps_range, exponential arrival gaps
    of mean ``mean_gap`` seconds.  Every request runs with the shock sensor
    and artificial viscosity (Mach numbers up to 0.85 form shocks on both
    geometries) unless ``av`` says otherwise."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(mean_gap)
        kind = ("cylinder", "airfoil")[int(rng.integers(2))]
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        P = int(rng.choice(P_choices))
        mach = float(rng.uniform(*mach_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        reqs.append(Request(i, kind, K, P, mach, steps, t, av))
    if build:
        for r in reqs:
            build_case(r)
    return reqs


def build_case(req: Request):
    """Mesh, node positions and freestream start of a request (host)."""
    rr, ss = dg.reference_nodes(req.P)
    scale = req.K_target / _DEFAULT_K[req.kind]
    # a start compatible with the slip wall (cylinders: the potential flow;
    # airfoils: the freestream damped to rest at the wall): the impulsive
    # start drives many meshes of the mix to rho, p <= 0
    start = "potential" if req.kind == "cylinder" else "damped"
    case = meshgen.make_case(req.kind, rr, ss, scale=scale, P=req.P, mach=req.mach, steps=req.steps,
                             start=start)
    case.av = True if req.av is None else bool(req.av)
    req.av = case.av
    req.case = case
    return case


@dataclass
class Report:
    requests: list
    wall_s: float
    precision: str
    budget: int
    max_slots: int
    chunk_steps: int
    peak_slots: int = 0
    busy_rejections: int = 0
    extra: dict = field(default_factory=dict)

    def summary(self):
        """Latency percentiles over every request (one that stopped on the
        state check or failed its setup counts at the time it stopped:
        censored, not dropped) and over the completed ones; throughput from
        the steps every request actually ran."""
        done = [r for r in self.requests if r.status == 0]
        lat_all = np.array([r.latency for r in self.requests])
        lat = np.array([r.latency for r in done]) if done else np.array([math.nan])
        total = sum(r.dofs * 5 * r.steps_run for r in self.requests)
        first = min(r.arrival for r in self.requests)
        last = max(r.finished for r in self.requests)
        return dict(n_requests=len(self.requests), precision=self.precision,
                    p50_latency_s=float(np.percentile(lat_all, 50)),
                    p99_latency_s=float(np.percentile(lat_all, 99)),
                    p50_latency_completed_s=float(np.percentile(lat, 50)),
                    p99_latency_completed_s=float(np.percentile(lat, 99)),
                    mean_latency_s=float(lat_all.mean()),
                    dof_updates=float(total),
                    aggregate_dof_updates_per_s=float(total / (last - first)),
                    makespan_s=float(last - first), peak_slots=self.peak_slots,
                    budget_bytes=self.budget, max_slots=self.max_slots,
                    chunk_steps=self.chunk_steps, busy_rejections=self.busy_rejections,
                    failed=int(sum(1 for r in self.requests if r.status != 0)), **self.extra)


class Server:
    """Continuous-batching server over one GPU."""

    def __init__(self, hbm_budget_bytes=1 << 30, max_slots=16, precision="fp32", chunk_steps=50,
                 device="cuda:0", keep_states=False, verbose=False):
        self.keep_states = bool(keep_states)
        self.verbose = bool(verbose)
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.chunk_steps = int(chunk_steps)
        self.device = device

    def _log(self, msg):
        if self.verbose:
            print(msg, flush=True)

    def tune(self, requests):
        """Workgroup shape per kind of solve in the mix (order, viscosity) at
        the server's precision: dg_autotune on the request of median size of
        each kind, unless the tuning table already holds it.  Batch groups
        created afterwards take these shapes.  Returns {(P, av): waves}."""
        if self.precision == "fp64":
            return {}
        kinds = {}
        for r in requests:
            kinds.setdefault((r.P, bool(r.av)), []).append(r)
        shapes = {}
        for (P, av), rs in sorted(kinds.items()):
            rs = sorted(rs, key=lambda r: r.case.K)
            req = rs[len(rs) // 2]
            sol = dg.Solver.from_case(req.case, self.precision, device=self.device)
            try:
                shapes[(P, av)] = sol.autotune(sol.state(req.case.U0))[0]
            finally:
                sol.close()
        return shapes

    def run(self, requests):
        import torch
        batch = dg.Batch(self.budget, self.max_slots)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        active = {}          # slot -> (request, solver, state, estimated bytes)
        reserved = 0         # estimated bytes of admitted requests
        peak = 0
        rejections = 0
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admit in arrival order while budget and slots allow
            while queue and len(active) < self.max_slots:
                req = queue[0]
                est = dg.estimate_footprint(req.case.K, req.P, self.precision, req.av)
                if est > self.budget:
                    # can never fit: fail it rather than block the queue
                    queue.popleft()
                    req.status = dg.DG_EBUSY
                    req.admitted = req.finished = time.perf_counter() - t0
                    continue
                if reserved + est > self.budget:
                    break
                try:
                    sol = dg.Solver.from_case(req.case, self.precision, device=self.device)
                except dg.DGError as e:
                    # a request whose setup fails is reported, not retried
                    queue.popleft()
                    req.status = e.code
                    req.error = str(e)
                    req.admitted = req.finished = time.perf_counter() - t0
                    self._log(f"request {req.rid} setup failed: {e}")
                    continue
                U = sol.state(req.case.U0)
                slot = batch.admit(sol, U, req.steps)
                if slot is None:
                    rejections += 1
                    sol.close()
                    break
                queue.popleft()
                req.admitted = time.perf_counter() - t0
                active[slot] = (req, sol, U, est)
                reserved += est
                peak = max(peak, len(active))
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            batch.advance(self.chunk_steps)
            for slot in batch.poll():
                req, sol, U, est = active.pop(slot)
                st = batch.stats(slot)
                req.finished = time.perf_counter() - t0
                req.status = st.status
                req.t_sim = st.t
                req.steps_run = st.steps
                if self.keep_states:
                    req.final_state = U.double().cpu().numpy()
                batch.release(slot)
                reserved -= est
                sol.close()
                self._log(f"request {req.rid} done: status {req.status}, latency {req.latency:.3f} s, "
                          f"{len(active)} active, {len(queue)} queued")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        captures, kinds = batch.info()
        batch.close()
        return Report(list(requests), wall, self.precision, self.budget, self.max_slots,
                      self.chunk_steps, peak, rejections,
                      extra=dict(graph_captures=captures, solve_kinds=kinds))


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="continuous-batching run over a seeded request mix")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--mean-gap", type=float, default=0.05)
    ap.add_argument("--seed", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=1.0)
    ap.add_argument("--max-slots", type=int, default=16)
    ap.add_argument("--chunk-steps", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--no-tune", action="store_true", help="batch groups keep the default workgroup shape")
    ap.add_argument("--tuning-cache", default=None,
                    help="tuning table file: loaded if it exists, written after tuning")
    a = ap.parse_args(argv)
    t = time.perf_counter()
    reqs = make_requests(a.requests, a.mean_gap, a.seed)
    print(f"built {len(reqs)} requests in {time.perf_counter() - t:.1f} s", flush=True)
    srv = Server(int(a.budget_gib * 2**30), a.max_slots, a.precision, a.chunk_steps, verbose=True)
    shapes = {}
    if not a.no_tune:
        import os
        if a.tuning_cache and os.path.exists(a.tuning_cache):
            dg.Tuning.load(a.tuning_cache)
        t = time.perf_counter()
        shapes = srv.tune(reqs)
        print(f"tuned {len(shapes)} kinds in {time.perf_counter() - t:.1f} s: "
              + ", ".join(f"P={P}{' av' if av else ''}: {w}" for (P, av), w in shapes.items()), flush=True)
        if a.tuning_cache:
            dg.Tuning.save(a.tuning_cache)
    rep = srv.run(reqs)
    summ = rep.summary()
    summ["workgroup_waves"] = {f"P{P}{'_av' if av else ''}": w for (P, av), w in shapes.items()}
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    main()
