"""Serving loop over the batched multi-solve pool (continuous batching).

Requests of mixed shape -- 2D grids, 3D grids, quasi-1D shock tubes, each
with its own gamma, step count and initial data -- arrive on a seeded Poisson
clock.  The loop admits arrived requests into the pool while their footprint
fits the arena (FIFO with backfill: a request that does not fit now is
passed over by smaller ones behind it), advances every resident solve with a
K-step graph replay, retires finished solves (moments copied to the host,
slot and arena space released) and admits more -- all while the others keep
running.  Latency is completion minus arrival; throughput is cell updates
over the makespan.

The comparison server runs the same trace one request at a time through the
single-solve API in FP64, with eager launches and no graphs.

Everything here is host-side orchestration; every step of every solve runs
in the HIP library.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm
from .inputs import smooth_fields_device, sod_fields

OPEN_X = lbm.LBM_BC(lbm.LBM_BC_ZERO_GRADIENT, lbm.LBM_BC_PERIODIC)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the trace starts
    kind: str               # "2d", "3d" or "tube"
    req: object             # lbm.lbm_request
    seed: int
    tube: tuple = None      # (left, right) states (rho, u, p) for tubes
    admitted: float = None
    done: float = None
    ok: bool = True
    note: str = ""
    mass: float = float("nan")
    extra: dict = field(default_factory=dict)

    @property
    def cells(self):
        return self.req.nx * self.req.ny * self.req.nz

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


def tube_states(rng):
    """One shock tube of the ensemble recipe: pressure ratio log-uniform in
    [2, 20], density ratio uniform in [2, 10], at rest; temperatures scaled
    so that their geometric mean is 1 (T = p / rho)."""
    pr = math.exp(rng.uniform(math.log(2.0), math.log(20.0)))
    dr = rng.uniform(2.0, 10.0)
    tl_over_tr = pr / dr
    t_r = 1.0 / math.sqrt(tl_over_tr)
    t_l = tl_over_tr * t_r
    rho_r = 1.0
    rho_l = dr * rho_r
    return (rho_l, 0.0, rho_l * t_l), (rho_r, 0.0, rho_r * t_r)


def tube_ensemble(n=512, steps=1000, seed=4, tau=0.8):
    """Quasi-1D shock tubes on D2Q37: Nx log-uniform in [100, 4000], Ny = 4,
    gamma uniform in [1.1, 1.67], zero-gradient ends, periodic in y."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx = int(round(math.exp(rng.uniform(math.log(100), math.log(4000)))))
        gamma = rng.uniform(1.1, 1.67)
        left, right = tube_states(rng)
        req = lbm.make_request(2, gamma, tau, tau, nx, 4, bc=OPEN_X, steps=steps)
        out.append(Request(k, 0.0, "tube", req, seed * 100000 + k, tube=(left, right)))
    return out


def request_bytes_moved(r, precision=lbm.LBM_FP32_DEV):
    q = 37 if r.req.dim == 2 else 107
    s = 4 if precision == lbm.LBM_FP32_DEV else 8
    return 2 * q * 2 * s * r.cells * r.req.steps


def poisson_trace(n, rate, seed=5, tube_steps=None):
    """The mixed request stream: 50% 2D grids (side log-uniform 256..2048),
    30% 3D grids (side log-uniform 64..192), 20% shock tubes; gamma uniform
    in [1.1, 1.67]; steps uniform in {200..2000}; smooth seeded fields (tubes:
    shock-tube states); exponential inter-arrival times at `rate` per second."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        gamma = rng.uniform(1.1, 1.67)
        steps = int(rng.integers(200, 2001))
        if u < 0.5:
            side = int(round(math.exp(rng.uniform(math.log(256), math.log(2048)))))
            req = lbm.make_request(2, gamma, 0.7, 0.8, side, side, steps=steps)
            out.append(Request(k, t, "2d", req, seed * 100000 + k))
        elif u < 0.8:
            side = int(round(math.exp(rng.uniform(math.log(64), math.log(192)))))
            req = lbm.make_request(3, gamma, 0.65, 0.65, side, side, side, steps=steps)
            out.append(Request(k, t, "3d", req, seed * 100000 + k))
        else:
            nx = int(round(math.exp(rng.uniform(math.log(100), math.log(4000)))))
            left, right = tube_states(rng)
            req = lbm.make_request(2, gamma, 0.8, 0.8, nx, 4, bc=OPEN_X,
                                   steps=tube_steps or steps)
            out.append(Request(k, t, "tube", req, seed * 100000 + k, tube=(left, right)))
    return out


def device_fields(r, device="cuda"):
    import torch
    q = r.req
    if r.kind == "tube":
        f = sod_fields(2, q.nx, q.ny, left=r.tube[0], right=r.tube[1])
        return [torch.from_numpy(np.ascontiguousarray(a.reshape(-1))).to(device) for a in f]
    rho, u, T = smooth_fields_device(q.dim, q.nx, q.ny, q.nz, seed=r.seed, device=device)
    return [rho, u.reshape(-1).contiguous(), T]


def _finish(r, rho, t0):
    r.done = time.perf_counter() - t0
    r.ok = bool(np.all(np.isfinite(rho)))
    r.mass = float(np.sum(rho)) if r.ok else float("nan")
    if not r.ok:
        r.note = "non-finite"


def _progress(every, n_done, total, t0, what):
    if every and n_done % every == 0:
        import sys
        print(f"# {what}: {n_done}/{total} requests done at "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)


def serve_pool(trace, budget_bytes, max_slots=256, ticks=8, precision=lbm.LBM_FP32_DEV,
               realtime=True, keep=None, progress_every=0):
    """Continuous batching of `trace` through one pool.  Returns the trace
    (with admitted / done / ok filled in) and the makespan in seconds.  With
    realtime=False every request is taken as arrived at t = 0.  `keep`, if
    given, is called as keep(request, pool, slot) before a finished slot is
    released.  progress_every > 0 prints a line to stderr every that many
    completions."""
    import torch
    pending = sorted(trace, key=lambda r: r.arrival)
    waiting = []
    resident = {}
    i = 0
    n_done = 0
    n_valid = len(pending)
    stream = torch.cuda.Stream()
    with lbm.Pool(budget_bytes, max_slots, precision) as pool:
        pool.set_stream(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while i < len(pending) or waiting or resident:
            now = time.perf_counter() - t0
            while i < len(pending) and (not realtime or pending[i].arrival <= now):
                waiting.append(pending[i])
                i += 1
            # admission, FIFO with backfill.  The library judges each request:
            # a footprint of 0 means it would refuse it (EINVAL), e.g. a gamma
            # that leaves delta < 0.  A request's device fields are built only
            # once the pool has a slot and the arena space for it, so waiting
            # requests hold no device memory.
            still = []
            info = pool.info()
            for r in waiting:
                need = lbm.lbm_pool_request_bytes(r.req, precision)
                if need == 0 or need > info["budget_bytes"]:
                    why = "invalid request" if need == 0 else "larger than the arena"
                    r.ok, r.note, r.done = False, f"rejected: {why}", now
                    n_valid -= 1
                    continue
                if info["resident"] >= info["max_slots"] or need > info["largest_free_bytes"]:
                    still.append(r)
                    continue
                with torch.cuda.stream(stream):
                    f = device_fields(r)
                slot = pool.admit_dev(r.req, *f)
                del f  # copied into the pool (the stream orders the reuse)
                if slot is None:
                    still.append(r)
                    continue
                r.admitted = time.perf_counter() - t0
                resident[slot] = r
                info = pool.info()
            waiting = still
            if not resident:
                if i < len(pending):
                    time.sleep(max(0.0, pending[i].arrival - (time.perf_counter() - t0)))
                continue
            pool.run(ticks)
            for slot in pool.poll():
                r = resident.pop(slot)
                rho, _, _ = pool.moments(slot)
                if keep:
                    keep(r, pool, slot)
                _finish(r, rho, t0)
                pool.release(slot)
                n_done += 1
                _progress(progress_every, n_done, n_valid, t0, "FP32 pool")
        makespan = time.perf_counter() - t0
    return trace, makespan


def serve_sequential(trace, precision=lbm.LBM_FP64, realtime=True, progress_every=0):
    """The same trace, one request at a time, single-solve API, eager
    launches (no graphs), in arrival order."""
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n, r in enumerate(sorted(trace, key=lambda r: r.arrival)):
        _progress(progress_every, n, len(trace), t0, "one at a time")
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        q = r.req
        r.admitted = time.perf_counter() - t0
        try:
            s = lbm.Solver(q.dim, q.gamma, q.tau_f, q.tau_g, q.nx, q.ny, q.nz, bc=q.bc,
                           precision=precision)
        except lbm.LBMError as e:  # the library refuses the request (EINVAL)
            if e.code != lbm.LBM_EINVAL:
                raise
            r.ok, r.note, r.done, r.admitted = False, "rejected: invalid request", None, None
            continue
        with s:
            s.set_stream(stream)
            with torch.cuda.stream(stream):
                f = device_fields(r)
            lbm.lbm_init_fields_dev(s.h, *f)
            s.step(q.steps)
            rho, _, _ = s.moments()
        _finish(r, rho, t0)
    return trace, time.perf_counter() - t0


def summarize(trace, makespan):
    done = [r for r in trace if r.done is not None and r.ok]
    lat = np.array([r.latency for r in done]) if done else np.array([float("nan")])
    updates = sum(r.cells * r.req.steps for r in done)
    # every admitted request's steps ran on the GPU, finite or not
    updates_all = sum(r.cells * r.req.steps for r in trace if r.done is not None
                      and not r.note.startswith("rejected"))
    return {
        "requests": len(trace), "completed": len(done),
        "rejected": sum(1 for r in trace if r.note.startswith("rejected")),
        "non_finite": sum(1 for r in trace if r.note == "non-finite"),
        "p50_s": round(float(np.percentile(lat, 50)), 4),
        "p99_s": round(float(np.percentile(lat, 99)), 4),
        "makespan_s": round(makespan, 3),
        "aggregate_mlups": round(updates / makespan / 1e6, 1),
        "aggregate_mlups_all_admitted": round(updates_all / makespan / 1e6, 1),
    }
