"""Throughput of the fused collide-and-stream step on one MI355X.

Headline: D3Q107, 256^3 periodic grid, smooth seeded perturbation (amplitude
0.01 in rho and T, 0.02 in u), gamma 1.4 (delta 2), tau_f = tau_g = 0.65,
populations in FP32 deviation storage, 500 timed steps.  The other paths
(D3Q107 FP64 and half-precision scaled storage; D2Q37 4096^2 in all three
storage precisions, tau_f 0.7, tau_g 0.8) are measured the same way and
reported under "paths".

One step = one launch of the fused step kernel over the whole grid (pull,
moments, equilibrium, BGK relaxation of g and h, store).  Inputs are resident
in HBM before the timed region; the timed region holds exactly K steps
bracketed by device synchronisation, timed with HIP events recorded on the
stream the kernels run on.

Roofline: algorithmic bytes per cell update = 2 (read + write) x Q x 2
(g and h) x bytes per stored value (8, 4 or 2); achieved GB/s = those bytes x cells / average
launch time; peak = 8 TB/s HBM3E.  Beside the peak, the same run measures
what plain data movement reaches on this device: a streaming copy and a
read-only sweep over as many bytes as one headline launch moves
(libhbmprobe.so).

The oracle leg (cpu_baseline, skipped with --no-cpu) times the FP64 CPU
oracle on a bounded sample of the headline workload, and puts the GPU's error
against the oracle next to every path, on a small sample of that path's own
recipe; for the shock-tube ensemble it adds each tube's L1 error against the
exact Riemann solution.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

STORAGE = {"fp64": ("FP64", 8), "fp32": ("FP32 deviation storage", 4),
           "fp16": ("FP16 scaled deviation storage", 2)}

PATHS = {}
for _store in ("fp32", "fp64", "fp16"):
    PATHS[f"d3q107_{_store}"] = dict(dim=3, shape=(256, 256, 256), gamma=1.4, tf=0.65, tg=0.65,
                                     store=_store, seed=3, steps=500)
for _store in ("fp32", "fp64", "fp16"):
    PATHS[f"d2q37_{_store}"] = dict(dim=2, shape=(4096, 4096, 1), gamma=1.4, tf=0.7, tg=0.8,
                                    store=_store, seed=2, steps=1000)
# gamma = 5/3 in 3D: delta = 0, so h carries nothing; it is still stored,
# loaded, relaxed and written in full (no h-skipping specialisation).
PATHS["d3q107_fp32_gamma53"] = dict(PATHS["d3q107_fp32"], gamma=5.0 / 3.0, steps=200)
# The D3Q107 step with its pulled rows staged in LDS (variant SPLIT_LDS),
# beside the default kernel that pulls straight from global memory.
for _store in ("fp32", "fp64", "fp16"):
    PATHS[f"d3q107_{_store}_lds"] = dict(PATHS[f"d3q107_{_store}"], steps=200,
                                         variant="split_lds")


# The finite-difference form of Sec. III on the same grids and fields: time
# step dt = c / (3r) with the fastest population's Courant number c = 0.25
# (2D) and 0.3 (3D), relaxation times in the units of dt.
_R = 1.196979770393074359
for _store in ("fp32", "fp64"):
    PATHS[f"d3q107_fd_{_store}"] = dict(dim=3, shape=(256, 256, 256), gamma=1.4, tf=0.12, tg=0.12,
                                        store=_store, seed=3, steps=100, dt=0.3 / (3 * _R))
    PATHS[f"d2q37_fd_{_store}"] = dict(dim=2, shape=(4096, 4096, 1), gamma=1.4, tf=0.1, tg=0.12,
                                       store=_store, seed=2, steps=300, dt=0.25 / (3 * _R))


def precision_of(store):
    from paper_1608_06345_amd import lbm
    return {"fp64": lbm.LBM_FP64, "fp32": lbm.LBM_FP32_DEV, "fp16": lbm.LBM_FP16_SCALED}[store]


def bytes_per_update(dim, store):
    q = 37 if dim == 2 else 107
    return 2 * q * 2 * STORAGE[store][1]


def describe(name, p):
    q = 37 if p["dim"] == 2 else 107
    grid = "x".join(str(n) for n in p["shape"][:p["dim"]])
    delta = 2.0 / (p["gamma"] - 1.0) - p["dim"]
    delta = 0.0 if abs(delta) < 1e-9 else delta
    scheme = (f"finite-difference form, dt {p['dt']:.4f}, " if p.get("dt") else "")
    if p.get("variant") == "split_lds":
        scheme = "pulled rows staged in LDS, "
    return (f"D{p['dim']}Q{q} {grid} periodic, smooth seeded field (seed {p['seed']}), "
            f"{scheme}gamma {p['gamma']:.6g} (delta {delta:g}), tau_f {p['tf']}, tau_g {p['tg']}, "
            f"{STORAGE[p['store']][0]}")


def _code_only(text):
    """C++ source without comments, trailing blanks and empty lines (the
    sources hold no string literal with // or /* in it)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash():
    """Hash of the step kernels' code, comments left out: the HBM byte
    counters in profiles/traffic.json stay valid across comment edits and go
    stale with any change of code."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "fd.hip", "step_core.h", "velocity_set.h", "lbm_internal.h",
              "api.hip"):
        with open(os.path.join(ROOT, "paper_1608_06345_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(name, cells):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known
    size), if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(name)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    if ent.get("cells") != cells:
        return None
    return ent["bytes_per_launch"]


def run_path(name, p, steps, warmup):
    import torch

    from paper_1608_06345_amd import lbm
    from paper_1608_06345_amd.inputs import smooth_fields

    nx, ny, nz = p["shape"]
    cells = nx * ny * nz
    prec = precision_of(p["store"])
    f = smooth_fields(p["dim"], nx, ny, nz, seed=p["seed"])
    stream = torch.cuda.Stream()  # the kernels' stream; the events go on it too
    with lbm.Solver(p["dim"], p["gamma"], p["tf"], p["tg"], nx, ny, nz, precision=prec,
                    dt=p.get("dt")) as s:
        s.set_stream(stream)
        if p.get("variant") == "split_lds":
            s.set_variant(lbm.LBM_VARIANT_SPLIT_LDS)
        dev = [torch.from_numpy(a.reshape(-1)).to("cuda") for a in f]
        torch.cuda.synchronize()
        lbm.lbm_init_fields_dev(s.h, *dev)
        s.step(warmup)
        torch.cuda.synchronize()
        del dev
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        s.step(steps)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        mass, mom, energy = s.totals()
    ms_step = ms / steps
    mlups = cells * steps / (ms * 1e-3) / 1e6
    bpu = bytes_per_update(p["dim"], p["store"])
    achieved = bpu * cells / (ms_step * 1e-3) / 1e9
    traffic = measured_traffic(name, cells)
    return {
        "workload": describe(name, p), "cells": cells, "steps": steps,
        "ms_per_step": round(ms_step, 4), "mlups": round(mlups, 1),
        "gbs": round(achieved, 1), "hbm_frac": round(achieved / PEAK_HBM_GBS, 4),
        "bytes_per_update": bpu, "traffic_bytes_per_launch": traffic,
        "mass": mass, "energy": energy,
    }


def hbm_ceiling(nbytes, reps=5, pattern_cells=None, pattern_nx=None):
    """What plain data movement reaches on this device (libhbmprobe.so): a
    streaming copy of nbytes / 2 bytes (nbytes of HBM traffic) and a
    read-only sweep of nbytes, each launch shape timed over `reps` launches
    with HIP events on the stream they run on, after one untimed launch.
    GB/s counts the bytes each launch must move (copy: read + write).
    With pattern_cells, also the D3Q107 step's own access shape with no
    arithmetic (hbm_probe_planes): 214 planes of that many cells, rows of
    pattern_nx."""
    import ctypes

    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1608_06345_amd", "libhbmprobe.so"))
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    lib.hbm_probe_variants.argtypes = [i32]
    lib.hbm_probe_variant_name.argtypes = [i32, i32]
    lib.hbm_probe_variant_name.restype = ctypes.c_char_p
    lib.hbm_probe_copy.argtypes = [vp, vp, sz, i32, vp]
    lib.hbm_probe_read.argtypes = [vp, sz, i32, vp, vp]
    half = (nbytes // 2) // 4096 * 4096
    buf = torch.empty(2 * half, dtype=torch.uint8, device="cuda")
    buf.fill_(1)  # ordinary float data (every float reads 2.4e-38)
    sink = torch.zeros(256, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    src, dst = buf.data_ptr(), buf.data_ptr() + half
    out = {"copy": {}, "read": {}, "copy_bytes_per_launch": 2 * half,
           "read_bytes_per_launch": 2 * half}
    torch.cuda.synchronize()
    for kind in (0, 1):
        for v in range(lib.hbm_probe_variants(kind)):
            name = lib.hbm_probe_variant_name(kind, v).decode()

            def once():
                if kind == 0:
                    rc = lib.hbm_probe_copy(ctypes.c_void_p(dst), ctypes.c_void_p(src), half, v,
                                            sp)
                else:
                    rc = lib.hbm_probe_read(ctypes.c_void_p(src), 2 * half, v,
                                            ctypes.c_void_p(sink.data_ptr()), sp)
                if rc != 0:
                    raise RuntimeError(f"hbm probe kind {kind} variant {name}: status {rc}")

            once()
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(reps):
                once()
            end.record(stream)
            torch.cuda.synchronize()
            ms = start.elapsed_time(end) / reps
            out["copy" if kind == 0 else "read"][name] = round(2 * half / (ms * 1e-3) / 1e9, 1)
    del buf, sink
    torch.cuda.empty_cache()
    out["copy_gbs"] = max(out["copy"].values())
    out["read_gbs"] = max(out["read"].values())
    if pattern_cells:
        lib.hbm_probe_planes.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, i32, vp]
        n = 214 * pattern_cells
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()

        def planes(a, b):
            rc = lib.hbm_probe_planes(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                      pattern_cells, pattern_cells, pattern_nx, sp)
            if rc != 0:
                raise RuntimeError(f"hbm_probe_planes: status {rc}")

        planes(src, dst)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for k in range(reps):
            planes(src, dst) if k % 2 == 0 else planes(dst, src)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / reps
        out["step_pattern_gbs"] = round(2 * 214 * pattern_cells * 4 / (ms * 1e-3) / 1e9, 1)
        out["step_pattern_ms"] = round(ms, 4)
        del src, dst
        torch.cuda.empty_cache()
    return out


def serving_runs(n_requests, servers=("pool", "sequential"), ensemble=True, rate=None):
    """The batched serving form.

    tube_ensemble: 512 quasi-1D shock tubes (D2Q37, Nx log-uniform in
      [100, 4000], Ny 4, gamma uniform in [1.1, 1.67], pressure ratio
      log-uniform in [2, 20], density ratio uniform in [2, 10]), FP32, 1000
      steps each, all resident in one pool and advanced by a single replay of
      one captured 1000-step graph.
    poisson_trace: the mixed request stream (50% 2D 256^2..2048^2, 30% 3D
      64^3..192^3, 20% tubes; gamma in [1.1, 1.67]; 200..2000 steps) arriving
      at 80% of the pool's measured capacity on this mix, served (a) by
      continuous batching in an FP32 pool with 8-step graph replays and (b)
      one request at a time in FP64 with eager launches.  Capacity: the cell
      updates per second the pool sustained over a back-to-back run of the
      trace's first 48 requests (all taken as arrived at once), divided by
      the mean cell updates per request of the mix.
    """
    import torch

    from paper_1608_06345_amd import lbm, serving

    out = {}
    if ensemble:
        tubes = serving.tube_ensemble(512, steps=1000, seed=4)
        budget = (sum(lbm.lbm_pool_request_bytes(r.req, lbm.LBM_FP32_DEV) for r in tubes)
                  + (1 << 30))
        tr, span = serving.serve_pool(tubes, budget, max_slots=600, ticks=1000, realtime=False)
        out["tube_ensemble"] = dict(serving.summarize(tr, span), graph_steps=1000,
                                    workload="512 shock tubes, D2Q37 FP32, 1000 steps, one graph")
        torch.cuda.empty_cache()
        print(f"# tube ensemble: {out['tube_ensemble']}", file=sys.stderr, flush=True)

    budget = int(250e9)  # the admission cap of the serving configuration
    pt = {"requests": n_requests}
    if rate is None:
        mix = serving.poisson_trace(400, 1.0, seed=5)
        mean_updates = np.mean([r.cells * r.req.steps for r in mix
                                if lbm.lbm_pool_request_bytes(r.req, lbm.LBM_FP32_DEV) > 0])
        cal = serving.poisson_trace(48, 1.0, seed=5)
        tr, span = serving.serve_pool(cal, budget, max_slots=256, ticks=8, realtime=False)
        cal_sum = serving.summarize(tr, span)
        capacity = cal_sum["aggregate_mlups_all_admitted"] * 1e6 / mean_updates
        rate = 0.8 * capacity
        pt["capacity"] = {"requests_per_s": round(capacity, 3),
                          "pool_mlups_back_to_back": cal_sum["aggregate_mlups_all_admitted"],
                          "mean_cell_updates_per_request": float(mean_updates),
                          "calibration_requests": 48, "makespan_s": cal_sum["makespan_s"]}
        torch.cuda.empty_cache()
        print(f"# serving capacity on the mix: {pt['capacity']}", file=sys.stderr, flush=True)
    every = 50 if n_requests >= 200 else (25 if n_requests >= 48 else 0)
    pt["rate_per_s"] = round(rate, 3)
    if "pool" in servers:
        trace = serving.poisson_trace(n_requests, rate, seed=5)
        tr, span = serving.serve_pool(trace, budget, max_slots=256, ticks=8,
                                      progress_every=every)
        pt["fp32_pool_continuous_batching"] = serving.summarize(tr, span)
        torch.cuda.empty_cache()
        print(f"# serving, FP32 pool: {pt['fp32_pool_continuous_batching']}", file=sys.stderr,
              flush=True)
    if "sequential" in servers:
        trace = serving.poisson_trace(n_requests, rate, seed=5)
        tr, span = serving.serve_sequential(trace, precision=lbm.LBM_FP64, progress_every=every)
        pt["fp64_single_solve_sequential"] = serving.summarize(tr, span)
        torch.cuda.empty_cache()
        print(f"# serving, FP64 one at a time: {pt['fp64_single_solve_sequential']}",
              file=sys.stderr, flush=True)
    out["poisson_trace"] = pt
    return out


def _errors(gpu, ref):
    """rho and T pointwise relative; u relative to max|u_oracle|."""
    (r, u, T), (r_o, u_o, T_o) = gpu, ref
    return {"rho": float(np.max(np.abs(r - r_o) / r_o)),
            "u": float(np.max(np.abs(u - u_o)) / np.max(np.abs(u_o))),
            "T": float(np.max(np.abs(T - T_o) / T_o)),
            "max_abs_u_oracle": float(np.max(np.abs(u_o)))}


def _gpu_sample(p, shape, steps, store=None, fields=None):
    from paper_1608_06345_amd import lbm
    from paper_1608_06345_amd.inputs import smooth_fields

    f = fields if fields is not None else smooth_fields(p["dim"], *shape, seed=p["seed"])
    with lbm.Solver(p["dim"], p["gamma"], p["tf"], p["tg"], *shape,
                    precision=precision_of(store or p["store"]), dt=p.get("dt")) as s:
        if p.get("variant") == "split_lds":
            s.set_variant(lbm.LBM_VARIANT_SPLIT_LDS)
        s.init_fields(*f)
        s.step(steps)
        rho, u, _ = s.moments()
        T = s.temperature()
    return rho, u, T


# Same-recipe samples for the per-path error against the oracle: small
# enough for the host, rows of whole LDS tiles (128 cells for the staged pull, 256
# for the finite-difference update), and for 3D few enough steps that seed 3's
# velocity modes are still alive (max |u| ~1e-2).
ACCURACY_SAMPLES = {
    ("lattice", 3): ((128, 64, 64), 30),
    ("lattice", 2): ((256, 256, 1), 300),
    ("fd", 3): ((256, 16, 16), 100),
    ("fd", 2): ((256, 128, 1), 300),
}


def cpu_baseline(p, paths, tubes=False):
    """The oracle leg.

    1. Timing: the FP64 oracle, as it stands, on a bounded sample of the
       headline workload -- the same lattice, parameters and field recipe on
       a 64^3 grid (256^3 would take over a minute per step on the host),
       over a fixed number of steps, on all host threads and (a smaller
       sample) on one.  MLUPS is per cell update, so it needs no rescaling.
       The GPU runs the same sample and its error is reported beside it.
    2. Accuracy of every path in `paths` (adds "max_rel_err_vs_oracle" to
       each): the path's own recipe, parameters, storage and kernel variant
       on a small grid (ACCURACY_SAMPLES), against the oracle run once per
       distinct recipe.
    3. With `tubes`, the shock-tube ensemble against the exact Riemann
       solution (tube_accuracy), returned under "tube_accuracy".
    """
    from oracle.model import OracleLBM, num_threads, set_num_threads
    from paper_1608_06345_amd.inputs import smooth_fields

    n = 64
    dim = p["dim"]
    shape = (n, n, n) if dim == 3 else (4 * n, 4 * n, 1)
    steps = 150
    f = smooth_fields(dim, *shape, seed=p["seed"])
    o = OracleLBM(dim, p["gamma"], p["tf"], p["tg"], *shape)
    o.init_fields(*f)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cells = shape[0] * shape[1] * shape[2]
    r_o, u_o, E_o = o.moments()
    ref = (r_o, u_o, o.temperature(u_o, E_o))
    err = _errors(_gpu_sample(p, shape, steps, fields=f), ref)
    # the same recipe on one core, on a smaller sample
    n1, steps1 = 32, 30
    shape1 = (n1, n1, n1) if dim == 3 else (4 * n1, 4 * n1, 1)
    o1 = OracleLBM(dim, p["gamma"], p["tf"], p["tg"], *shape1)
    o1.init_fields(*smooth_fields(dim, *shape1, seed=p["seed"]))
    threads = num_threads()
    set_num_threads(1)
    try:
        t1 = time.perf_counter()
        o1.step(steps1)
        dt1 = time.perf_counter() - t1
    finally:
        set_num_threads(threads)
    cells1 = shape1[0] * shape1[1] * shape1[2]
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass

    # per-path accuracy, one oracle run per distinct recipe
    refs = {}
    for name, path in paths.items():
        q = PATHS[name]
        key = ("fd" if q.get("dt") else "lattice", q["dim"])
        shp, nst = ACCURACY_SAMPLES[key]
        rk = (key, q["gamma"], q["tf"], q["tg"], q.get("dt"), q["seed"])
        if rk not in refs:
            fr = smooth_fields(q["dim"], *shp, seed=q["seed"])
            orc = OracleLBM(q["dim"], q["gamma"], q["tf"], q["tg"], *shp, dt=q.get("dt"))
            orc.init_fields(*fr)
            orc.step(nst)
            ro, uo, Eo = orc.moments()
            refs[rk] = (fr, (ro, uo, orc.temperature(uo, Eo)))
        fr, ref_p = refs[rk]
        e = _errors(_gpu_sample(q, shp, nst, fields=fr), ref_p)
        e["sample"] = f"{'x'.join(str(v) for v in shp[:q['dim']])}, {nst} steps, same recipe"
        path["max_rel_err_vs_oracle"] = e
    out = {"tube_accuracy": tube_accuracy()} if tubes else {}
    return {**out, "value": round(cells * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, D{dim}Q{o.Q} "
                      f"{'x'.join(str(v) for v in shape[:dim])} periodic, same recipe and "
                      f"parameters as the headline, {steps} steps ({dt:.1f} s)",
            "cpu_model": cpu_model, "gpu_vs_oracle_max_rel_err": err,
            "single_core": {"value": round(cells1 * steps1 / dt1 / 1e6, 3), "unit": "MLUPS",
                            "cores": 1,
                            "sample": f"same recipe, {'x'.join(str(v) for v in shape1[:dim])}, "
                                      f"{steps1} steps ({dt1:.1f} s)"}}


def tube_accuracy(n=512, seed=4):
    """Part of the oracle leg: every tube of the ensemble recipe against the
    exact Riemann solution (Sec. V's reference) at its comparison step --
    the last step at which every wave of the exact solution is still 10
    cells from an end, at most 1000 -- run in one FP32 pool.  A tube is
    "in range" when every state of its exact solution has 0.7 <= T <= 1.4
    and Mach < 0.8 and no wave outruns the lattice (speed < 3r).  L1 per field
    is relative to the size of that field's jump (rho, p) or to |u*|."""
    import math

    import torch

    from oracle.riemann import RiemannSolution, l1_errors, shock_tube_profile
    from paper_1608_06345_amd import lbm, serving

    rr = lbm.lbm_lattice(37)[2]
    tubes = serving.tube_ensemble(n, steps=1000, seed=seed)
    meta = {}
    for r in tubes:
        left, right = r.tube
        g = r.req.gamma
        sol = RiemannSolution(left, right, g)
        nx = r.req.nx
        x_d = nx // 2
        n_cmp = max(1, min(1000, int((min(x_d, nx - x_d) - 10) * rr / sol.max_speed())))
        states = [left, right, (sol.rho_star_l, sol.u_star, sol.p_star),
                  (sol.rho_star_r, sol.u_star, sol.p_star)]
        temps = [pp / rho for rho, _, pp in states]
        mach = max(abs(u) / math.sqrt(g * pp / rho) for rho, u, pp in states)
        in_range = (min(temps) >= 0.7 and max(temps) <= 1.4 and mach < 0.8
                    and sol.max_speed() < 3 * rr)
        r.req.steps = n_cmp
        meta[r.rid] = (sol, n_cmp, in_range)
    got = {}

    def keep(r, pool, slot):
        rho, u, _ = pool.moments(slot)
        got[r.rid] = (rho, u, pool.temperature(slot))

    budget = sum(lbm.lbm_pool_request_bytes(r.req, lbm.LBM_FP32_DEV) for r in tubes) + (1 << 30)
    serving.serve_pool(tubes, budget, max_slots=600, ticks=50, realtime=False, keep=keep)
    torch.cuda.empty_cache()
    rel_in, rel_all, bad = [], [], 0
    for r in tubes:
        sol, n_cmp, in_range = meta[r.rid]
        rho, u, T = got[r.rid]
        nx = r.req.nx
        if not np.all(np.isfinite(rho[:nx])):
            bad += 1
            continue
        ex = shock_tube_profile(r.tube[0], r.tube[1], r.req.gamma, nx, n_cmp, rr)
        l1 = l1_errors(rho[:nx], u[0][:nx], (rho * T)[:nx], *ex)
        scale = (abs(r.tube[0][0] - r.tube[1][0]), max(1e-3, abs(sol.u_star)),
                 abs(r.tube[0][2] - r.tube[1][2]))
        rel = max(a / sc for a, sc in zip(l1, scale))
        rel_all.append(rel)
        if in_range:
            rel_in.append(rel)

    def stats(v):
        return ({"median": round(float(np.median(v)), 5), "max": round(float(np.max(v)), 5)}
                if v else None)

    return {"tubes": n, "in_range": sum(1 for m in meta.values() if m[2]),
            "non_finite_at_comparison_step": bad,
            "relative_l1_in_range": stats(rel_in), "relative_l1_all_finite": stats(rel_all),
            "normalisation": "each tube's temperatures scaled to geometric mean 1",
            "tau": 0.8, "storage": "FP32 deviation storage",
            "comparison_step": "last step with every exact wave 10 cells from an end (<= 1000)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--path", default="d3q107_fp32", choices=sorted(PATHS))
    ap.add_argument("--no-extra", action="store_true", help="skip the other paths")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the batched tube ensemble and the serving trace")
    ap.add_argument("--serving-requests", type=int, default=96,
                    help="requests in the Poisson serving trace")
    ap.add_argument("--serving-only", choices=("pool", "sequential", "both"), default=None,
                    help="after the headline path, run only the Poisson serving trace with "
                         "these servers (no other paths, no tube ensemble, no CPU baseline)")
    ap.add_argument("--serving-rate", type=float, default=None,
                    help="arrival rate of the serving trace in requests/s (default: 80%% of "
                         "the pool's capacity measured on the same mix)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the HBM copy / read ceiling probe")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes 5 times with the streaming copy of "
                         "libhbmprobe.so (a plain copy kernel of known size, to scale the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import ctypes

        import torch
        lib = ctypes.CDLL(os.path.join(ROOT, "paper_1608_06345_amd", "libhbmprobe.so"))
        lib.hbm_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_int, ctypes.c_void_p]
        n = args.copy_probe // 16 * 16
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):  # variant 2: 4 x 16 B per lane, non-temporal
            rc = lib.hbm_probe_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                    n, 2, None)
            if rc != 0:
                raise RuntimeError(f"hbm_probe_copy: status {rc}")
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 5, "kernel": "k_probe_copy<4, true>"}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    head = PATHS[args.path]
    res = run_path(args.path, head, args.steps, args.warmup)
    print(f"# {args.path}: {res['mlups']} MLUPS, {res['gbs']} GB/s", file=sys.stderr, flush=True)
    paths = {args.path: res}
    if args.serving_only:
        args.no_extra = args.no_cpu = True
    if not args.no_extra:
        for name, p in PATHS.items():
            if name == args.path:
                continue
            paths[name] = run_path(name, p, p["steps"], args.warmup)
            print(f"# {name}: {paths[name]['mlups']} MLUPS, {paths[name]['gbs']} GB/s",
                  file=sys.stderr, flush=True)
    traffic = res["traffic_bytes_per_launch"]
    algo_bytes = res["bytes_per_update"] * res["cells"]
    ceiling = None
    if not args.no_ceiling and not args.serving_only:
        three_d = head["dim"] == 3
        ceiling = hbm_ceiling(algo_bytes, pattern_cells=res["cells"] if three_d else None,
                              pattern_nx=head["shape"][0] if three_d else None)
        print(f"# HBM ceiling: copy {ceiling['copy_gbs']} GB/s, read {ceiling['read_gbs']} GB/s, "
              f"step access pattern {ceiling.get('step_pattern_gbs')} GB/s", file=sys.stderr,
              flush=True)
    out = {
        "metric": "MLUPS (million lattice-cell updates per second)",
        "value": res["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)"}[head["store"]],
        "data": "synthetic",
        "config": {"workload": res["workload"], "grid": list(head["shape"][:head["dim"]]),
                   "velocity_set": f"D{head['dim']}Q{37 if head['dim'] == 2 else 107}",
                   "storage": STORAGE[head["store"]][0],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": res["gbs"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": res["hbm_frac"],
                     # counter-measured HBM bytes per launch over the live
                     # average launch time (null if the kernel changed since)
                     "traffic": (round(traffic / (res["ms_per_step"] * 1e-3) / 1e9, 1)
                                 if traffic else None),
                     "traffic_bytes_per_launch": traffic,
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "bytes_per_update": res["bytes_per_update"],
                     "kernel": "k_step_split (fused pull, moments, equilibrium, relax, store)"},
        "paths": {k: {kk: v[kk] for kk in ("workload", "mlups", "gbs", "hbm_frac",
                                            "ms_per_step", "steps")}
                  for k, v in paths.items()},
    }
    if ceiling:
        # measured in this run, on this device, over as many bytes as one
        # headline launch moves
        out["roofline"].update({
            "copy_gbs": ceiling["copy_gbs"], "read_gbs": ceiling["read_gbs"],
            "frac_of_copy": round(res["gbs"] / ceiling["copy_gbs"], 4),
            "step_pattern_gbs": ceiling.get("step_pattern_gbs"),
            "frac_of_step_pattern": (round(res["gbs"] / ceiling["step_pattern_gbs"], 4)
                                     if ceiling.get("step_pattern_gbs") else None),
            "ceiling_probe": ceiling})
    if args.serving_only:
        servers = ("pool", "sequential") if args.serving_only == "both" else (args.serving_only,)
        out["serving"] = serving_runs(args.serving_requests, servers=servers, ensemble=False,
                                      rate=args.serving_rate)
    elif not args.no_serving:
        out["serving"] = serving_runs(args.serving_requests, rate=args.serving_rate)
    if not args.no_cpu:
        ens = out.get("serving", {}).get("tube_ensemble")
        out["cpu_baseline"] = cpu_baseline(head, out["paths"], tubes=ens is not None)
        if ens is not None:
            ens["accuracy_vs_exact_riemann"] = out["cpu_baseline"].pop("tube_accuracy")
        print("# oracle leg done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
