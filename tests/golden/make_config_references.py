"""Writes the oracle's values for the benchmark's smooth-field
configurations at their full step counts, for the GPU parity tests
(tests/test_gpu_config_recipes.py).  Test infrastructure: it runs only the
FP64 oracle (oracle/) on the seeded input recipe (paper_1608_06345_amd/
inputs.py, which holds no method arithmetic).

Cases (recipe A12: 8 seeded modes per field, 1 <= max|k| <= 8, amplitudes
0.01 in rho and T and 0.02 in u):
  config2_4096       D2Q37 4096^2 periodic, seed 2, gamma 1.4, tau_f 0.7,
                     tau_g 0.8, 1000 steps: the configuration itself;
  config3_g14, _g53  D3Q107 periodic, seed 3, tau 0.65, gamma 1.4 and 5/3,
                     500 steps, on 128 x 64 x 256.  The configuration's
                     256^3 needs ~60 GB and ~40 core-hours of the oracle;
                     this grid keeps the recipe, the parameters and the step
                     count, and is shaped so that seed 3's velocity modes
                     (all with |k| >= 3) keep max |u| at ~5e-3 after 500
                     steps (on 64^3-96^3 they decay to 1e-4 - 1e-7).

Each file holds the parameters, the oracle's max |u| and extremes over the
whole grid, the totals, and rho, u, T at 1024 seeded random cells plus the
cells where |u_k|, rho and T reach their extremes.

Usage: python tests/golden/make_config_references.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CASES = {
    "config2_4096": dict(dim=2, shape=(4096, 4096, 1), gamma=1.4, tf=0.7, tg=0.8, seed=2,
                         steps=1000),
    "config3_g14": dict(dim=3, shape=(128, 64, 256), gamma=1.4, tf=0.65, tg=0.65, seed=3,
                        steps=500),
    "config3_g53": dict(dim=3, shape=(128, 64, 256), gamma=5.0 / 3.0, tf=0.65, tg=0.65, seed=3,
                        steps=500),
}
N_SAMPLES = 1024


def path_of(name):
    return os.path.join(HERE, f"{name}.txt")


def sample_cells(rho, u, T, seed=12345):
    n = rho.size
    rng = np.random.default_rng(seed)
    cells = set(int(c) for c in rng.choice(n, size=N_SAMPLES, replace=False))
    for a in (rho, T, *u):
        cells.add(int(np.argmax(a)))
        cells.add(int(np.argmin(a)))
    return sorted(cells)


def make(name):
    from oracle.model import OracleLBM
    from paper_1608_06345_amd.inputs import smooth_fields
    c = CASES[name]
    f = smooth_fields(c["dim"], *c["shape"], seed=c["seed"])
    o = OracleLBM(c["dim"], c["gamma"], c["tf"], c["tg"], *c["shape"])
    o.init_fields(*f)
    del f
    t0 = time.perf_counter()
    o.step(c["steps"])
    dt = time.perf_counter() - t0
    rho, u, E = o.moments()
    T = o.temperature(u, E)
    mass, mom, energy = o.totals()
    cells = sample_cells(rho, u, T)
    tmp = path_of(name) + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(f"# {name}: FP64 oracle, written by tests/golden/make_config_references.py\n")
        for k in ("dim", "shape", "gamma", "tf", "tg", "seed", "steps"):
            fh.write(f"# {k} = {c[k]!r}\n")
        fh.write(f"# max_abs_u = {float(np.max(np.abs(u))).hex()}\n")
        fh.write(f"# rho_range = {float(rho.min()).hex()} {float(rho.max()).hex()}\n")
        fh.write(f"# T_range = {float(T.min()).hex()} {float(T.max()).hex()}\n")
        fh.write(f"# totals = {float(mass).hex()} "
                 f"{' '.join(float(v).hex() for v in mom)} {float(energy).hex()}\n")
        fh.write(f"# oracle_seconds = {dt:.1f} threads = {os.environ.get('OMP_NUM_THREADS', '')}\n")
        fh.write("# cell rho u_0 .. u_{dim-1} T (float hex)\n")
        for cell in cells:
            vals = [rho[cell]] + [u[k][cell] for k in range(c["dim"])] + [T[cell]]
            fh.write(f"{cell} " + " ".join(float(v).hex() for v in vals) + "\n")
    os.replace(tmp, path_of(name))
    print(f"{name}: {len(cells)} cells, oracle {dt:.0f} s, max|u| {np.max(np.abs(u)):.3e}",
          flush=True)


def load(name):
    """(params, meta, cells [n], values [n][dim + 2]) of a written case."""
    meta = {}
    rows = []
    with open(path_of(name)) as fh:
        for line in fh:
            if line.startswith("#"):
                if " = " in line:
                    k, v = line[2:].split(" = ", 1)
                    meta[k.strip()] = v.strip()
                continue
            parts = line.split()
            rows.append([int(parts[0])] + [float.fromhex(p) for p in parts[1:]])
    cells = np.array([r[0] for r in rows], dtype=np.int64)
    vals = np.array([r[1:] for r in rows], dtype=np.float64)
    return CASES[name], meta, cells, vals


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        make(name)
