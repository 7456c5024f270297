"""Host-side checks of bench.py (no GPU): the one-GPU guard, the algorithmic
byte counts its roofline divides by, and the workloads it times."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_cell_update():
    # one read and one write of each of the 2Q stored values (g and h)
    for dim, q in ((2, 37), (3, 107)):
        for store, size in (("fp64", 8), ("fp32", 4), ("fp16", 2)):
            assert bench.bytes_per_update(dim, store) == 2 * q * 2 * size
    assert bench.bytes_per_update(3, "fp32") == 1712
    assert bench.bytes_per_update(2, "fp64") == 1184


def test_headline_and_paths():
    p = bench.PATHS["d3q107_fp32"]
    assert p["dim"] == 3 and p["shape"] == (256, 256, 256) and p["store"] == "fp32"
    assert "D3Q107 256x256x256" in bench.describe("d3q107_fp32", p)
    for name, p in bench.PATHS.items():
        d = bench.describe(name, p)
        assert ("finite-difference" in d) == ("dt" in p)
        assert ("LDS" in d) == (p.get("variant") == "split_lds")
    assert len(bench.kernel_source_hash()) == 16


def test_kernel_hash_follows_code_not_comments():
    code = "int a = 1; // one\n/* block\n comment */\nint b = a / 2;  \n\n"
    assert bench._code_only(code) == "int a = 1;\nint b = a / 2;"
    assert bench._code_only("x /* a */ + /* b */ y") == "x  +  y"
    # a changed comment leaves the code the same, a changed operator does not
    assert bench._code_only(code.replace("one", "two")) == bench._code_only(code)
    assert bench._code_only(code.replace("a / 2", "a * 2")) != bench._code_only(code)
    # the traffic record is used only for the hash of the current sources
    import json
    with open(os.path.join(bench.ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    hashes = {v["kernel_hash"] for v in rec.values() if isinstance(v, dict)}
    assert hashes, "no traffic entries"
    for name, ent in rec.items():
        if isinstance(ent, dict):
            want = ent["bytes_per_launch"] if ent["kernel_hash"] == bench.kernel_source_hash() else None
            assert bench.measured_traffic(name, ent["cells"]) == want


def test_gamma_five_thirds_path_keeps_h():
    p = bench.PATHS["d3q107_fp32_gamma53"]
    assert abs(p["gamma"] - 5.0 / 3.0) < 1e-15 and p["store"] == "fp32"
    assert "delta 0)" in bench.describe("d3q107_fp32_gamma53", p)
    # same bytes per update as gamma 1.4: h is stored and moved in full
    assert bench.bytes_per_update(p["dim"], p["store"]) == 1712


def test_every_path_has_an_accuracy_sample():
    for name, p in bench.PATHS.items():
        key = ("fd" if p.get("dt") else "lattice", p["dim"])
        shape, steps = bench.ACCURACY_SAMPLES[key]
        assert steps > 0 and shape[0] % 128 == 0  # whole tiles for the LDS kernels
        assert (p["dim"] == 2) == (shape[2] == 1)
