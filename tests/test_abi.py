"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/lbm.h declares, derives the same lattice as
the oracle (independently), sizes footprints, and rejects invalid arguments
before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1608_06345_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lbm_\w+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert {"lbm_create", "lbm_init_fields", "lbm_step", "lbm_moments"} <= names
    lib = ctypes.CDLL(lbm.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("dim,vs", [(2, 37), (3, 107)])
def test_library_lattice_matches_oracle(dim, vs):
    from oracle.lattice import lattice
    e, w, r = lbm.lbm_lattice(vs)
    lat = lattice(dim)
    assert e.shape == (vs, 3) and abs(r - lat.r) <= 2e-16
    if dim == 2:
        assert np.all(e[:, 2] == 0)
    mine = {tuple(int(a) for a in v[:dim]): x for v, x in zip(e, w)}
    assert len(mine) == vs
    for v, x in zip(lat.e, lat.w):
        assert abs(mine[tuple(int(a) for a in v)] - x) <= 4e-16 * x
    # rest first, then opposite pairs next to each other
    assert np.all(e[0] == 0)
    assert np.all(e[1::2] == -e[2::2])


def test_footprint():
    fp = lbm.lbm_footprint_bytes(3, 107, lbm.LBM_FP32_DEV, 256, 256, 256)
    assert fp >= 2 * 2 * 107 * 256 ** 3 * 4
    assert fp < 1.01 * 2 * 2 * 107 * 256 ** 3 * 4
    assert lbm.lbm_footprint_bytes(3, 107, lbm.LBM_FP64, 256, 256, 256) > 1.99 * fp
    assert lbm.lbm_footprint_bytes(2, 107, 0, 4, 4, 1) == 0
    assert lbm.lbm_footprint_bytes(2, 37, 0, 4, 4, 2) == 0


@pytest.mark.parametrize("args", [
    (2, 107, 1.4, 0.7, 0.7, 8, 8, 1, 0),        # dim / velocity set mismatch
    (3, 37, 1.4, 0.7, 0.7, 8, 8, 8, 0),
    (4, 37, 1.4, 0.7, 0.7, 8, 8, 1, 0),
    (2, 37, 1.4, 0.5, 0.7, 8, 8, 1, 0),         # tau <= 1/2
    (2, 37, 1.4, 0.7, 0.4, 8, 8, 1, 0),
    (2, 37, 1.0, 0.7, 0.7, 8, 8, 1, 0),         # gamma <= 1
    (3, 107, 1.7, 0.7, 0.7, 8, 8, 8, 0),        # delta < 0
    (2, 37, 2.1, 0.7, 0.7, 8, 8, 1, 0),
    (2, 37, 1.4, 0.7, 0.7, 0, 8, 1, 0),         # empty grid
    (2, 37, 1.4, 0.7, 0.7, 8, 8, 2, 0),         # nz != 1 in 2D
    (2, 37, 1.4, 0.7, 0.7, 8, 8, 1, 2),         # unknown bc code
    (2, 37, 1.4, 0.7, 0.7, 8, 8, 1, 1 << 4),    # z bc in 2D
    (2, 37, 1.4, 0.7, 0.7, 8, 8, 1, 1 << 7),
    (3, 107, 1.4, 0.7, 0.7, 1024, 1024, 1024, 0),  # plane beyond 2^31 bytes
])
def test_create_rejects_invalid_arguments(args):
    assert lbm.lbm_create_rc(*args) == lbm.LBM_EINVAL
    assert lbm.lbm_create_rc(*args, precision=lbm.LBM_FP32_DEV) == lbm.LBM_EINVAL


def test_invalid_precision_and_null_handles():
    assert lbm.lbm_create_rc(2, 37, 1.4, 0.7, 0.7, 8, 8, 1, 0, precision=7) == lbm.LBM_EINVAL
    lib = lbm._lib
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_destroy(None) == lbm.LBM_OK
    assert lib.lbm_set_variant(None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_set_collision(None, 1) == lbm.LBM_EINVAL
    assert lbm.lbm_strerror(lbm.LBM_ENONFINITE).startswith("non-finite")
    assert lbm.lbm_strerror(12345) == "unknown status"


R = 1.196979770393074359  # lattice scale; the FD time step is bounded by 1 / (3 r)


@pytest.mark.parametrize("args", [
    (2, 37, 1.4, 0.5, 0.5, 0.0, 8, 8, 1, 0),                # dt = 0
    (2, 37, 1.4, 0.5, 0.5, -0.1, 8, 8, 1, 0),               # dt < 0
    (2, 37, 1.4, 0.5, 0.5, float("nan"), 8, 8, 1, 0),
    (2, 37, 1.4, 0.5, 0.5, 1.0 / (3 * R) * 1.01, 8, 8, 1, 0),  # fastest speed > 1 cell/step
    (3, 107, 1.4, 0.05, 0.5, 0.1, 8, 8, 8, 0),              # dt / tau_f > 1
    (2, 37, 1.4, 0.5, 0.09, 0.1, 8, 8, 1, 0),               # dt / tau_g > 1
    (2, 37, 1.4, 0.0, 0.5, 0.1, 8, 8, 1, 0),                # tau <= 0
    (2, 107, 1.4, 0.5, 0.5, 0.1, 8, 8, 1, 0),               # dim / velocity set mismatch
    (3, 107, 1.7, 0.5, 0.5, 0.1, 8, 8, 8, 0),               # delta < 0
    (2, 37, 1.4, 0.5, 0.5, 0.1, 8, 8, 2, 0),                # nz != 1 in 2D
    (2, 37, 1.4, 0.5, 0.5, 0.1, 8, 8, 1, 2),                # unknown bc code
    (5, 37, 1.4, 0.5, 0.5, 0.1, 8, 8, 1, 0),
])
def test_create_fd_rejects_invalid_arguments(args):
    assert lbm.lbm_create_fd_rc(*args) == lbm.LBM_EINVAL
    assert lbm.lbm_create_fd_rc(*args, precision=lbm.LBM_FP32_DEV) == lbm.LBM_EINVAL
    assert lbm.lbm_create_fd_rc(*args[:6], 8, 8, 1, 0, precision=9) == lbm.LBM_EINVAL


def test_create_fd_refuses_half_storage():
    # valid in every other respect: half storage alone is refused
    assert lbm.lbm_create_fd_rc(2, 37, 1.4, 0.1, 0.1, 0.07, 8, 8, 1, 0,
                                precision=lbm.LBM_FP16_SCALED) == lbm.LBM_EINVAL


def _probe_declared():
    text = open(os.path.join(ROOT, "include", "hbm_probe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hbm_probe_\w+)\s*\(", text, re.M))


def test_hbm_probe_library_exports_and_checks_arguments():
    names = _probe_declared()
    assert {"hbm_probe_copy", "hbm_probe_read", "hbm_probe_variants"} <= names
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1608_06345_amd", "libhbmprobe.so"))
    for n in sorted(names):
        assert hasattr(lib, n), n
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    lib.hbm_probe_copy.argtypes = [vp, vp, sz, i32, vp]
    lib.hbm_probe_read.argtypes = [vp, sz, i32, vp, vp]
    lib.hbm_probe_variant_name.restype = ctypes.c_char_p
    nv = lib.hbm_probe_variants(0)
    assert nv >= 1 and lib.hbm_probe_variants(1) == nv and lib.hbm_probe_variants(2) == -1
    assert lib.hbm_probe_variant_name(0, nv) is None
    # argument checks come before any device call
    assert lib.hbm_probe_copy(None, vp(4096), 1024, 0, None) == -1
    assert lib.hbm_probe_copy(vp(8192), vp(4096), 1000, 0, None) == -1    # not a multiple of 16
    assert lib.hbm_probe_copy(vp(8200), vp(4096), 1024, 0, None) == -1    # misaligned
    assert lib.hbm_probe_copy(vp(4096 + 512), vp(4096), 1024, 0, None) == -1  # overlap
    assert lib.hbm_probe_copy(vp(8192), vp(4096), 1024, nv, None) == -1   # no such variant
    assert lib.hbm_probe_read(vp(4096), 1024, 0, None, None) == -1
    lib.hbm_probe_planes.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, i32, vp]
    big = 1 << 40  # far apart: only the shape checks below can fail
    assert lib.hbm_probe_planes(vp(big), vp(4096), 256 * 4, 256 * 4, 100, None) == -1  # nx % 128
    assert lib.hbm_probe_planes(vp(big), vp(4096), 256 * 4 + 5, 256 * 4 + 5, 256, None) == -1
    assert lib.hbm_probe_planes(vp(big), vp(4096), 256 * 4, 256, 256, None) == -1  # stride < cells
    assert lib.hbm_probe_planes(vp(4096 + 64), vp(4096), 256 * 4, 256 * 4, 256, None) == -1


def test_pool_request_bytes_is_zero_for_any_invalid_request():
    ok = lbm.make_request(3, 1.4, 0.65, 0.65, 16, 16, 16, steps=10)
    assert lbm.lbm_pool_request_bytes(ok, lbm.LBM_FP32_DEV) >= 2 * 2 * 107 * 16 ** 3 * 4
    # gamma 1.67 > 5/3 leaves delta < 0 in 3D (fine in 2D); gamma 5/3 snaps to delta 0
    assert lbm.lbm_pool_request_bytes(
        lbm.make_request(3, 1.67, 0.65, 0.65, 16, 16, 16, steps=10), lbm.LBM_FP32_DEV) == 0
    assert lbm.lbm_pool_request_bytes(
        lbm.make_request(2, 1.67, 0.7, 0.8, 16, 16, steps=10), lbm.LBM_FP32_DEV) > 0
    assert lbm.lbm_pool_request_bytes(
        lbm.make_request(3, 5.0 / 3.0, 0.65, 0.65, 16, 16, 16, steps=10), lbm.LBM_FP32_DEV) > 0
    for bad in (lbm.make_request(2, 1.0, 0.7, 0.8, 16, 16, steps=10),
                lbm.make_request(2, 1.4, 0.5, 0.8, 16, 16, steps=10),
                lbm.make_request(2, 1.4, 0.7, 0.8, 16, 16, steps=-1),
                lbm.make_request(2, 1.4, 0.7, 0.8, 0, 16, steps=10),
                lbm.make_request(2, 1.4, 0.7, 0.8, 16, 16, bc=3, steps=10)):
        assert lbm.lbm_pool_request_bytes(bad, lbm.LBM_FP32_DEV) == 0
