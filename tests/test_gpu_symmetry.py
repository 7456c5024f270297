"""Translation invariance on the GPU: on a periodic grid, shifting the
initial fields by whole cells shifts the state after n steps by the same
cells, bit for bit (every cell runs the same arithmetic).  It exercises the
pull indexing, the workgroup-to-tile mappings and the LDS-staged kernels,
whose tiles, halos and sub-bands all move relative to the data."""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import smooth_fields
from parity_util import gpu_run

pytestmark = pytest.mark.gpu

R = lbm.lbm_lattice(37)[2]
AUTO, LANE, SPLIT = lbm.LBM_VARIANT_AUTO, lbm.LBM_VARIANT_LANE, lbm.LBM_VARIANT_SPLIT
TWO, LDS = lbm.LBM_VARIANT_TWO_PASS, lbm.LBM_VARIANT_SPLIT_LDS


def _roll(fields, shape, shift):
    nx, ny, nz = shape
    sx, sy, sz = shift
    out = []
    for a in fields:
        lead = a.shape[:-1]
        g = a.reshape(lead + (nz, ny, nx))
        g = np.roll(g, (sz, sy, sx), axis=(-3, -2, -1))
        out.append(g.reshape(lead + (-1,)))
    return out


@pytest.mark.parametrize("dim,shape,variant,precision,dt", [
    (3, (48, 10, 6), AUTO, lbm.LBM_FP32_DEV, None),
    (3, (128, 6, 5), LDS, lbm.LBM_FP32_DEV, None),
    (3, (40, 7, 9), SPLIT, lbm.LBM_FP16_SCALED, None),
    (2, (96, 40, 1), AUTO, lbm.LBM_FP64, None),
    (2, (256, 12, 1), TWO, lbm.LBM_FP32_DEV, 0.25 / (3 * R)),
    (3, (256, 5, 4), TWO, lbm.LBM_FP64, 0.3 / (3 * R)),
    (3, (30, 8, 7), SPLIT, lbm.LBM_FP64, 0.3 / (3 * R)),
])
def test_translation_is_bitwise(dim, shape, variant, precision, dt):
    shift = (5, 3, 2) if dim == 3 else (5, 3, 0)
    tau = (0.65, 0.75) if dt is None else (0.12, 0.14)
    f = smooth_fields(dim, *shape, seed=31, a_rho=0.05, a_u=0.05, a_T=0.05)
    fs = _roll(f, shape, shift)
    a = gpu_run(dim, 1.4, *tau, shape, f, 20, precision=precision, variant=variant, dt=dt)
    b = gpu_run(dim, 1.4, *tau, shape, fs, 20, precision=precision, variant=variant, dt=dt)
    for x, y in zip(_roll(list(a[:3]), shape, shift), b[:3]):
        assert np.array_equal(x, y)
