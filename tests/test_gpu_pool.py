"""The batched multi-solve pool (serving form) on the GPU.

  * a request's result is bitwise the same alone and in a mix of other
    requests (different dimensions, sizes, gamma, tau, boundaries and step
    counts), with admissions and releases between graph replays;
  * the pool agrees with the single-solve path and with the FP64 oracle;
  * graph replays and eager launches give identical bits;
  * admission control: EBUSY when the arena is full, ENOMEM when a request
    can never fit, EINVAL for invalid requests; released space is reused.
"""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import shear_wave_fields, smooth_fields, sod_fields
from parity_util import TOL_FP32, TOL_FP64, assert_close, oracle_run

pytestmark = pytest.mark.gpu

OPEN_X = lbm.LBM_BC(lbm.LBM_BC_ZERO_GRADIENT, lbm.LBM_BC_PERIODIC)


def _requests():
    """(request, fields) pairs of a small mixed workload."""
    out = []
    r = lbm.make_request(2, 1.4, 0.7, 0.8, 70, 45, steps=23)
    out.append((r, smooth_fields(2, 70, 45, seed=31)))
    r = lbm.make_request(3, 1.4, 0.65, 0.65, 24, 10, 9, steps=17)
    out.append((r, shear_wave_fields(3, 24, 10, 9, seed=32)))
    r = lbm.make_request(2, 1.25, 0.8, 0.8, 300, 4, bc=OPEN_X, steps=40)
    out.append((r, sod_fields(2, 300, 4, left=(1.0, 0.0, 1.2), right=(0.6, 0.0, 0.6))))
    r = lbm.make_request(3, 5.0 / 3.0, 0.7, 0.9, 33, 7, 5, bc=lbm.LBM_BC(1, 0, 1), steps=9)
    out.append((r, smooth_fields(3, 33, 7, 5, seed=34, a_rho=0.03, a_u=0.03, a_T=0.03)))
    r = lbm.make_request(2, 2.0, 0.6, 0.6, 128, 66, steps=31)  # 66 rows: whole-rows-per-XCD order
    out.append((r, shear_wave_fields(2, 128, 66, seed=35)))
    r = lbm.make_request(3, 1.4, 0.65, 0.65, 40, 9, 8, steps=0)  # zero steps: S_0 back
    out.append((r, smooth_fields(3, 40, 9, 8, seed=36)))
    return out


def _run_to_end(pool, slots, ticks, eager=False):
    left = set(slots)
    for _ in range(1000):
        if not left:
            return
        (pool.run_eager if eager else pool.run)(ticks)
        left -= set(pool.poll())
    raise AssertionError("pool did not finish")


def _alone(req, f, precision, ticks=5, eager=False):
    with lbm.Pool(1 << 30, 4, precision) as pool:
        s = pool.admit(req, *f)
        _run_to_end(pool, [s], ticks, eager)
        assert pool.steps_done(s) == req.steps
        return pool.moments(s) + (pool.temperature(s),)


@pytest.mark.parametrize("precision", [lbm.LBM_FP32_DEV, lbm.LBM_FP64])
def test_alone_equals_mix_bitwise(precision):
    reqs = _requests()
    alone = [_alone(r, f, precision) for r, f in reqs]
    with lbm.Pool(2 << 30, 8, precision) as pool:
        # staggered admission: half now, the rest after some replays
        slots = {}
        for k in (0, 1, 2):
            slots[k] = pool.admit(*[reqs[k][0]], *reqs[k][1])
        pool.run(7)
        pool.run(7)
        for k in (3, 4, 5):
            slots[k] = pool.admit(reqs[k][0], *reqs[k][1])
        results = {}
        for _ in range(100):
            if len(results) == len(reqs):
                break
            pool.run(7)
            for s in pool.poll():
                k = [kk for kk, ss in slots.items() if ss == s][0]
                results[k] = pool.moments(s) + (pool.temperature(s),)
                pool.release(s)
        assert len(results) == len(reqs)
    for k, (a, b) in enumerate(zip(alone, [results[i] for i in range(len(reqs))])):
        for x, y in zip(a, b):
            assert np.all(np.isfinite(x)), f"request {k} is not finite"
            assert np.array_equal(x, y), f"request {k} differs between alone and mix"


def test_graph_equals_eager():
    r, f = _requests()[1]
    a = _alone(r, f, lbm.LBM_FP32_DEV, ticks=4, eager=False)
    b = _alone(r, f, lbm.LBM_FP32_DEV, ticks=4, eager=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,tol", [(lbm.LBM_FP64, TOL_FP64), (lbm.LBM_FP32_DEV, TOL_FP32)])
def test_pool_matches_single_solve_and_oracle(precision, tol):
    for req, f in _requests()[:2] + _requests()[4:5]:
        dim = req.dim
        shape = (req.nx, req.ny, req.nz)
        rho, u, E, T = _alone(req, f, precision)
        with lbm.Solver(dim, req.gamma, req.tau_f, req.tau_g, *shape, bc=req.bc,
                        precision=precision) as s:
            s.init_fields(*f)
            s.step(req.steps)
            r2, u2, E2 = s.moments()
            T2 = s.temperature()
        # same kernels' arithmetic: identical to the single-solve path
        assert np.array_equal(rho, r2) and np.array_equal(u, u2) and np.array_equal(E, E2)
        assert np.array_equal(T, T2)
        o = oracle_run(dim, req.gamma, req.tau_f, req.tau_g, shape, f, req.steps)
        assert_close((rho, u, T), o, tol, f"pool D{dim}")


def test_totals_and_info():
    r, f = _requests()[0]
    with lbm.Pool(1 << 30, 4, lbm.LBM_FP64) as pool:
        s = pool.admit(r, *f)
        m0, p0, e0 = pool.totals(s)
        _run_to_end(pool, [s], 6)
        m1, p1, e1 = pool.totals(s)
        assert m1 == pytest.approx(m0, rel=1e-13)
        assert np.allclose(p1, p0, rtol=0, atol=1e-10)
        inf = pool.info()
        assert inf["resident"] == 1 and inf["used_bytes"] == lbm.lbm_pool_request_bytes(r, 0)
        pool.release(s)
        assert pool.info()["resident"] == 0 and pool.info()["used_bytes"] == 0


def test_admission_control():
    req = lbm.make_request(2, 1.4, 0.7, 0.7, 256, 256, steps=5)
    need = lbm.lbm_pool_request_bytes(req, lbm.LBM_FP32_DEV)
    f = smooth_fields(2, 256, 256, seed=1)
    with lbm.Pool(2 * need + need // 2, 16, lbm.LBM_FP32_DEV) as pool:
        a = pool.admit(req, *f)
        b = pool.admit(req, *f)
        assert a is not None and b is not None
        assert pool.admit(req, *f) is None  # arena full: EBUSY
        big = lbm.make_request(2, 1.4, 0.7, 0.7, 1024, 1024, steps=5)
        with pytest.raises(lbm.LBMError) as ei:
            pool.admit(big, *smooth_fields(2, 1024, 1024, seed=1))
        assert ei.value.code == lbm.LBM_ENOMEM
        bad = lbm.make_request(2, 1.4, 0.5, 0.7, 16, 16, steps=5)
        with pytest.raises(lbm.LBMError) as ei:
            pool.admit(bad, *smooth_fields(2, 16, 16, seed=1))
        assert ei.value.code == lbm.LBM_EINVAL
        pool.release(a)
        c = pool.admit(req, *f)  # the released space is reused
        assert c is not None
        _run_to_end(pool, [b, c], 3)
    with lbm.Pool(1 << 24, 1, lbm.LBM_FP32_DEV) as pool:
        small = lbm.make_request(2, 1.4, 0.7, 0.7, 8, 8, steps=1)
        assert pool.admit(small, *smooth_fields(2, 8, 8, seed=1)) is not None
        assert pool.admit(small, *smooth_fields(2, 8, 8, seed=1)) is None  # no free slot
