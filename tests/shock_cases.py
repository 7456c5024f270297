"""The shock-tube cases that carry an FP32 or FP64 parity bar, and their
bars, shared by the CPU test of the float model (test_f32_model.py) and the
GPU tests (test_gpu_f32_shock.py and the shock-tube tests that use BARS).

A shock front turns the rounding of each step into field differences far
above those on smooth fields (where the bars are 1e-12 in FP64 and 1e-5 in
FP32).  How far depends on the floating-point type and on how each collision
rounds its conserved sums, not on one implementation: the float model of the
step (f32_model.py) evaluates the same arithmetic in five orders (pairwise
and sequential sums, one-ulp perturbations, target sums in float64, and
without the exact-moment fold), and correct evaluations in one type differ
from the oracle -- and from each other -- by up to the amounts recorded
here; in float32 the orders span a factor of 10-15 on each case.  Each bar
is 3-4 times the largest such difference; the CPU test re-measures them and
checks that every bar stays within 2-40x of them.

Metrics: "pointwise" is the largest of max |rho - rho_o| / rho_o,
max |u - u_o| (absolute: the tubes start at rest) and max |T - T_o| / T_o;
"l1" is the largest of sum |q - q_o| / sum |q_o| over q = rho, u, T (used
where 500 steps of rounding move the front by a fraction of a cell, so that
the pointwise difference at the front is of the order of the jump).
"""
R = 1.196979770393074359
SOD_L, SOD_R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
PAPER_L, PAPER_R = (4.0, 0.0, 4.0), (1.0, 0.0, 1.0)   # Sec. V: rho 4 : 1 at T = 1
FD_DT = 0.25 / (3 * R)

# name: (dim, gamma, tau, nx, left, right, steps, dt, metric); left/right are
# (rho, u, p).  The tubes are members 9, 17 and 21 of the shock-tube ensemble
# recipe (seed 4), run to their comparison steps.
CASES = {
    "sod200_48": (2, 1.4, 0.6, 200, SOD_L, SOD_R, 48, None, "pointwise"),
    "sod200_250": (2, 1.4, 0.6, 200, SOD_L, SOD_R, 250, None, "pointwise"),
    "sod1600_500": (2, 1.4, 0.6, 1600, SOD_L, SOD_R, 500, None, "l1"),
    "paper2d_180": (2, 1.4, 2.0 / 3.0, 1000, PAPER_L, PAPER_R, 180, None, "pointwise"),
    "paper3d_180": (3, 1.4, 2.0 / 3.0, 1000, PAPER_L, PAPER_R, 180, None, "pointwise"),
    "fd_sod200": (2, 1.4, 0.1 / R, 200, SOD_L, SOD_R, int(round((48.0 / R) / FD_DT)), FD_DT,
                  "pointwise"),
    "tube9": (2, 1.4852064930121096, 0.8, 613, (3.735840211375961, 0.0, 4.728556680955496),
              (1.0, 0.0, 0.7900593063465324), 200, None, "pointwise"),
    "tube17": (2, 1.6230561764546123, 0.8, 2536, (2.6297612040852387, 0.0, 3.0006220007022053),
               (1.0, 0.0, 0.8764053597786801), 200, None, "pointwise"),
    "tube21": (2, 1.4614293200244985, 0.8, 345, (6.936918056729777, 0.0, 7.165207099675886),
               (1.0, 0.0, 0.9681392261562913), 107, None, "pointwise"),
}

# Largest difference between a correct evaluation and the oracle over the
# model's five orders, per floating-point type, and the bars set from them.
FP32_GAP = {"sod200_48": 2.9e-4, "sod200_250": 8.8e-4, "sod1600_500": 6.6e-4,
            "paper2d_180": 4.5e-5, "paper3d_180": 4.6e-5, "fd_sod200": 6.5e-4,
            "tube9": 1.3e-5, "tube17": 1.2e-5, "tube21": 3.8e-5}
FP64_GAP = {"sod200_48": 2.3e-12, "sod200_250": 2.4e-12, "sod1600_500": 2.1e-12,
            "paper2d_180": 6.9e-13, "paper3d_180": 2.0e-12, "fd_sod200": 6.8e-12,
            "tube9": 4.4e-13, "tube17": 3.6e-13, "tube21": 2.1e-13}
FP32_BAR = {k: 3.5 * v for k, v in FP32_GAP.items()}
FP64_BAR = {k: 4 * v for k, v in FP64_GAP.items()}
