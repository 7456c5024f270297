"""The shock-tube cases that carry an FP32 or FP64 parity bar, and their
bars, shared by the CPU test of the float model (test_f32_model.py) and the
GPU test (test_gpu_f32_shock.py).

A shock front turns the rounding of each step into field differences far
above those on smooth fields (where the bars are 1e-12 in FP64 and 1e-5 in
FP32).  How far is a property of the floating-point type, not of one
implementation: the float model of the step (f32_model.py) evaluates the
same arithmetic in several orders, and correct evaluations in one type
differ from the oracle -- and from each other -- by the amounts recorded
here.  Each bar is a few times the largest such difference; the CPU test
re-measures the differences and checks that every bar stays within 2-40x of
them (so a bar can neither hide a real defect behind a wide margin nor sit
inside the rounding noise).

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

# name: (dim, gamma, tau, nx, left, right, steps, dt, metric)
CASES = {
    "sod200_48": (2, 1.4, 0.6, 200, SOD_L, SOD_R, 48, None, "pointwise"),
    "sod200_250": (2, 1.4, 0.6, 200, SOD_L, SOD_R, 250, None, "pointwise"),
    "sod1600_500": (2, 1.4, 0.6, 1600, SOD_L, SOD_R, 500, None, "l1"),
    "paper2d_180": (2, 1.4, 2.0 / 3.0, 1000, PAPER_L, PAPER_R, 180, None, "pointwise"),
    "paper3d_180": (3, 1.4, 2.0 / 3.0, 1000, PAPER_L, PAPER_R, 180, None, "pointwise"),
    "fd_sod200": (2, 1.4, 0.1 / R, 200, SOD_L, SOD_R, int(round((48.0 / R) / FD_DT)), FD_DT,
                  "pointwise"),
}

# Largest difference between a correct evaluation and the oracle, measured
# with the float model (float32: pairwise, sequential and perturbed orders;
# float64 likewise), and the bars set from them.
FP32_GAP = {"sod200_48": 8.9e-5, "sod200_250": 7.8e-5, "sod1600_500": 7.4e-5,
            "paper2d_180": 1.3e-5, "paper3d_180": 1.3e-5, "fd_sod200": 8.9e-5}
FP64_GAP = {"sod200_48": 3.8e-13, "sod200_250": 1.7e-12, "sod1600_500": 1.0e-12,
            "paper2d_180": 6.9e-13, "paper3d_180": 2.1e-12, "fd_sod200": 1.2e-12}
FP32_BAR = {k: 4 * v for k, v in FP32_GAP.items()}
FP64_BAR = {k: 4 * v for k, v in FP64_GAP.items()}
