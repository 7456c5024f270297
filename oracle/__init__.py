"""FP64 CPU oracle for the thermal lattice Boltzmann scheme with arbitrary
specific-heat ratio (Hu, Zhang & Geng, arXiv:1608.06345).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the serving loop) may import, link or call anything in this
package.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code, table or constant generator with the
HIP path: it derives its own lattice (``lattice.py``), steps the scheme in
plain C (``lbm_oracle.c``) and carries its own exact Riemann solver
(``riemann.py``).

Modules
-------
lattice   Gauss-Hermite lattices D2Q37 / D3Q107 solved in 40-digit arithmetic
          from the Gaussian moment conditions (Sec. IV, Tables I and II).
model     ctypes wrapper of the C stepper: init / step / moments / totals,
          plus the plain per-cell equilibrium and collision for the pins.
riemann   exact solution of the 1D Riemann problem (shock tube, Sec. V).
"""
