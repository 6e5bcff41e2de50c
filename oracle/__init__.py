"""FP64 CPU oracle of one Hessian-free ray-Born frequency step (arXiv 2211.00316).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the GPU path is
checked against. Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it; the library path never does, and it imports nothing from the GPU package.

Each function follows the passage of the paper it cites, in the paper's order and notation,
with NumPy/SciPy primitives as steps and no blocking, fusion or reordering. Every function
is pinned by a test against a closed form, an invariant, a brute-force sum or a textbook
routine (tests/test_oracle_*.py); the readings taken where the paper is silent are listed in
the module docstrings.

Modules:
  medium  - ring and grid geometry, refractive index, box smoothing, cubic B-spline
  trace   - Hamiltonian ray + paraxial system by Heun's method (Algorithm 1, Section 4)
  binning - ray-to-grid triangulation and receiver tables (Section 4.5, Section 6.3)
  linking - secant ray linking of every emitter-receiver pair (Sections 4 and 6.3)
  green   - ray Green's functions and reciprocal operands (Eqs. 2D_greens, greens-time-reversed)
  born    - Born forward operator, Q=1 adjoint, Hessian-free back-projection (Section 3)
  step    - predicted data, residual, model update, one frequency step, data synthesis
"""
