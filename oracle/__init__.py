"""The oracle: a plain FP64 CPU statement of what the generalized-FDTD hot
path computes, for checking the HIP library.

TEST INFRASTRUCTURE.  Only the test-suite (tests/), the smoke check in
__graft_entry__.smoke() and the CPU-baseline leg of bench.py may import,
call, link or execute anything in this package.  The HIP library and its
Python binding never do; they share no code with it.  Inputs for both come
from the separate `workloads` module, which holds no arithmetic of the
method.

Contents
  stepper    -- C stepper for eq. (10a-d) + Table 1, per-step moving
                profile, soft source, first-order Mur ends, probes with a
                running DFT (oracle/stepper.c, built by oracle/build.py).
  stepper2d  -- the same scheme in 2D, TE and TM, interfaces normal to v
                (oracle/stepper2d.c).
  stability  -- 2x2 amplification matrix of one step (Section 5, App. A).
  analytic   -- Doppler factors, interface and slab closed forms, a
                transfer-matrix method (App. B).

Each function is pinned by tests/test_oracle_*.py against what the paper
prints or what mathematics fixes; see those tests for the pins.
"""
from . import analytic, stability, stepper2d  # noqa: F401
from .stepper import solve, solve_many  # noqa: F401
