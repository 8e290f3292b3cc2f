"""Plain CPU FP64 oracle for the two-temperature radiative cooling step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or execute this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, header, table or constant with the HIP path: every formula
here is written out again from the paper (Section II for the rates, Section
III.B for the source step) in NumPy/SciPy double precision, slow and plain, so
that a reader can check it against the paper by eye.

Modules
-------
constants  CODATA-2018 cgs constants and the fit coefficients printed in the paper.
physics    closed-form rates: bremsstrahlung (II.A), synchrotron with
           self-absorption (II.B), Compton enhancement (II.C), optically-thick
           bridge (II.D), Coulomb exchange (II.G).
tables     log-spaced node grids, table construction, the FP32 storage form and
           multilinear interpolation (II.F / III.A).
step       rates at a cell, the backward-Euler implicit update and the 16-substep
           explicit update with the 30 % limiter (III.B.1), floor (III.B.2).
grad       gradient of the radiated energy through the implicit update.
finegrid   brute-force references on tiny inputs: a fine 2-D scan of the
           implicit equations and a many-substep RK4 integration.

Parity status of each function is stated in its module header.
"""
