"""Plain FP64 CPU oracle for the localized FBSDE / local-linear-regression scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, constants or helpers with the HIP
library under ``paper_2510_02635_amd/csrc``; the two meet only through the
seeded inputs that a test hands to both.

Modules
  philox    -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror,
               Shaw, SC'11) and the Box-Muller normal transform, written from
               their published definitions.
  scheme    -- the time-stepping scheme: Euler-Maruyama particles (paper
               Sec. 2.3, eq. Xk), kernel-weighted ridge local linear regression
               for the gradient (Sec. 2.4, eqs. leastsq / Dj / normal-eq, ridge
               remark), scalar Newton for Y (Sec. 2.5, eqs. nonlinearf /
               NRiter), Algorithm 1's driver, and a hand-written reverse mode.
  colehopf  -- independent reference values: the Cole-Hopf expectation for the
               HJB case by 2-D quadrature, and the heat-equation closed form.

Every function is FP64, evaluates the definition directly (dense direct
solves, no Krylov iteration, no blocking or fusion), and cites the passage of
the paper it follows.
"""
