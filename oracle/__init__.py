"""Plain FP64 CPU oracle for the restricted additive Vanka (RAV) multigrid.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package; only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` do.  It shares no code with the HIP library:
the two meet only in the seeded draws of ``rav_inputs``.

The oracle follows the paper (Saberi, Meschke, Vogel, "A restricted additive
Vanka smoother for geometric multigrid", arXiv 2103.10127) step by step:

* ``fem``        Q2/Q1 reference-element quantities, 3-point Gauss (Sec. 2, eqs. 5-7)
* ``grid``       uniform-grid DoF numbering and Dirichlet masks (eq. 6 ordering [u; p])
* ``assemble``   global block system [[A, B], [B^T, 0]] and right-hand side (eqs. 6-7)
* ``mms``        divergence-free manufactured solutions and their forcing (eq. 1)
* ``transfer``   nested-space interpolation P and restriction P^T (Sec. 2, Fig. 1)
* ``patches``    Vanka subdomains, restricted (owned) sets, colours (Sec. 3)
* ``smoothers``  MV (eq. 11), AV (eq. 12), RAV (eq. 13), fixed-point form (eq. 10)
* ``mg``         V-cycle, coarse direct solve, solve to a residual reduction (Sec. 2, 4)
* ``learned``    per-patch damping network and two-grid loss (extension of the
                 diagonal weighting omega_i of eq. 11)

Parity status of each function is given in its docstring; functions with no
external pin say "parity unpinned".
"""
