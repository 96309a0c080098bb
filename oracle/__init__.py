"""CPU oracle for the DDQMC propagation step (arXiv:1802.05931).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1802_05931_amd``) and never imports it.

* :mod:`oracle.orc`   -- ctypes binding of the plain C step (``ddqmc_oracle.c``).
* :mod:`oracle.exact` -- the exact Liouvillian (Kronecker form, Sec. III.C) and
  the exact steady state ("solving the linear system", Sec. V) with numpy/scipy.
"""
