"""CPU oracle for scanline DP, RMS and EDP (Mozerov, arXiv 1410.7922).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call or link anything in
this directory.  The product library never routes through it, and it shares
no code with the GPU path: it reads the seeded inputs of ``synth`` and
nothing else.

* ``edp_ref``  -- plain numpy / Python: the definitions (straightforward
  minimum search, brute-force DP, exhaustive enumeration, literal EDP).
* ``dsi_ref``  -- numpy: the data cost of Sec. 2 eq. Cost_value and the
  composite three-view cost of Sec. 5.1 eq. Cost_cmp.
* ``cref``     -- ctypes wrapper of ``edp_oracle.c``, the same definitions in
  plain C for full-size workloads (built by ``__graft_entry__.build()``).
"""
