"""Reference (oracle) implementation of the phase-field lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow CPU restatement of
the method of Zhang, Liang & Guo, "On the formulations of interfacial force in
the phase-field-based lattice Boltzmann method" (arXiv:2012.14729).  Only the
test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The HIP library never calls it, and it shares no
code, tables or helpers with the HIP library.

Modules
-------
lbm_ref : vectorised torch-CPU stepper (float64 by default; also runs in
          float32 to measure the single-precision floor, and in complex128
          for complex-step derivatives; autograd through it is the oracle's
          adjoint).
brute   : per-cell, per-direction pure-Python loops for tiny grids, written
          independently of ``lbm_ref`` to pin its vectorisation.
"""
