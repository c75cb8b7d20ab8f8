"""Plain, slow, CPU FP64 oracle for the truncated-Wigner Schrodinger-Poisson ensemble.

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it. The GPU product path never calls into it and shares no code with it.

Modules
-------
philox       Philox4x64-10 counter-based generator (Salmon et al., SC'11)
twa_oracle   Wigner sampling, Strang split-step evolution, ensemble moments
"""
