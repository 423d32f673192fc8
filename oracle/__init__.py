"""CPU oracle for the core-level BSE solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy code written from the paper (Gilmore et al., "Efficient
implementation of core-excitation Bethe-Salpeter equation calculations",
sections 2 and 3.2) to check the GPU library against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU library (``paper_1601_07728_amd``)
and never imports it; the only module both sides use is ``synth`` (seeded input
generation, which holds none of the method's arithmetic).

Modules:
  bse        H*v (Algorithm 1 and the local term), dense H, Haydock, continued fraction
  multiplet  spin-orbit, Slater/Gaunt short-range matrices and dipole amplitudes (quadrature)
  mlp        reference MLP forward/backward/Adam for the learned terminator
"""
