"""MI355X-native DMC hot path (Slater-Jastrow, Gaussian LCAO orbitals).

The compute path is the C-ABI library ``libdmcx.so`` built from ``csrc/``
(hand-written HIP for gfx950); ``dmcx`` is its thin ctypes binding and
``synth`` draws the seeded synthetic inputs.  Importing this package loads
nothing; ``dmcx.load()`` loads the library and fails loudly if it is absent.
"""
