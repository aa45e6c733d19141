"""CPU oracle for the tiled hierarchical QR path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls into it and
shares no code with it.

Contents
--------
* :mod:`oracle.qr` -- unblocked double-precision Householder QR (C, via
  ctypes) and helpers built on it (apply Q^T / Q, thin Q, least squares,
  sign normalisation of R).  It is the plain definition of what any tiled
  elimination list computes (Section II: every list has the weight of the
  standard Householder algorithm and yields the same R up to row signs).
* :mod:`oracle.elimlist` -- an independent pure-Python enumeration of the
  elimination lists (reduction trees of Section III and the hierarchical
  composition of Section IV), the validity rules of Section II, the kernel
  expansion of Algorithm 2 and the coarse unit-time step model.
"""
