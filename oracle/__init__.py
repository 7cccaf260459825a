"""CPU oracle for the pTEBD layer (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import
anything from this package.  It never imports the GPU package and the GPU package never
imports it.
"""
