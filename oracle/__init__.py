"""CPU oracle for BMMC permutations -- test infrastructure, not the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this folder.  The
GPU library never routes through it; the two share no code.
"""
