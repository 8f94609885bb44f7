"""FP64 CPU oracle of the burst merge -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the HIP path.
The reference implementation lives in ``oracle.merge``.
"""
