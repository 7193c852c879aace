"""FP64 CPU oracle of the DARTS hot path. TEST INFRASTRUCTURE: only tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it."""
