"""CPU FP64 oracle for the overlap / Wess-Zumino hot path.

TEST INFRASTRUCTURE ONLY: loaded by the tests, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports it.
"""
