"""FP64 CPU oracle for the Monte Carlo dust radiative-transfer path.

Test infrastructure: imported only by tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of bench.py. It shares no code with the HIP library.
"""
