"""FP64 CPU oracle for the kernel-compensated MFD band solve.

TEST INFRASTRUCTURE ONLY: used by tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product path never imports it, and
it shares no code with the HIP library.
"""
