"""Plain FP64 CPU oracle of the MSM -- TEST INFRASTRUCTURE ONLY.

May be imported only by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; the product library never touches it.
"""
