"""CPU oracle for the Camelot hot path: plain, slow, obviously-correct FP64 code.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
anything under this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP path
(the only common dependency is ``workload_gen``, which draws seeded inputs).

Modules
-------
stages     stage math of the synthetic microservices (FP64 unless a rounding point
           is part of the definition)
delivery   exactly-once / in-order delivery check with splitmix64 id checksums
alloc      brute-force solver of the max-peak-load problem (Eq. 1) and the
           minimum-resource problem (Eq. 3), integer-exact
predictor  FP64 forward/backward/Adam of the learned contention predictor
stats      nearest-rank percentiles and the latency telescoping identity

Parity status of each function is stated in its module header.
"""
