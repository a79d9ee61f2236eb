"""Latency statistics and timing invariants (test infrastructure only).

Tail latency is the quantity the paper's QoS target bounds (the 99%-ile latency,
Section VIII-A). Percentiles use the nearest-rank definition: the q-quantile of n
sorted values is the ceil(q n)-th smallest.

Per query, with arrival a, stage i start s_i / end e_i and completion d:
    d - a = sum_i [(s_i - e_{i-1}) + (e_i - s_i)] + (d - e_last),  e_0 := a
The identity is exact by telescoping; the invariant checked on device timestamps
is that every term is non-negative and the sum reproduces the latency.
Pinned by hand-computed cases and a brute-force check of the rank rule.
"""
from __future__ import annotations

import math


def nearest_rank(values, q: float):
    """The ceil(q n)-th smallest value (q in (0, 1])."""
    v = sorted(values)
    if not v:
        raise ValueError("empty sample")
    r = math.ceil(q * len(v))
    return v[max(r, 1) - 1]


def latency_terms(arrival, starts, ends, done):
    """Queue and service terms for one query; returns (queues, services, egress)."""
    queues, services = [], []
    prev = arrival
    for s, e in zip(starts, ends):
        queues.append(s - prev)
        services.append(e - s)
        prev = e
    return queues, services, done - prev


def check_latency_identity(arrival, starts, ends, done):
    """True when every term is >= 0 and the terms sum to done - arrival."""
    q, s, g = latency_terms(arrival, starts, ends, done)
    terms = q + s + [g]
    return all(t >= 0 for t in terms) and sum(terms) == done - arrival
