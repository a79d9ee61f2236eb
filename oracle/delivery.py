"""Exactly-once, in-order delivery check for pipeline queries (test infrastructure).

Every query carries a 64-bit id, strictly increasing in submit order. A pipeline
delivers correctly when (i) the drained ids are exactly the submitted ids, each
once, and (ii) they come out in submit order. The device side additionally sums
a hash of every id that crosses each stage boundary, with wrap-around addition
and with XOR; both reductions are order-independent, so their expected values
are exact integers.

The hash is the output function of SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) applied to
id + 0x9E3779B97F4A7C15, i.e. the first output of a SplitMix64 generator seeded
with the id. Pinned by the generator's published first outputs
(tests/test_oracle_misc.py, fixture tests/golden/splitmix64.txt).
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_next(state: int):
    """One SplitMix64 step: returns (new_state, output)."""
    state = (state + GOLDEN_GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def id_hash(qid: int) -> int:
    """First SplitMix64 output for seed = qid."""
    return splitmix64_next(qid & MASK64)[1]


def checksums(ids):
    """(sum of hashes mod 2^64, xor of hashes) over an iterable of ids."""
    s = 0
    x = 0
    for q in ids:
        h = id_hash(int(q))
        s = (s + h) & MASK64
        x ^= h
    return s, x


def check_delivery(submitted, drained):
    """Return a list of problems (empty when delivery was exactly-once, in order)."""
    submitted = [int(q) for q in submitted]
    drained = [int(q) for q in drained]
    problems = []
    seen = set()
    dups = set()
    for q in drained:
        if q in seen:
            dups.add(q)
        seen.add(q)
    if dups:
        problems.append(f"duplicated ids: {sorted(dups)[:10]}")
    sub_set = set(submitted)
    lost = sub_set - seen
    extra = seen - sub_set
    if lost:
        problems.append(f"lost ids: {sorted(lost)[:10]} ({len(lost)} total)")
    if extra:
        problems.append(f"unknown ids: {sorted(extra)[:10]}")
    if not problems and drained != submitted:
        first = next(i for i, (a, b) in enumerate(zip(drained, submitted)) if a != b)
        problems.append(f"order differs first at position {first}")
    return problems
