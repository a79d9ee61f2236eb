"""Brute-force solver of Camelot's two allocation problems (test infrastructure only).

Max peak load (Section VII-B, Eq. 1): choose a batch size b, an instance count N_i
and a CU share p_i per stage to maximise the pipeline throughput
    T = min_i N_i * b / L_i(p_i, b)          (queries/s, L_i in seconds)
subject to
    sum_i N_i p_i <= R                        (computational resources)
    sum_i N_i <= I,  1 <= N_i <= I            (instance cap; optionally a lower
                                              bound per stage, e.g. 1 for a stage
                                              that must stay single)
    sum_i N_i bw_i(p_i, b) <= BW              (global-memory bandwidth)
    sum_i N_i M(i, b) <= F                    (global-memory capacity)
    W(b) + sum_i L_i(p_i, b) <= QoS           (latency target)

Minimum resource at load lambda (Section VII-C, Eq. 3): minimise sum_i N_i p_i under
the same constraints plus T >= lambda.

Readings where the paper is loose (each listed in the design notes):
* Eq. 1's b(p_i) is the bandwidth and g(p_i) the stage duration L_i; the latency
  constraint adds the batch-formation wait W(b) (an input per batch size).
* Eq. 3 has no throughput constraint, which would make N_i = 0 optimal; the load
  constraint T >= lambda and N_i >= 1 are added.
* Shares are whole multiples of a CU step (p = (k+1) * step), the table is indexed
  by (stage, share index, batch index); entries <= 0 mark unmeasured points.
* One GPU: Eq. 2's GPU count must be 1, so C = 1 throughout.
* Ties: peak -> larger T, then fewer CUs, then lower latency, then the
  lexicographically smallest (batch index, N_1, k_1, N_2, k_2, ...);
  min -> fewer CUs, then larger T, then lower latency, then lexicographic.

Throughputs are exact rationals (fractions.Fraction) so comparisons are exact.
Pinned in tests/test_oracle_alloc.py by closed forms (proportional shares,
identical stages, a single stage), monotonicity and hand-solved tiny grids.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from fractions import Fraction
from math import gcd
from typing import List, Optional, Sequence

import numpy as np

NS_PER_S = 10 ** 9


@dataclass
class Problem:
    cu_total: int
    cu_step: int
    max_instances: int                 # I
    max_inst_per_stage: int            # search bound for N_i (<= I)
    batches: Sequence[int]
    qos_ns: int
    hbm_bytes_budget: int              # F
    hbm_bw_budget: int                 # BW, bytes/s
    lat_ns: np.ndarray                 # [S, K, nb] int64
    bw_bps: np.ndarray                 # [S, K, nb] int64
    mem_bytes: np.ndarray              # [S, nb] int64
    batch_wait_ns: Optional[Sequence[int]] = None   # W(b) per batch index
    inst_max: Optional[Sequence[int]] = None        # per-stage bound on N_i (default: max_inst_per_stage)

    @property
    def n_stages(self) -> int:
        return int(self.lat_ns.shape[0])

    @property
    def n_shares(self) -> int:
        return self.cu_total // self.cu_step


@dataclass
class Alloc:
    batch: int
    batch_index: int
    n: List[int]
    cu: List[int]
    thr_num: int
    thr_den: int
    lat_ns: int
    cu_used: int
    key: tuple = field(default=(), repr=False)

    @property
    def thr(self) -> Fraction:
        return Fraction(self.thr_num, self.thr_den)


def _stage_options(p: Problem, s: int):
    """(N_i, k_i) choices of stage s: 1 <= N_i <= its instance bound, every share."""
    K = p.n_shares
    if p.lat_ns.shape[1] < K or p.bw_bps.shape[1] < K:
        raise ValueError("tables hold fewer CU shares than cu_total / cu_step")
    nmax = min(p.max_inst_per_stage, p.max_instances)
    if p.inst_max is not None:
        nmax = min(nmax, int(p.inst_max[s]))
    return [(n, k) for n in range(1, nmax + 1) for k in range(K)]


def evaluate(p: Problem, bi: int, choice) -> Optional[Alloc]:
    """Check one point (batch index, ((N_i, k_i) per stage)); None if infeasible."""
    b = int(p.batches[bi])
    wait = int(p.batch_wait_ns[bi]) if p.batch_wait_ns is not None else 0
    cu_used = 0
    inst = 0
    bw = 0
    mem = 0
    lat = wait
    thr = None
    arg = None
    for s, (n, k) in enumerate(choice):
        L = int(p.lat_ns[s, k, bi])
        if L <= 0:
            return None
        share = (k + 1) * p.cu_step
        cu_used += n * share
        inst += n
        bw += n * int(p.bw_bps[s, k, bi])
        mem += n * int(p.mem_bytes[s, bi])
        lat += L
        t = Fraction(n * b * NS_PER_S, L)
        if thr is None or t < thr:
            thr = t
            arg = (n * b * NS_PER_S, L)
    if cu_used > p.cu_total or inst > p.max_instances:
        return None
    if bw > p.hbm_bw_budget or mem > p.hbm_bytes_budget or lat > p.qos_ns:
        return None
    g = gcd(*arg)
    key = (bi,) + tuple(x for nk in choice for x in nk)
    return Alloc(batch=b, batch_index=bi, n=[c[0] for c in choice],
                 cu=[(c[1] + 1) * p.cu_step for c in choice],
                 thr_num=arg[0] // g, thr_den=arg[1] // g,
                 lat_ns=lat, cu_used=cu_used, key=key)


def all_feasible(p: Problem):
    opts = [_stage_options(p, s) for s in range(p.n_stages)]
    for bi in range(len(p.batches)):
        for choice in itertools.product(*opts):
            a = evaluate(p, bi, choice)
            if a is not None:
                yield a


def alloc_peak(p: Problem) -> Optional[Alloc]:
    """Eq. 1 by exhaustive enumeration; None when nothing is feasible."""
    best = None
    for a in all_feasible(p):
        k = (-a.thr, a.cu_used, a.lat_ns, a.key)
        if best is None or k < best[0]:
            best = (k, a)
    return None if best is None else best[1]


def alloc_min(p: Problem, load_num: int, load_den: int) -> Optional[Alloc]:
    """Eq. 3 (+ T >= load) by exhaustive enumeration; None when infeasible."""
    lam = Fraction(load_num, load_den)
    best = None
    for a in all_feasible(p):
        if a.thr < lam:
            continue
        k = (a.cu_used, -a.thr, a.lat_ns, a.key)
        if best is None or k < best[0]:
            best = (k, a)
    return None if best is None else best[1]


def even_split(p: Problem, bi: int) -> Optional[Alloc]:
    """The even-allocation baseline: one instance per stage and the CU steps dealt
    round-robin, so shares differ by at most one step (e.g. 88/88/80 of 256)."""
    S = p.n_stages
    steps = p.n_shares
    per = [steps // S + (1 if s < steps % S else 0) for s in range(S)]
    choice = tuple((1, per[s] - 1) for s in range(S))
    return evaluate(p, bi, choice)


# ---------------------------------------------------------------- simulated annealing
# Section VII-C: Camelot solves both problems by simulated annealing over the vector
# V = [N_1 .. N_S, p_1 .. p_S]; each iteration moves V one step in a random direction,
# rejects a move that breaks a constraint, and otherwise takes it if it improves the
# objective, or with a probability that shrinks as the iterations go on. The best
# valid V seen is the answer. The paper gives neither the move set, the schedule nor
# how the acceptance probability is computed; the readings here (in the design
# notes) are:
# * the state also holds the batch index (batch size is a decision variable); a move
#   changes one coordinate (batch index, one N_i or one share index k_i) by +-1,
#   coordinate and direction uniform; a move off the grid is no move;
# * start: largest batch, N_i = 1, share index K // S - 1 (about an even split);
# * while the current state is invalid, every move is taken (a walk towards the
#   valid region); from a valid state an invalid candidate is rejected;
# * Metropolis acceptance of a worse valid candidate with probability
#   exp(-d / temp), d the relative loss (peak: (T - T') / T; min: (R' - R) / R with R
#   the CUs in use), temp = 0.3 at the start and multiplied by 0.95 every 100
#   iterations;
# * the best state seen is compared with the exhaustive solvers' tie rules;
# * random numbers come from one SplitMix64 stream (splitmix64_next, pinned to the
#   generator's published outputs) seeded with `seed`: per iteration one draw for the
#   coordinate (mod 2S + 1), one for the direction (low bit), and, only when a worse
#   valid candidate is tested, one for u = (draw >> 11) / 2^53.
SA_T0, SA_COOLING, SA_LEVEL = 0.3, 0.95, 100


def simulated_annealing(p: Problem, iters: int, seed: int, load: Optional[Fraction] = None) -> Optional[Alloc]:
    """Eq. 1 (load None) or Eq. 3 at `load` queries/s by simulated annealing; None
    when no valid state was visited."""
    import math
    from oracle.delivery import splitmix64_next

    S, K, nb = p.n_stages, p.n_shares, len(p.batches)
    nmax = []
    for s in range(S):
        m = min(p.max_inst_per_stage, p.max_instances)
        if p.inst_max is not None:
            m = min(m, int(p.inst_max[s]))
        nmax.append(m)
    bi = nb - 1
    n = [1] * S
    k = [max(0, K // S - 1)] * S
    rng = seed & ((1 << 64) - 1)

    def draw():
        nonlocal rng
        rng, out = splitmix64_next(rng)
        return out

    def score(bi_, n_, k_):
        a = evaluate(p, bi_, tuple(zip(n_, k_)))
        if a is not None and load is not None and a.thr < load:
            return None
        return a

    def key(a):
        if load is None:
            return (-a.thr, a.cu_used, a.lat_ns, a.key)
        return (a.cu_used, -a.thr, a.lat_ns, a.key)

    cur = score(bi, n, k)
    best = cur
    temp = SA_T0
    for t in range(iters):
        if t > 0 and t % SA_LEVEL == 0:
            temp *= SA_COOLING
        c = draw() % (2 * S + 1)
        step = 1 if draw() & 1 else -1
        bi2, n2, k2 = bi, list(n), list(k)
        if c == 0:
            bi2 += step
            if not 0 <= bi2 < nb:
                continue
        elif c <= S:
            n2[c - 1] += step
            if not 1 <= n2[c - 1] <= nmax[c - 1]:
                continue
        else:
            k2[c - S - 1] += step
            if not 0 <= k2[c - S - 1] < K:
                continue
        cand = score(bi2, n2, k2)
        if cur is None:
            take = True
        elif cand is None:
            take = False
        else:
            if load is None:
                tc, tn = float(cur.thr), float(cand.thr)
                d = (tc - tn) / tc
            else:
                d = (cand.cu_used - cur.cu_used) / cur.cu_used
            if d <= 0:
                take = True
            else:
                u = (draw() >> 11) / float(1 << 53)
                take = u < math.exp(-d / temp)
        if take:
            bi, n, k, cur = bi2, n2, k2, cand
            if cur is not None and (best is None or key(cur) < key(best)):
                best = cur
    return best
