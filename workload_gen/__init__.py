"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This module only draws random numbers and lays them out. It holds none of the
pipeline's arithmetic (no transforms, no products, no allocation logic): both the
oracle and the HIP path receive the same bytes from here and compute on their own.

Workloads (shapes follow the pipeline configurations the method is evaluated on):

* two-stage FP32 pipeline: queries X ~ N(0,1) [n,512]; W1 ~ N(0,1/512) [512,512];
  W2 ~ N(0,1/512) [512,10]; weights are [in, out] row-major.
* speech-assistant pipeline: 2000-sample 16 kHz clips = white noise (sigma 0.1) plus
  three sinusoids (f ~ U(100, 7900) Hz, amplitude ~ U(0.1, 1), phase ~ U(0, 2pi));
  MLP 440->2048->2048->2048->4096 with weights N(0, 1/fan_in) rounded to BF16 and
  stored [out, in] (K contiguous).
* Poisson arrival schedules (exponential gaps, integer nanoseconds) and uneven
  request sizes U{1..128}.
* random integer latency / bandwidth / footprint tables for allocator tests.
"""
from __future__ import annotations

import numpy as np

# Keys that separate the random streams of different configurations / purposes.
_STREAMS = {
    "c0_weights": 1, "c0_queries": 2, "c1_audio": 3, "c1_weights": 4,
    "arrivals": 5, "requests": 6, "tables": 7, "predictor": 8, "c4": 9,
    "handoff": 10, "dtree": 11, "artifact": 12,
}


def rng(purpose: str, seed: int = 0, sub: int = 0) -> np.random.Generator:
    """A numpy Generator for (purpose, seed, sub); streams never overlap."""
    return np.random.default_rng(np.random.SeedSequence([seed, _STREAMS[purpose], sub]))


# ---------------------------------------------------------------- two-stage FP32
C0_D_IN, C0_D_HID, C0_D_OUT = 512, 512, 10


def c0_weights(seed: int = 0):
    g = rng("c0_weights", seed)
    w1 = (g.standard_normal((C0_D_IN, C0_D_HID)) / np.sqrt(C0_D_IN)).astype(np.float32)
    w2 = (g.standard_normal((C0_D_HID, C0_D_OUT)) / np.sqrt(C0_D_HID)).astype(np.float32)
    return w1, w2


def c0_queries(n: int, seed: int = 0, first: int = 0) -> np.ndarray:
    """Query vectors [n, 512] FP32; row j depends only on (seed, first + j)."""
    out = np.empty((n, C0_D_IN), np.float32)
    for j in range(n):
        out[j] = rng("c0_queries", seed, first + j).standard_normal(C0_D_IN)
    return out


def c0_queries_fast(n: int, seed: int = 0) -> np.ndarray:
    """Bulk variant (one stream for all rows) for large pools."""
    return rng("c0_queries", seed, 1 << 30).standard_normal((n, C0_D_IN), dtype=np.float32)


# ---------------------------------------------------------------- speech pipeline
C1_RATE = 16000
C1_SAMPLES = 2000
C1_MLP_DIMS = (440, 2048, 2048, 2048, 4096)


def c1_audio(n: int, seed: int = 0, first: int = 0, samples: int = C1_SAMPLES) -> np.ndarray:
    """White noise (sigma 0.1) + 3 random sinusoids per clip, FP32 [n, samples]."""
    t = np.arange(samples, dtype=np.float64) / C1_RATE
    out = np.empty((n, samples), np.float32)
    for j in range(n):
        g = rng("c1_audio", seed, first + j)
        x = 0.1 * g.standard_normal(samples)
        f = g.uniform(100.0, 7900.0, 3)
        a = g.uniform(0.1, 1.0, 3)
        ph = g.uniform(0.0, 2 * np.pi, 3)
        for i in range(3):
            x += a[i] * np.sin(2 * np.pi * f[i] * t + ph[i])
        out[j] = x
    return out


def c1_audio_fast(n: int, seed: int = 0, samples: int = C1_SAMPLES) -> np.ndarray:
    """Vectorised bulk variant for large query pools (one stream for all rows)."""
    g = rng("c1_audio", seed, 1 << 30)
    t = np.arange(samples, dtype=np.float64) / C1_RATE
    x = 0.1 * g.standard_normal((n, samples))
    f = g.uniform(100.0, 7900.0, (n, 3, 1))
    a = g.uniform(0.1, 1.0, (n, 3, 1))
    ph = g.uniform(0.0, 2 * np.pi, (n, 3, 1))
    x += (a * np.sin(2 * np.pi * f * t[None, None, :] + ph)).sum(axis=1)
    return x.astype(np.float32)


def _to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round FP32 to BF16 (nearest-even) and return the 16-bit patterns.

    Used only to *store* generated weights in BF16; values are finite N(0, s)."""
    u = np.array(x32, dtype=np.float32).view(np.uint32)   # a copy we can work in place on
    lsb = (u >> 16) & np.uint32(1)
    u += np.uint32(0x7FFF)          # finite inputs: no 32-bit overflow
    u += lsb
    u >>= 16
    return u.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def c1_mlp_weights(seed: int = 0, dims=C1_MLP_DIMS):
    """List of BF16 weight matrices as uint16 bit patterns, each [out, in]."""
    g = rng("c1_weights", seed)
    ws = []
    for din, dout in zip(dims[:-1], dims[1:]):
        w = g.standard_normal((dout, din), dtype=np.float32)
        w *= np.float32(1.0 / np.sqrt(din))
        ws.append(_to_bf16_bits(w))
    return ws


# ---------------------------------------------------------------- arrivals
def poisson_arrivals_ns(n: int, rate_qps: float, seed: int = 0, sub: int = 0) -> np.ndarray:
    """Arrival times (int64 ns from 0) of a Poisson process with the given rate."""
    gaps = rng("arrivals", seed, sub).exponential(1e9 / rate_qps, n)
    return np.floor(np.cumsum(gaps)).astype(np.int64)


def request_rows(n: int, seed: int = 0, lo: int = 1, hi: int = 128) -> np.ndarray:
    """Uneven request sizes U{lo..hi}."""
    return rng("requests", seed).integers(lo, hi + 1, n).astype(np.int32)


# ---------------------------------------------------------------- embedding tables
def fp16_table(rows: int, dim: int, seed: int = 0) -> np.ndarray:
    """Embedding table N(0,1) stored as FP16 [rows, dim]."""
    g = rng("c4", seed, 1)
    out = np.empty((rows, dim), np.float16)
    step = 1 << 20
    for i in range(0, rows, step):
        out[i:i + step] = g.standard_normal((min(step, rows - i), dim), dtype=np.float32)
    return out


def fp16_table_chunks(rows: int, dim: int, seed: int = 0, base_rows: int = 1 << 20):
    """A large N(0,1) FP16 table, chunk by chunk (yields (first_row, chunk)): one
    seeded block of base_rows N(0,1) rows, and each chunk its rows in a seeded order
    with seeded sign flips (a sign flip keeps N(0,1)), so 10M rows cost one block's
    draws. fp16_table_row_chunk(..) regenerates any one chunk."""
    base = fp16_table(min(rows, base_rows), dim, seed=seed)
    for c0 in range(0, rows, base_rows):
        yield c0, _tiled_chunk(base, rows, dim, seed, c0 // base_rows)


def _tiled_chunk(base, rows, dim, seed, c):
    n = min(base.shape[0], rows - c * base.shape[0])
    if c == 0:
        return base[:n]
    g = rng("c4", seed, 100 + c)
    perm = g.permutation(base.shape[0])[:n]
    flip = (g.integers(0, 2, (n, dim), dtype=np.uint8).astype(np.uint16) << np.uint16(15))
    return (base[perm].view(np.uint16) ^ flip).view(np.float16)


def fp16_table_row_chunk(rows: int, dim: int, seed: int, c: int, base=None, base_rows: int = 1 << 20):
    """Chunk c of fp16_table_chunks (pass `base`, the seeded block, to avoid redrawing it)."""
    if base is None:
        base = fp16_table(min(rows, base_rows), dim, seed=seed)
    return _tiled_chunk(base, rows, dim, seed, c)


def zipf_ids(n: int, per_row: int, n_items: int, s: float = 1.1, seed: int = 0) -> np.ndarray:
    """[n, per_row] int32 ids with Zipf(s) popularity over n_items: ranks drawn by
    inverse CDF of p(r) ~ r^-s on 1..n_items, mapped to rows by a seeded
    permutation so popular rows are scattered."""
    g = rng("c4", seed, 2)
    ranks = np.arange(1, n_items + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** -s)
    cdf /= cdf[-1]
    r = np.searchsorted(cdf, g.random(n * per_row), side="right")
    perm = g.permutation(n_items)
    return perm[np.minimum(r, n_items - 1)].astype(np.int32).reshape(n, per_row)


# ---------------------------------------------------------------- 5-stage (vision + retrieval) pipeline
C4_H, C4_W, C4_C = 56, 56, 64
C4_MLP_DIMS = (64, 1024, 1024)


def c4_feature_maps(n: int, seed: int = 0, h: int = C4_H, w: int = C4_W, c: int = C4_C) -> np.ndarray:
    """N(0,1) feature maps rounded to BF16, bit patterns [n, h, w, c] (NHWC)."""
    g = rng("c4", seed, 10)
    x = g.standard_normal((n, h, w, c), dtype=np.float32)
    return _to_bf16_bits(x)


def c4_conv_weights(seed: int = 0, c: int = C4_C, cout: int = 64) -> np.ndarray:
    """3x3 conv weights N(0, 2/(9 c)) rounded to BF16, bit patterns [cout, 3, 3, c]."""
    g = rng("c4", seed, 11)
    w = g.standard_normal((cout, 3, 3, c), dtype=np.float32) * np.float32(np.sqrt(2.0 / (9 * c)))
    return _to_bf16_bits(w)


# ---------------------------------------------------------------- allocator tables
def random_problem_tables(n_stages: int, n_shares: int, batches, seed: int = 0,
                          sub: int = 0):
    """Integer latency (ns), bandwidth (B/s) and footprint (B) tables shaped like a
    solo profile: latency falls with CU share and grows with batch, plus noise.

    Returns (lat [S,K,nb] int64, bw [S,K,nb] int64, mem [S,nb] int64)."""
    g = rng("tables", seed, sub)
    batches = np.asarray(batches, np.int64)
    nb = len(batches)
    lat = np.empty((n_stages, n_shares, nb), np.int64)
    bw = np.empty((n_stages, n_shares, nb), np.int64)
    mem = np.empty((n_stages, nb), np.int64)
    for s in range(n_stages):
        work = g.uniform(2e3, 2e5)          # ns of work per query on one share step
        fixed = g.uniform(1e3, 2e4)         # ns fixed cost per batch
        byt = g.uniform(1e5, 4e7)           # bytes per batch
        for k in range(n_shares):
            for j, b in enumerate(batches):
                base = fixed + work * b / (k + 1) ** g.uniform(0.6, 1.0)
                lat[s, k, j] = max(1, int(base * g.uniform(0.9, 1.1)))
                bw[s, k, j] = int(byt * (1 + 0.01 * b) * 1e9 / lat[s, k, j])
        for j, b in enumerate(batches):
            mem[s, j] = int(byt + b * g.uniform(1e3, 1e6))
    return lat, bw, mem


# ---------------------------------------------------------------- predictor
def predictor_init(seed: int = 0, dims=(16, 64, 64, 1)):
    """He-normal weights ([in, out] row-major) and zero biases, FP32."""
    g = rng("predictor", seed)
    params = []
    for din, dout in zip(dims[:-1], dims[1:]):
        params.append((g.standard_normal((din, dout)) * np.sqrt(2.0 / din)).astype(np.float32))
        params.append(np.zeros(dout, np.float32))
    return params


def predictor_batch(m: int, seed: int = 0, sub: int = 0, n_in: int = 16):
    """A random regression minibatch (features U(0,1), targets N(10, 1))."""
    g = rng("predictor", seed, 1000 + sub)
    x = g.uniform(0.0, 1.0, (m, n_in)).astype(np.float32)
    y = g.normal(10.0, 1.0, m).astype(np.float32)
    return x, y


# ---------------------------------------------------------------- artifact stages
ARTIFACT_D = 1024                   # words per row
ARTIFACT_P_WORDS = (1024, 4096, 16384)         # p1, p2, p3: 4 / 16 / 64 KiB per row over the host link
ARTIFACT_C_ITERS = (256, 1024, 4096)           # c1, c2, c3: 0.5 / 2 / 8 MFLOP per row
ARTIFACT_M_WORDS = (65536, 262144, 1048576)    # m1, m2, m3: 256 KiB / 1 MiB / 4 MiB per row from HBM


def artifact_words(n: int, seed: int = 0, sub: int = 0) -> np.ndarray:
    """n uniform random uint32 words (artifact queries, tables)."""
    return rng("artifact", seed, sub).integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
