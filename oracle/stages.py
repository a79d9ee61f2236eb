"""FP64 stage math of the synthetic microservice stages (test infrastructure only).

The paper leaves the microservices' internals to third-party models (Section III,
Table I); the stages here are the synthetic stand-ins the pipeline is measured on.
Each function states its definition; where the definition has rounding points
(BF16 activations), they are part of the definition and are applied here too.

Pins (tests/test_oracle_stages.py): DFT vs a library real FFT and Parseval;
bin-centred pure tone amplitude; mel partition of unity; identity-weight GEMM;
brute-force top-k; BF16 rounding of exactly representable and halfway values.
"""
from __future__ import annotations

import math

import numpy as np

# ----------------------------------------------------------------- FP32 GEMM stages


def gemm_relu(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Y = max(0, X W) in FP64; X [B, K], W [K, N] ([in, out] row-major)."""
    y = np.asarray(x, np.float64) @ np.asarray(w, np.float64)
    return np.maximum(y, 0.0)


def argmax_lowest(s: np.ndarray) -> np.ndarray:
    """Row-wise argmax; equal maxima resolve to the lowest column index."""
    s = np.asarray(s)
    out = np.empty(s.shape[0], np.int32)
    for r in range(s.shape[0]):
        best = 0
        for c in range(1, s.shape[1]):
            if s[r, c] > s[r, best]:
                best = c
        out[r] = best
    return out


def gemm_argmax(y: np.ndarray, w: np.ndarray):
    """Scores S = Y W (FP64) and their row argmax (lowest index on ties)."""
    s = np.asarray(y, np.float64) @ np.asarray(w, np.float64)
    return s, argmax_lowest(s)


# ----------------------------------------------------------------- BF16 rounding


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round real values to the nearest BF16 number, ties to even (FP64 in/out).

    BF16 keeps 8 significant bits. For |x| in [2^e, 2^(e+1)) the spacing is
    2^(e-7); numpy's round() rounds halves to even, which on the integer
    significand is round-half-to-even. Values here stay far from the BF16
    overflow/underflow limits (asserted)."""
    x = np.asarray(x, np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # guard log2 rounding at exact powers of two
    e = np.where(2.0 ** e > ax, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= ax, e + 1, e)
    assert np.all(e > -126) and np.all(e < 127), "value outside the normal BF16 range"
    ulp = 2.0 ** (e - 7)
    out[nz] = np.sign(x[nz]) * np.round(ax / ulp) * ulp
    return out


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Decode BF16 bit patterns (uint16) into FP64 values."""
    b = np.asarray(bits, np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


# ----------------------------------------------------------------- BF16 MLP chain


def mlp_bf16(x: np.ndarray, weights_bf16_bits) -> np.ndarray:
    """MLP chain with BF16 weights and BF16 activations, FP64 accumulation.

    h0 = bf16(x); h_l = bf16(max(0, h_{l-1} W_l^T)) for the hidden layers;
    y = h_{L-1} W_L^T returned unrounded. W_l are [out, in] BF16 bit patterns."""
    h = bf16_round(np.asarray(x, np.float64))
    ws = [bf16_bits_to_f64(w) for w in weights_bf16_bits]
    for li, w in enumerate(ws):
        a = h @ w.T
        if li + 1 < len(ws):
            h = bf16_round(np.maximum(a, 0.0))
        else:
            h = a
    return h


# ----------------------------------------------------------------- top-k


def topk(s: np.ndarray, k: int):
    """Per row: the k largest values in descending order, equal values ordered by
    ascending index. Returns (idx int32 [B,k], val [B,k])."""
    s = np.asarray(s)
    B, n = s.shape
    idx = np.empty((B, k), np.int32)
    val = np.empty((B, k), s.dtype)
    for r in range(B):
        order = sorted(range(n), key=lambda c: (-float(s[r, c]), c))[:k]
        idx[r] = order
        val[r] = s[r, order]
    return idx, val


# ----------------------------------------------------------------- log-mel front end

SAMPLE_RATE = 16000
FRAME_LEN = 400          # 25 ms
FRAME_HOP = 160          # 10 ms
N_FRAMES = 11            # 11 x 40 = 440 features per query
N_FFT = 512
N_BINS = N_FFT // 2 + 1  # 257
N_MELS = 40
LOG_FLOOR = 1e-10


def hamming(n: int = FRAME_LEN) -> np.ndarray:
    """Symmetric Hamming window 0.54 - 0.46 cos(2 pi i / (n - 1))."""
    i = np.arange(n, dtype=np.float64)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * i / (n - 1))


def dft_direct(frame: np.ndarray, n_fft: int = N_FFT) -> np.ndarray:
    """X_k = sum_n x_n exp(-2 pi i k n / n_fft), k = 0..n_fft/2, by the direct sum
    (the frame is implicitly zero-padded to n_fft)."""
    x = np.asarray(frame, np.float64)
    n = np.arange(x.shape[0], dtype=np.float64)
    out = np.empty(n_fft // 2 + 1, np.complex128)
    for k in range(n_fft // 2 + 1):
        ang = -2.0 * np.pi * k * n / n_fft
        out[k] = np.sum(x * np.cos(ang)) + 1j * np.sum(x * np.sin(ang))
    return out


def hz_to_mel(f):
    return 2595.0 * np.log10(1.0 + np.asarray(f, np.float64) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, np.float64) / 2595.0) - 1.0)


def mel_filterbank() -> np.ndarray:
    """[40, 257] triangular filters: 42 points equally spaced on the HTK mel scale
    over 0..8000 Hz; filter m rises linearly from point m to point m+1 and falls to
    point m+2, evaluated at the bin frequencies k * 16000 / 512."""
    pts = mel_to_hz(np.linspace(hz_to_mel(0.0), hz_to_mel(SAMPLE_RATE / 2), N_MELS + 2))
    fk = np.arange(N_BINS, dtype=np.float64) * SAMPLE_RATE / N_FFT
    fb = np.zeros((N_MELS, N_BINS))
    for m in range(N_MELS):
        lo, c, hi = pts[m], pts[m + 1], pts[m + 2]
        for k in range(N_BINS):
            f = fk[k]
            if lo <= f <= c:
                fb[m, k] = (f - lo) / (c - lo)
            elif c < f <= hi:
                fb[m, k] = (hi - f) / (hi - c)
    return fb


def log_mel(audio: np.ndarray) -> np.ndarray:
    """[B, 2000] clips -> [B, 440] features: 11 frames of 400 samples (hop 160),
    Hamming window, 512-point DFT power spectrum, 40 mel energies,
    ln(max(E, 1e-10)); layout frame-major (feature = frame * 40 + mel)."""
    audio = np.asarray(audio, np.float64)
    win = hamming()
    fb = mel_filterbank()
    B = audio.shape[0]
    out = np.empty((B, N_FRAMES * N_MELS))
    for b in range(B):
        for f in range(N_FRAMES):
            seg = audio[b, f * FRAME_HOP: f * FRAME_HOP + FRAME_LEN] * win
            X = dft_direct(seg)
            p = X.real ** 2 + X.imag ** 2
            e = fb @ p
            out[b, f * N_MELS:(f + 1) * N_MELS] = np.log(np.maximum(e, LOG_FLOOR))
    return out


# ----------------------------------------------------------------- embedding gather


def gather_mean(ids: np.ndarray, table: np.ndarray) -> np.ndarray:
    """Per row: the mean over its ids of table[id] (FP64); ids outside the table
    contribute zero but still count in the mean's denominator."""
    ids = np.asarray(ids)
    t = np.asarray(table, np.float64)
    out = np.zeros((ids.shape[0], t.shape[1]))
    for r in range(ids.shape[0]):
        for i in ids[r]:
            if 0 <= i < t.shape[0]:
                out[r] += t[i]
        out[r] /= ids.shape[1]
    return out


def gather_score(q: np.ndarray, ids: np.ndarray, table: np.ndarray, dim: int) -> np.ndarray:
    """Per row: q is heads x dim query vectors (flattened), ids its item rows;
    score[h * n_ids + j] = <q_h, table[id_j]> (FP64), zero for ids outside the table."""
    q = np.asarray(q, np.float64)
    t = np.asarray(table, np.float64)
    B = q.shape[0]
    heads = q.shape[1] // dim
    n_ids = ids.shape[1]
    out = np.zeros((B, heads * n_ids))
    for r in range(B):
        for h in range(heads):
            qh = q[r, h * dim:(h + 1) * dim]
            for j, i in enumerate(ids[r]):
                if 0 <= i < t.shape[0]:
                    out[r, h * n_ids + j] = qh @ t[i]
    return out


# ----------------------------------------------------------------- 3x3 convolution + pool


def conv3x3_relu_pool(x_bf16_bits: np.ndarray, w_bf16_bits: np.ndarray) -> np.ndarray:
    """Per row: x is a BF16 feature map [H][W][C] (NHWC), w BF16 [Cout][3][3][C];
    out[co] = mean over pixels (y, x) of max(0, sum_{ky,kx,ci} w[co,ky,kx,ci] *
    x[y+ky-1, x+kx-1, ci]) with zero padding, in FP64."""
    x = bf16_bits_to_f64(x_bf16_bits)
    w = bf16_bits_to_f64(w_bf16_bits)
    B, H, W, C = x.shape
    out = np.zeros((B, w.shape[0]))
    for b in range(B):
        pad = np.zeros((H + 2, W + 2, C))
        pad[1:H + 1, 1:W + 1] = x[b]
        y = np.zeros((H, W, w.shape[0]))
        for ky in range(3):
            for kx in range(3):
                y += pad[ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
        out[b] = np.maximum(y, 0.0).mean(axis=(0, 1))
    return out


# ----------------------------------------------------------------- error metric


def normwise_err(y, ref) -> float:
    """max |y - ref| / max |ref| (the parity metric; robust to ReLU zeros)."""
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(y - ref))) if ref.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


# ------------------------------------------------------------------ artifact stages
# The paper's artifact suite (Section III-B, Section VIII-E) re-created from its
# description: a PCIe-intensive, a compute-intensive and a memory-intensive
# microservice with tunable intensity. The stage definitions (what a row becomes)
# are the library's; here they are written out with plain integer and float32
# NumPy operations, row by row.
def artifact_fold(x_u32: np.ndarray, table_u32: np.ndarray, block_words: int, float_out: bool) -> np.ndarray:
    """ARTIFACT_P (float_out False) / ARTIFACT_M (True). x [rows, D] uint32; the row
    takes block b = x[r, 0] mod (len(table) // block_words) of the table, XORs its
    words j, j + D, j + 2D, ... into word j, XORs that into the row; M then keeps the
    top 24 bits of each word as a float in [0, 1)."""
    x = np.asarray(x_u32, np.uint32)
    rows, D = x.shape
    nblocks = len(table_u32) // block_words
    out = np.empty_like(x)
    for r in range(rows):
        b = int(x[r, 0]) % nblocks
        block = table_u32[b * block_words:(b + 1) * block_words].reshape(block_words // D, D)
        out[r] = x[r] ^ np.bitwise_xor.reduce(block, axis=0)
    if float_out:
        return (out >> np.uint32(8)).astype(np.float32) * np.float32(2.0 ** -24)
    return out


ARTIFACT_C_MUL = np.float32(1.0 - 2.0 ** -11)
ARTIFACT_C_ADD = np.float32(2.0 ** -10)


def artifact_compute(x_u32: np.ndarray, iters: int) -> np.ndarray:
    """ARTIFACT_C: word w -> the float32 with bits (w >> 9) | 0x3F800000, then `iters`
    times x = x * (1 - 2^-11) rounded, + 2^-10 rounded; returns the bits (uint32)."""
    x = ((np.asarray(x_u32, np.uint32) >> np.uint32(9)) | np.uint32(0x3F800000)).view(np.float32)
    for _ in range(iters):
        x = (x * ARTIFACT_C_MUL).astype(np.float32)
        x = (x + ARTIFACT_C_ADD).astype(np.float32)
    return x.view(np.uint32)
