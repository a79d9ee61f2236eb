"""Pins of the oracle's stage math against facts fixed outside the oracle."""
import numpy as np
import pytest

from oracle import stages as O
import workload_gen as G


# ---------------------------------------------------------------- DFT
def test_dft_matches_library_rfft():
    x = G.rng("handoff", 11).standard_normal(400)
    ref = np.fft.rfft(np.concatenate([x, np.zeros(112)]))
    got = O.dft_direct(x)
    assert got.shape == (257,)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def test_dft_parseval():
    x = G.rng("handoff", 12).standard_normal(400)
    X = O.dft_direct(x)
    p = np.abs(X) ** 2
    full = p[0] + p[-1] + 2 * p[1:-1].sum()      # conjugate symmetry of a real input
    assert abs(full - 512 * np.sum(x * x)) < 1e-8 * full


def test_dft_bin_centred_tone():
    k0, A = 37, 0.75
    n = np.arange(512)
    X = O.dft_direct(A * np.cos(2 * np.pi * k0 * n / 512))
    assert abs(abs(X[k0]) - A * 512 / 2) < 1e-9
    others = np.delete(np.abs(X), k0)
    assert np.max(others) < 1e-9


# ---------------------------------------------------------------- mel
def test_mel_scale_roundtrip_and_anchor():
    # HTK: 1000 Hz is ~1000 mel (2595 log10(1 + 1000/700) = 999.985...)
    assert abs(O.hz_to_mel(1000.0) - 999.9855) < 1e-3
    f = np.array([0.0, 123.0, 4000.0, 8000.0])
    assert np.allclose(O.mel_to_hz(O.hz_to_mel(f)), f)


def test_mel_filterbank_partition_of_unity():
    fb = O.mel_filterbank()
    assert fb.shape == (40, 257)
    assert np.all(fb >= 0) and np.all(fb <= 1.0 + 1e-12)
    pts = O.mel_to_hz(np.linspace(0, O.hz_to_mel(8000.0), 42))
    fk = np.arange(257) * 16000 / 512
    inner = (fk >= pts[1]) & (fk <= pts[40])
    s = fb.sum(axis=0)
    assert np.allclose(s[inner], 1.0, atol=1e-12)
    # outside the filterbank's span only the outer slopes contribute (< 1)
    assert np.all(s[~inner] < 1.0)
    # each filter is supported between its neighbours' centres, peaks in order
    peaks = fb.argmax(axis=1)
    assert np.all(np.diff(peaks) >= 0)


# ---------------------------------------------------------------- log-mel
def test_log_mel_impulse_pins_framing_window_and_filters():
    clip = np.zeros((1, 2000))
    clip[0, 170] = 1.0                       # lands in frames 0 (pos 170) and 1 (pos 10)
    feat = O.log_mel(clip).reshape(11, 40)
    fb = O.mel_filterbank()
    w = O.hamming()
    # a windowed impulse has a flat power spectrum w[pos]^2
    for frame, pos in ((0, 170), (1, 10)):
        ref = np.log(np.maximum(w[pos] ** 2 * fb.sum(axis=1), 1e-10))
        assert np.allclose(feat[frame], ref, atol=1e-12)
    assert np.all(feat[2:] == np.log(1e-10))


def test_log_mel_matches_library_fft_path():
    clip = G.c1_audio(2, seed=3)
    got = O.log_mel(clip)
    w = np.hamming(400)                      # library symmetric Hamming window
    fb = O.mel_filterbank()
    ref = np.empty_like(got)
    for b in range(2):
        for f in range(11):
            seg = clip[b, f * 160: f * 160 + 400].astype(np.float64) * w
            p = np.abs(np.fft.rfft(seg, 512)) ** 2
            ref[b, f * 40:(f + 1) * 40] = np.log(np.maximum(fb @ p, 1e-10))
    assert np.max(np.abs(got - ref)) < 1e-9


def test_log_mel_floor():
    feat = O.log_mel(np.zeros((1, 2000)))
    assert np.all(feat == np.log(1e-10))


# ---------------------------------------------------------------- GEMM / argmax / top-k
def test_gemm_relu_identity():
    x = G.c0_queries(4, seed=1)
    y = O.gemm_relu(x, np.eye(512, dtype=np.float32))
    assert np.array_equal(y, np.maximum(x.astype(np.float64), 0))


def test_gemm_relu_hand_case():
    x = np.array([[1.0, -2.0]])
    w = np.array([[3.0, -1.0, 0.5], [1.0, 1.0, 2.0]])
    assert np.array_equal(O.gemm_relu(x, w), [[1.0, 0.0, 0.0]])


def test_argmax_lowest_index_on_ties():
    s = np.array([[1.0, 3.0, 3.0, -1.0], [0.0, 0.0, 0.0, 0.0], [-5.0, -4.0, -4.5, -4.0]])
    assert list(O.argmax_lowest(s)) == [1, 0, 1]


def test_topk_against_stable_sort():
    g = G.rng("handoff", 5)
    s = np.round(g.standard_normal((6, 300)), 1)      # many exact ties
    idx, val = O.topk(s, 25)
    for r in range(6):
        ref = np.argsort(-s[r], kind="stable")[:25]
        assert list(idx[r]) == list(ref)
        assert np.array_equal(val[r], s[r, ref])


# ---------------------------------------------------------------- BF16
def _bf16_from_f32_bits(x32):
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_round_matches_bit_rounding_on_fp32_inputs():
    x = G.rng("handoff", 7).standard_normal(20000).astype(np.float32) * 3
    assert np.array_equal(O.bf16_round(x.astype(np.float64)), _bf16_from_f32_bits(x))


def test_bf16_round_halfway_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: rounds to the even significand (1)
    assert O.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert O.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    for v in (1.0, -2.5, 0.0078125, 3.0 * 2 ** 20):
        assert O.bf16_round(np.array([v]))[0] == v


def test_mlp_bf16_identity_chain():
    eye = G._to_bf16_bits(np.eye(8, dtype=np.float32))
    x = G.rng("handoff", 8).standard_normal((3, 8))
    y = O.mlp_bf16(x, [eye, eye])
    assert np.array_equal(y, O.bf16_round(np.maximum(O.bf16_round(x), 0)))


def test_normwise_err():
    assert O.normwise_err([1.0, 0.0], [1.0, 0.0]) == 0.0
    assert O.normwise_err([1.0, 0.5], [2.0, 0.0]) == 0.5


# ---------------------------------------------------------------- gather
def test_gather_mean_hand_case_and_out_of_range():
    t = np.array([[1.0, 2.0], [10.0, 20.0], [100.0, 200.0]])
    got = O.gather_mean(np.array([[0, 2, 2, 99], [1, 1, -1, 0]]), t)
    assert np.array_equal(got, [[(1 + 200) / 4, (2 + 400) / 4], [(20 + 1) / 4, (40 + 2) / 4]])


def test_gather_mean_matches_fancy_indexing():
    t = G.fp16_table(1000, 64, seed=2)
    ids = G.zipf_ids(7, 32, 1000, seed=2)
    ref = t.astype(np.float64)[ids].mean(axis=1)
    assert np.allclose(O.gather_mean(ids, t), ref, rtol=0, atol=1e-12)


def test_zipf_ids_are_skewed_and_in_range():
    ids = G.zipf_ids(2000, 32, 10000, seed=1)
    assert ids.min() >= 0 and ids.max() < 10000
    _, counts = np.unique(ids, return_counts=True)
    top = np.sort(counts)[::-1]
    assert top[0] > 20 * np.median(counts)     # a heavy head


# ---------------------------------------------------------------- conv / score
def test_conv_centre_delta_is_relu_mean_of_channel():
    x = G.c4_feature_maps(2, seed=3, h=5, w=7)
    w = np.zeros((64, 3, 3, 64), np.float32)
    for co in range(64):
        w[co, 1, 1, co] = 1.0                       # centre tap: identity
    got = O.conv3x3_relu_pool(x, G._to_bf16_bits(w))
    xf = O.bf16_bits_to_f64(x)
    assert np.allclose(got, np.maximum(xf, 0).mean(axis=(1, 2)), atol=1e-12)


def test_conv_matches_direct_sum_and_pads_with_zero():
    x = G.c4_feature_maps(1, seed=4, h=4, w=3)
    w = G.c4_conv_weights(seed=4)
    xf, wf = O.bf16_bits_to_f64(x)[0], O.bf16_bits_to_f64(w)
    H, W = 4, 3
    ref = np.zeros(64)
    for y in range(H):
        for xx in range(W):
            for co in range(64):
                acc = 0.0
                for ky in range(3):
                    for kx in range(3):
                        yy, xs = y + ky - 1, xx + kx - 1
                        if 0 <= yy < H and 0 <= xs < W:
                            acc += float(wf[co, ky, kx] @ xf[yy, xs])
                ref[co] += max(acc, 0.0)
    assert np.allclose(O.conv3x3_relu_pool(x, w)[0], ref / (H * W), rtol=1e-12, atol=1e-12)


def test_gather_score_hand_case():
    t = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    q = np.array([[1.0, 1.0, 2.0, -1.0]])           # two heads of dim 2
    got = O.gather_score(q, np.array([[0, 2, 7]]), t, 2)
    assert np.array_equal(got, [[1.0, 2.0, 0.0, 2.0, 1.0, 0.0]])


# ------------------------------------------------------------------ artifact stages
def test_artifact_fold_by_hand():
    D = 4
    table = np.arange(48, dtype=np.uint32)               # 3 blocks of 16 words
    x = np.array([[7, 0, 0, 0], [3, 1, 2, 3], [2, 0, 0, 0xFFFFFFFF]], np.uint32)
    got = O.artifact_fold(x, table, 16, False)
    # block index = x[r, 0] mod 3; fold word j = XOR of block words j, j+4, j+8, j+12
    for r in range(3):
        b = int(x[r, 0]) % 3
        blk = [int(v) for v in table[16 * b:16 * b + 16]]
        for j in range(D):
            f = blk[j] ^ blk[j + 4] ^ blk[j + 8] ^ blk[j + 12]
            assert int(got[r, j]) == (int(x[r, j]) ^ f)
    # a zero table leaves the row; a table of one repeated slice folds to that slice
    # (an even number of copies cancels)
    assert np.array_equal(O.artifact_fold(x, np.zeros(48, np.uint32), 16, False), x)
    rep = np.tile(np.array([5, 6, 7, 8], np.uint32), 8)            # blocks of 2 slices
    assert np.array_equal(O.artifact_fold(x, rep, 8, False), x)
    rep3 = np.tile(np.array([5, 6, 7, 8], np.uint32), 9)           # blocks of 3 slices
    assert np.array_equal(O.artifact_fold(x, rep3, 12, False), x ^ np.array([5, 6, 7, 8], np.uint32))


def test_artifact_memory_output_is_the_top_24_bits():
    x = np.array([[0, 0xFFFFFFFF, 0x00000100, 0x80000000]], np.uint32)
    got = O.artifact_fold(x, np.zeros(4, np.uint32), 4, True)
    assert got.dtype == np.float32
    assert list(got[0]) == [0.0, (2 ** 24 - 1) / 2 ** 24, 2.0 ** -24, 0.5]


def test_artifact_compute_steps():
    # zero iterations: the word's top 23 bits as the mantissa of a float in [1, 2)
    w = np.array([0, 0xFFFFFFFF, 1 << 31, 511], np.uint32)
    x0 = O.artifact_compute(w, 0).view(np.float32)
    assert list(x0) == [1.0, 2.0 - 2.0 ** -23, 1.5, 1.0]
    # one iteration from 1: 1 - 2^-11 + 2^-10 = 1 + 2^-11, exact in FP32
    assert int(O.artifact_compute(np.array([0], np.uint32), 1)[0]) == 0x3F801000
    # two roundings, not one fused operation: for this word (one of 1,022 of the 2^23
    # mantissas where the two differ) a single rounding of x a + b gives another float
    w = np.array([0x40200], np.uint32)
    x = ((w >> np.uint32(9)) | np.uint32(0x3F800000)).view(np.float32)[0]
    two = np.float32(np.float32(x * O.ARTIFACT_C_MUL) + O.ARTIFACT_C_ADD)
    fused = np.float32(np.float64(x) * np.float64(O.ARTIFACT_C_MUL) + np.float64(O.ARTIFACT_C_ADD))
    step = O.artifact_compute(w, 1).view(np.float32)[0]
    assert step == two and step != fused
    # the iteration contracts towards its fixed point 2 (= 2^-10 / 2^-11); in FP32 it
    # settles below, at 2 - 2^-13 (bits 0x3FFFFC00), where a step no longer moves it
    far = O.artifact_compute(np.array([0, 1 << 31], np.uint32), 40000)
    assert list(far) == [0x3FFFFC00, 0x3FFFFC00]
    assert list(O.artifact_compute(np.array([0], np.uint32), 40001)) == [0x3FFFFC00]
