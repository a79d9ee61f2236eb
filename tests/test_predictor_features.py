"""Host logic of the learned predictor: feature layout and standardisation."""
import numpy as np
import pytest

from paper_2005_02088_amd import camelot as cm

BATCHES = [1, 2, 4, 8, 16, 32, 64, 128]


def _tables():
    k, s, b = np.meshgrid(np.arange(3), np.arange(32), np.arange(8), indexing="ij")
    hbm = (k + s / 100.0 + b / 1000.0).astype(np.float32)
    mfma = (10 + k + s / 100.0 + b / 1000.0).astype(np.float32)
    return cm.SoloTablesArrays(8, BATCHES, hbm, mfma)


def test_feature_layout_three_stages():
    t = _tables()
    f = cm.camelot_predictor_features(t, [2, 0, 1], [16, 64, 8], [1, 3, 7])
    # row 0: kind 2, 16 CUs (share index 1), batch 2 (index 1)
    np.testing.assert_allclose(f[0, :4], [16 / 256, 1 / 7, 2 + 0.01 + 0.001, 12 + 0.01 + 0.001], rtol=1e-6)
    assert list(f[0, 4:7]) == [0, 0, 1]
    # no other instance of kind 2: the sibling slot is empty
    assert np.all(f[0, 7:11] == 0)
    # the kernels of other kinds, aggregated: kind 0 (64 CUs, batch 8) and kind 1
    # (8 CUs, batch 128): summed shares, mean log2 batch, summed solo rates
    np.testing.assert_allclose(f[0, 11:15], [(64 + 8) / 256, (3 / 7 + 7 / 7) / 2,
                                             (0 + 0.07 + 0.003) + (1 + 0.0 + 0.007),
                                             (10 + 0.07 + 0.003) + (11 + 0.0 + 0.007)], rtol=1e-6)
    np.testing.assert_allclose(f[:, 15], (16 + 64 + 8) / 256)
    # row 1 (kind 0) sees kinds 2 and 1 in the other-kinds slot
    assert list(f[1, 4:7]) == [1, 0, 0]
    np.testing.assert_allclose(f[1, 11], (16 + 8) / 256)


def test_feature_layout_instances():
    """Several instances of one kind: each sees its siblings in the sibling slot."""
    t = _tables()
    kinds, cu, bi = [1, 1, 2, 1], [64, 64, 16, 32], [7, 7, 7, 5]
    f = cm.camelot_predictor_features(t, kinds, cu, bi)
    hbm = lambda k, c, b: k + (c // 8 - 1) / 100.0 + b / 1000.0
    # row 0 (kind 1, 64 CUs): siblings rows 1 and 3, the other kind row 2
    np.testing.assert_allclose(f[0, 7:11], [(64 + 32) / 256, (7 / 7 + 5 / 7) / 2, hbm(1, 64, 7) + hbm(1, 32, 5),
                                            10 + hbm(1, 64, 7) + 10 + hbm(1, 32, 5)], rtol=1e-6)
    np.testing.assert_allclose(f[0, 11:15], [16 / 256, 7 / 7, hbm(2, 16, 7), 10 + hbm(2, 16, 7)], rtol=1e-6)
    # row 2 (kind 2): no siblings, three kind-1 kernels in the other slot
    assert np.all(f[2, 7:11] == 0)
    np.testing.assert_allclose(f[2, 11], (64 + 64 + 32) / 256)
    np.testing.assert_allclose(f[2, 12], (7 / 7 + 7 / 7 + 5 / 7) / 3, rtol=1e-6)
    np.testing.assert_allclose(f[:, 15], (64 + 64 + 16 + 32) / 256)
    # rows 0 and 1 are alike (identical instances)
    np.testing.assert_array_equal(f[0], f[1])


def test_feature_layout_solo_has_empty_corunner_slots():
    t = _tables()
    f = cm.camelot_predictor_features(t, [1], [256], [0])
    assert np.all(f[0, 7:15] == 0)
    np.testing.assert_allclose(f[0, 15], 1.0)
    np.testing.assert_allclose(f[0, 0], 1.0)


def test_feature_validation():
    t = _tables()
    for kinds, cu, bi in (([3], [8], [0]), ([0], [12], [0]), ([0], [264], [0]), ([0], [8], [8]),
                          ([0] * 9, [8] * 9, [0] * 9)):
        with pytest.raises(cm.CamelotError):
            cm.camelot_predictor_features(t, kinds, cu, bi)


def test_standardisation_matches_numpy():
    x = np.random.default_rng(3).normal(5, 2, (500, 16)).astype(np.float32)
    x[:, 4] = 1.0                               # a constant column: std floored, not zero
    mean, std = cm.camelot_predictor_fit_norm(x)
    np.testing.assert_allclose(mean, x.mean(axis=0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(std[np.arange(16) != 4], x.std(axis=0)[np.arange(16) != 4], rtol=1e-4)
    assert std[4] >= 1e-6
    z = cm.camelot_predictor_standardize(x, mean, std)
    np.testing.assert_allclose(z, (x - mean) / std, rtol=1e-5, atol=1e-5)
